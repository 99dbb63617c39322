"""Molecular dynamics with on-the-fly extrapolation control (paper, section 2.3).

Velocity Verlet (NVE) on one batch, every step on the device: mtp_md_kick
(half kick and drift), mtp_eval at the new positions (with a Verlet skin
the neighbour lists are reused), mtp_md_kick (half kick).  When the
potential has an active set, the extrapolation grade gamma of every
configuration is computed each step from the descriptors (mtp_grade_from_b)
and the two thresholds of the paper's active learning apply: a
configuration with gamma above `gamma_select` is recorded as a candidate
for training, and the run stops as soon as some gamma exceeds `gamma_break`.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib
from .model import Batch, Potential, _stream


def kick(P: Potential, batch: Batch, vel, forces, masses, dt, drift, stream=None):
    """vel += (dt/2) F/m and, with drift, pos += dt vel (mtp_md_kick)."""
    m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
    if m.size != P.n_species:
        raise ValueError("one mass per species")
    check(lib().mtp_md_kick(P._h, batch.n_atoms, batch.species.data_ptr(), batch.pos.data_ptr(), vel.data_ptr(),
                            forces.data_ptr(), m.ctypes.data_as(ctypes.c_void_p), float(dt), 1 if drift else 0,
                            _stream(stream)),
          "mtp_md_kick")


def run(P: Potential, batch: Batch, vel, masses, dt=1.0, n_steps=100, precision="fp64", skin=0.3,
        gamma_select=None, gamma_break=None):
    """n_steps of velocity Verlet on `batch` (positions updated in place) with
    velocities `vel` [N,3] (A/fs, device FP64, updated in place).  Returns
    {"energy": potential energy per step [steps+1, K], "kinetic": kinetic
    energy per step [steps+1, K] (eV), "gamma": per step [steps+1, K] or None,
    "selected": [(step, configuration)] with gamma > gamma_select,
    "stopped_at": the step at which gamma exceeded gamma_break, or None}."""
    P.set_skin(skin)
    grade = gamma_select is not None or gamma_break is not None
    mass_atom = torch.as_tensor(np.asarray(masses, dtype=np.float64), device=vel.device)[batch.species.long()]
    cfg_of_atom = torch.repeat_interleave(torch.arange(batch.n_configs, device=vel.device),
                                          batch.atom_offsets.diff())
    # 1/2 m v^2 in eV: amu A^2 / fs^2 = 103.6427 eV
    ekin = lambda: torch.zeros(batch.n_configs, dtype=torch.float64, device=vel.device).index_add_(
        0, cfg_of_atom, 0.5 * 103.642696562 * mass_atom * (vel * vel).sum(dim=1))
    energies, kinetic, gammas, selected, stopped = [], [], [], [], None

    def evaluate(step):
        nonlocal stopped
        out = P.eval(batch, precision=precision, forces=True, virial=False, b=grade)
        energies.append(out["energy"].clone())
        kinetic.append(ekin())
        if grade:
            g, _ = P.grade_from_b(out["b"])
            gammas.append(g.clone())
            gh = g.cpu().numpy()
            if gamma_select is not None:
                selected.extend((step, int(k)) for k in np.nonzero(gh > gamma_select)[0])
            if gamma_break is not None and (gh > gamma_break).any():
                stopped = step
        return out["forces"]

    F = evaluate(0)
    for step in range(1, n_steps + 1):
        if stopped is not None:
            break
        kick(P, batch, vel, F, masses, dt, drift=True)
        F = evaluate(step)
        kick(P, batch, vel, F, masses, dt, drift=False)
        kinetic[-1] = ekin()    # the kinetic energy after the second half kick
    return {"energy": torch.stack(energies).cpu().numpy(), "kinetic": torch.stack(kinetic).cpu().numpy(),
            "gamma": torch.stack(gammas).cpu().numpy() if grade else None, "selected": selected,
            "stopped_at": stopped}
