"""Molecular dynamics and relaxation with on-the-fly extrapolation control
(paper, section 2.3).

Velocity Verlet (NVE) on one batch, every step on the device: mtp_md_kick
(half kick and drift), mtp_eval at the new positions (with a Verlet skin
the neighbour lists are reused), mtp_md_kick (half kick).  When the
potential has an active set, the extrapolation grade gamma of every
configuration is computed each step from the descriptors (mtp_grade_from_b)
and the two thresholds of the paper's active learning apply: a
configuration with gamma above `gamma_select` is recorded as a candidate
for training, and the run stops as soon as some gamma exceeds `gamma_break`.

Relaxation (`relax`) runs FIRE steps (mtp_fire_step, every configuration
with its own step size) between evaluations, with the same thresholds.
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


def kinetic_energy(P: Potential, batch: Batch, vel, masses, stream=None):
    """Kinetic energy [K] (eV) of every configuration (mtp_kinetic_energy)."""
    m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
    if m.size != P.n_species:
        raise ValueError("one mass per species")
    out = torch.empty(batch.n_configs, dtype=torch.float64, device=vel.device)
    check(lib().mtp_kinetic_energy(P._h, batch.n_configs, batch.atom_offsets.data_ptr(), batch.n_atoms,
                                   batch.species.data_ptr(), vel.data_ptr(), m.ctypes.data_as(ctypes.c_void_p),
                                   out.data_ptr(), _stream(stream)),
          "mtp_kinetic_energy")
    return out


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
    ekin = lambda: kinetic_energy(P, batch, vel, masses)
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


# FIRE parameters of Bitzek et al. (2006): dt_max (fs), n_min, f_inc, f_dec, alpha_start, f_alpha
FIRE_DEFAULTS = {"dt_max": 5.0, "n_min": 5, "f_inc": 1.1, "f_dec": 0.5, "alpha_start": 0.1, "f_alpha": 0.99}


def fire_state(batch: Batch, dt0=0.5, alpha_start=0.1):
    """Initial FIRE state [K, 4] on the device: (dt0, alpha_start, 0, 0)."""
    st = torch.zeros((batch.n_configs, 4), dtype=torch.float64, device=batch.pos.device)
    st[:, 0] = dt0
    st[:, 1] = alpha_start
    return st


def fire_step(P: Potential, batch: Batch, vel, forces, masses, state, params=None, stream=None):
    """One FIRE step of every configuration (mtp_fire_step): vel and the
    batch positions are updated in place, state [K, 4] too."""
    p = dict(FIRE_DEFAULTS, **(params or {}))
    m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
    if m.size != P.n_species:
        raise ValueError("one mass per species")
    pr = np.array([p["dt_max"], p["n_min"], p["f_inc"], p["f_dec"], p["alpha_start"], p["f_alpha"]], np.float64)
    check(lib().mtp_fire_step(P._h, batch.n_configs, batch.atom_offsets.data_ptr(), batch.n_atoms,
                              batch.species.data_ptr(), batch.pos.data_ptr(), vel.data_ptr(), forces.data_ptr(),
                              m.ctypes.data_as(ctypes.c_void_p), state.data_ptr(),
                              pr.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
          "mtp_fire_step")


def relax(P: Potential, batch: Batch, masses, fmax=0.01, max_steps=500, dt0=0.5, params=None, check_every=10,
          precision="fp64", skin=0.0, gamma_select=None, gamma_break=None):
    """FIRE relaxation of every configuration of `batch` (positions updated
    in place) until the largest force of each is below `fmax` (eV/A, checked
    every `check_every` steps) or `max_steps`.  Returns {"energy": [checks, K],
    "fmax": [checks, K], "converged": bool [K], "steps", and, when an active
    set is present and thresholds are given, "gamma", "selected" and
    "stopped_at" as run() does}."""
    p = dict(FIRE_DEFAULTS, **(params or {}))
    P.set_skin(skin)
    grade = gamma_select is not None or gamma_break is not None
    vel = torch.zeros((batch.n_atoms, 3), dtype=torch.float64, device=batch.pos.device)
    state = fire_state(batch, dt0, p["alpha_start"])
    offs = batch.atom_offsets.cpu().numpy()
    energies, fmaxes, gammas, selected, stopped = [], [], [], [], None
    converged = np.zeros(batch.n_configs, bool)
    step = 0
    while True:
        out = P.eval(batch, precision=precision, forces=True, virial=False, b=grade)
        if grade:
            g, _ = P.grade_from_b(out["b"])
            gh = g.cpu().numpy()
            gammas.append(gh)
            if gamma_select is not None:
                selected.extend((step, int(k)) for k in np.nonzero(gh > gamma_select)[0])
            if gamma_break is not None and (gh > gamma_break).any():
                stopped = step
        if step % check_every == 0 or step == max_steps or stopped is not None:
            f = np.linalg.norm(out["forces"].cpu().numpy(), axis=1)
            fm = np.array([f[offs[k]:offs[k + 1]].max() if offs[k + 1] > offs[k] else 0.0
                           for k in range(batch.n_configs)])
            energies.append(out["energy"].cpu().numpy())
            fmaxes.append(fm)
            converged = fm < fmax
            if converged.all():
                break
        if step == max_steps or stopped is not None:
            break
        fire_step(P, batch, vel, out["forces"], masses, state, p)
        step += 1
    res = {"energy": np.array(energies), "fmax": np.array(fmaxes), "converged": converged, "steps": step}
    if grade:
        res.update(gamma=np.array(gammas), selected=selected, stopped_at=stopped)
    return res
