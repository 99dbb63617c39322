"""Molecular dynamics driver (paper_2007_08555_amd.md; the MD of the paper's
active learning, section 2.3): velocity Verlet on the device with the
library's forces.  Parity: ten steps of the 108-atom fcc box at level 8
against the same integrator written out in numpy on the oracle's forces;
total energy conserved over 300 steps; the two extrapolation thresholds."""
import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu

MASS_AL = 26.9815        # amu
EV_PER_AMU_A2_FS2 = 103.642696562


def initial_velocities(n, mass, T=300.0, seed=0):
    kT = 8.617333262e-5 * T
    v = np.random.default_rng(seed).normal(0.0, np.sqrt(kT / (mass * EV_PER_AMU_A2_FS2)), size=(n, 3))
    return v - v.mean(axis=0)


def test_velocity_verlet_matches_oracle_integration():
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    box = synth.fcc108(seed=3)
    N = int(box["n_atoms"][0])
    v0 = initial_velocities(N, MASS_AL, seed=1)
    dt, steps = 1.0, 10
    # the oracle's trajectory: x += dt v + dt^2 a / 2 as kick / drift / kick
    pot = read_potential(pot_path("lev8_s1"))
    pos, sp, cell, pbc = synth.config_of(box, 0)
    x, v = pos.copy(), v0.copy()
    F = omtp.evaluate(pot, x, sp, cell, pbc)["forces"]
    for _ in range(steps):
        v = v + 0.5 * dt * F / (MASS_AL * EV_PER_AMU_A2_FS2)
        x = x + dt * v
        F = omtp.evaluate(pot, x, sp, cell, pbc)["forces"]
        v = v + 0.5 * dt * F / (MASS_AL * EV_PER_AMU_A2_FS2)
    P = Potential(pot_path("lev8_s1"))
    B = Batch.from_arrays(box, "cuda:0")
    vel = torch.as_tensor(v0, device="cuda:0").contiguous()
    md.run(P, B, vel, [MASS_AL], dt=dt, n_steps=steps)
    dx = np.abs(B.pos.cpu().numpy() - x).max()
    dv = np.abs(vel.cpu().numpy() - v).max()
    log(f"[md driver] after {steps} steps: position difference {dx:.3e} A, velocity difference {dv:.3e} A/fs")
    assert dx <= 1e-10 and dv <= 1e-12


def test_total_energy_is_conserved():
    # The test potentials are fitted to synthetic data, not physically stable
    # (forces near 13 eV/A on the displaced box; long runs reach r < R_min),
    # so conservation is checked over 5 fs: 100 steps of 0.05 fs, in which
    # the velocity-Verlet error (of order dt^2) keeps the total energy within
    # 1e-3 of the potential energy's change.
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    box = synth.fcc108(seed=4)
    N = int(box["n_atoms"][0])
    P = Potential(pot_path("lev8_s1"))
    B = Batch.from_arrays(box, "cuda:0")
    vel = torch.as_tensor(initial_velocities(N, MASS_AL, seed=2), device="cuda:0").contiguous()
    res = md.run(P, B, vel, [MASS_AL], dt=0.05, n_steps=100)
    epot = res["energy"][:, 0]
    etot = epot + res["kinetic"][:, 0]
    drift = np.abs(etot - etot[0]).max()
    swing = np.abs(epot - epot[0]).max()
    log(f"[md driver] 100 steps of 0.05 fs: largest total-energy change {drift / N:.3e} eV/atom, "
        f"largest potential-energy change {swing / N:.3e} eV/atom")
    assert drift <= 1e-3 * swing


def test_extrapolation_thresholds():
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    batch = synth.mixed_batch(seed=71, n_configs=6, n_min=16, n_max=48, n_species_model=3)
    P = Potential(pot_path("lev16_s3"))
    P.set_active_set(np.load(pot_path("lev16_s3").replace("potentials/lev16_s3.mtp", "active_lev16_s3.npz"))["A"])
    B = Batch.from_arrays(batch, "cuda:0")
    g0 = P.grade_from_b(P.eval(B, precision="fp64", b=True)["b"])[0].cpu().numpy()
    vel = torch.zeros((B.n_atoms, 3), dtype=torch.float64, device="cuda:0")
    masses = [26.98, 58.69, 63.55]
    # every configuration above the selection threshold at step 0; none above the break threshold
    res = md.run(P, B, vel, masses, dt=0.5, n_steps=3, gamma_select=0.5 * g0.min(), gamma_break=10 * g0.max())
    assert res["stopped_at"] is None and {k for s, k in res["selected"] if s == 0} == set(range(6))
    assert np.allclose(res["gamma"][0], g0, rtol=1e-12)
    # a break threshold below the largest grade stops the run before the first step
    B2 = Batch.from_arrays(batch, "cuda:0")
    res = md.run(P, B2, torch.zeros_like(vel), masses, dt=0.5, n_steps=3, gamma_break=0.5 * g0.max())
    log(f"[md driver] gamma at step 0 {np.round(g0, 3).tolist()}; stopped at {res['stopped_at']}")
    assert res["stopped_at"] == 0 and res["energy"].shape[0] == 1
