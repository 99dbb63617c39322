"""GPU parity of the FIRE relaxation step (mtp_fire_step) and the relaxation
driver against the oracle's FIRE step, and convergence on a quadratic bowl."""
import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import mtp as omtp
from oracle import relax as orx
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu

PRM = dict(dt_max=2.0, n_min=1, f_inc=1.1, f_dec=0.5, alpha_start=0.1, f_alpha=0.99)


def _batch_arrays(sizes, seed):
    rng = np.random.default_rng(seed)
    cfgs = []
    for n in sizes:
        pos = rng.uniform(0, 10, (n, 3))
        cfgs.append((pos, rng.integers(0, 2, n).astype(np.int32), np.eye(3) * 10.0, 1))
    return synth._batch(cfgs)


def test_fire_step_matches_the_oracle():
    """Eight steps on seeded velocities and forces (both signs of P, the step
    growing after n_min), configurations of 5 and 300 atoms (more atoms than
    threads), against the oracle step per configuration."""
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    P = Potential(pot_path("lev12_s2"))
    b = _batch_arrays([5, 300, 0, 17], seed=3)
    B = Batch.from_arrays(b)
    rng = np.random.default_rng(4)
    masses = np.array([26.98, 58.69])
    vel = rng.normal(0, 0.01, (b["n_atoms"].sum(), 3))
    state = md.fire_state(B, dt0=0.5, alpha_start=PRM["alpha_start"])
    vel_d = torch.as_tensor(vel, device="cuda").contiguous()
    pos_o, vel_o = b["pos"].copy(), vel.copy()
    st_o = [(0.5, PRM["alpha_start"], 0)] * len(b["n_atoms"])
    off = b["atom_offsets"]
    m_atom = masses[b["species"]]
    for step in range(8):
        F = rng.normal(0, 1.0, pos_o.shape) + (0.5 if step % 3 else -0.5) * vel_o * 100
        md.fire_step(P, B, vel_d, torch.as_tensor(F, device="cuda").contiguous(), masses, state, PRM)
        for k in range(len(b["n_atoms"])):
            s = slice(off[k], off[k + 1])
            pos_o[s], vel_o[s], st_o[k] = orx.fire_step(pos_o[s], vel_o[s], F[s], m_atom[s], st_o[k], **PRM)
        torch.cuda.synchronize()
        np.testing.assert_allclose(B.pos.cpu().numpy(), pos_o, rtol=0, atol=1e-12)
        np.testing.assert_allclose(vel_d.cpu().numpy(), vel_o, rtol=0, atol=1e-13)
        np.testing.assert_allclose(state.cpu().numpy()[:, :3], np.array(st_o), rtol=1e-14)
    log(f"[fire] states after 8 steps {np.array(st_o)}")


def test_fire_converges_on_a_quadratic_bowl():
    """F = -k (x - x0): every configuration relaxes to its own x0 with its
    own step size."""
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    P = Potential(pot_path("lev12_s2"))
    b = _batch_arrays([3, 40, 260], seed=5)
    B = Batch.from_arrays(b)
    rng = np.random.default_rng(6)
    x0 = torch.as_tensor(b["pos"] + rng.normal(0, 0.3, b["pos"].shape), device="cuda")
    kk = torch.as_tensor(np.repeat([1.0, 5.0, 20.0], b["n_atoms"])[:, None], device="cuda")
    vel = torch.zeros_like(x0)
    state = md.fire_state(B, dt0=0.5)
    for step in range(3000):
        F = (-kk * (B.pos - x0)).contiguous()
        if float(F.abs().max()) < 1e-8:
            break
        md.fire_step(P, B, vel, F, np.array([26.98, 58.69]), state, PRM)
    err = float((B.pos - x0).abs().max())
    log(f"[fire bowl] steps {step}, max |x - x0| {err:.2e}, dt per configuration {state[:, 0].cpu().numpy()}")
    assert err < 1e-8


def test_relax_driver_follows_the_oracle():
    """md.relax for four steps from a perturbed fcc box equals the oracle's
    FIRE steps on the oracle's forces."""
    from paper_2007_08555_amd import Batch, Potential, md
    P = Potential(pot_path("lev8_s1"))
    pot = read_potential(pot_path("lev8_s1"))
    b = synth.fcc108(seed=2)
    B = Batch.from_arrays(b)
    masses = np.array([26.98])
    res = md.relax(P, B, masses, fmax=1e-12, max_steps=4, dt0=0.5, params=PRM, check_every=1)
    pos, sp, cell, pbc = synth.config_of(b, 0)
    x, v, st = pos.copy(), np.zeros_like(pos), (0.5, PRM["alpha_start"], 0)
    E = []
    for step in range(4):
        r = omtp.evaluate(pot, x, sp, cell, pbc)
        E.append(r["energy"])
        x, v, st = orx.fire_step(x, v, r["forces"], np.full(len(x), 26.98), st, **PRM)
    log(f"[relax] energies gpu {res['energy'][:4, 0]} oracle {E}")
    assert res["steps"] == 4
    np.testing.assert_allclose(res["energy"][:4, 0], E, rtol=1e-12)
    np.testing.assert_allclose(B.pos.cpu().numpy(), x, rtol=0, atol=1e-10)


def test_kinetic_energy_per_configuration():
    """mtp_kinetic_energy against sum m |v|^2 / 2 in eV per configuration
    (1 amu A^2/fs^2 = 103.642696562 eV), empty configurations included."""
    import torch
    from paper_2007_08555_amd import Batch, Potential, md
    P = Potential(pot_path("lev12_s2"))
    b = _batch_arrays([7, 0, 300, 1], seed=9)
    B = Batch.from_arrays(b)
    v = np.random.default_rng(10).normal(0, 0.02, (b["n_atoms"].sum(), 3))
    masses = np.array([26.98, 58.69])
    e = md.kinetic_energy(P, B, torch.as_tensor(v, device="cuda").contiguous(), masses).cpu().numpy()
    off = b["atom_offsets"]
    m = masses[b["species"]]
    ref = np.array([0.5 * np.sum(m[off[k]:off[k + 1], None] * v[off[k]:off[k + 1]] ** 2) / orx.EV_PER_A_AMU_IN_A_PER_FS2
                    for k in range(len(b["n_atoms"]))])
    np.testing.assert_allclose(e, ref, rtol=1e-13)
    assert e[1] == 0.0
