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


def _morse_pair_potential(path):
    """A level-2 potential, V_i = sum_j f_0(r_ij), whose radial function is
    the least-squares fit (numpy, on the Chebyshev radial basis) of half a
    Morse pair potential D[(1 - exp(-a(r - r0)))^2 - 1] with D = 0.3 eV,
    a = 1.5 / A, r0 = 2.55 A: a pair potential with a minimum at the
    nearest-neighbour distance of fcc with lattice constant 3.6 A."""
    from oracle import basis as obasis
    from oracle import mtp as omtp
    from oracle.potential import write_potential
    level, n_q, r_min, r_cut = 2, 8, 2.0, 5.0
    r = np.linspace(1.8, r_cut, 400)
    Q, _ = omtp.radial_basis(r, r_min, r_cut, n_q)
    target = 0.5 * 0.3 * ((1 - np.exp(-1.5 * (r - 2.55))) ** 2 - 1)
    c = np.linalg.lstsq(Q, target, rcond=None)[0]
    pot = dict(level=level, n_species=1, n_q=n_q, r_min=r_min, r_cut=r_cut, moments=obasis.moments_used(level),
               graphs=list(obasis.connected_contractions(level)), basis=list(obasis.basis(level)),
               c=c.reshape(1, 1, 1, n_q), xi=np.ones(1))
    write_potential(path, pot)
    return pot


def test_fire_relaxes_a_perturbed_crystal_on_a_pair_potential(tmp_path):
    """FIRE (md.relax) on a potential with a minimum: a 108-atom fcc box
    (a = 3.6 A) with every coordinate perturbed by N(0, 0.08^2) A relaxes
    until the largest force is below 1e-4 eV/A; the oracle confirms the
    forces at the final positions, and the box returns to the perfect
    lattice (up to a common translation) and its energy."""
    import torch
    from oracle import mtp as omtp
    from paper_2007_08555_amd import Batch, Potential, md
    path = str(tmp_path / "morse_lev2.mtp")
    pot = _morse_pair_potential(path)
    a = 3.6
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    ideal = np.array([(np.array([i, j, k]) + b) * a for i in range(3) for j in range(3) for k in range(3)
                      for b in base])
    cell = np.eye(3) * 3 * a
    rng = np.random.default_rng(17)
    start = ideal + rng.normal(0, 0.08, ideal.shape)
    batch = synth._batch([(start, np.zeros(len(ideal), np.int32), cell, 1)])
    P = Potential(path)
    B = Batch.from_arrays(batch)
    res = md.relax(P, B, masses=np.array([63.5]), fmax=1e-4, max_steps=4000)
    final = B.pos.cpu().numpy()
    log(f"[relax morse] steps {res['steps']}, converged {bool(res['converged'][0])}, "
        f"fmax {res['fmax'][-1][0]:.2e}, energy {res['energy'][0][0]:.6f} -> {res['energy'][-1][0]:.6f} eV")
    assert res["converged"][0]
    f_o = omtp.evaluate(pot, final, np.zeros(len(ideal), np.int32), cell, 1)["forces"]
    assert np.abs(f_o).max() <= 2e-4
    # back on the lattice: displacement from the ideal sites is one common
    # translation (minimum image per atom)
    d = final - ideal
    d -= np.round(d / (3 * a)) * (3 * a)
    shift = d.mean(axis=0)
    dev = np.abs(d - shift).max()
    e_ideal = omtp.evaluate(pot, ideal + shift, np.zeros(len(ideal), np.int32), cell, 1)["energy"]
    log(f"[relax morse] largest deviation from the shifted lattice {dev:.2e} A; energy {res['energy'][-1][0]:.8f}, "
        f"perfect lattice {e_ideal:.8f} eV")
    assert dev <= 1e-3
    assert abs(res["energy"][-1][0] - e_ideal) <= 1e-6 * len(ideal)
