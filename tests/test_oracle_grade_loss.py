"""Pins of the oracle's grade, MaxVol, loss and loss gradient against the
paper (sections 2.2 and 2.3) and the mathematics."""
import itertools

import numpy as np
import pytest

import synth
from oracle import grade as og
from oracle import loss as ol
from oracle import mtp

from test_oracle_mtp import make_pot


def pool_rows(pot, n_cfg=40, seed=0):
    b = synth.mixed_batch(seed=seed, n_configs=n_cfg, n_min=8, n_max=24,
                          n_species_model=pot["n_species"])
    rows, energies = [], []
    for k in range(n_cfg):
        r = mtp.evaluate(pot, *synth.config_of(b, k))
        rows.append(r["b"])
        energies.append(r["energy"])
    return np.array(rows), np.array(energies), b


def test_grade_of_active_rows_is_one():
    pot = make_pot(level=8, S=1)
    B, _, _ = pool_rows(pot)
    rows, _ = og.maxvol(B)
    A = B[rows]
    gam, arg, c = og.grade(A, A)
    assert np.allclose(gam, 1.0, atol=1e-10)
    assert np.array_equal(arg, np.arange(len(rows)))
    assert np.allclose(c, np.eye(len(rows)), atol=1e-10)


def test_linear_case_identity():
    # the fit to the active set solves A xi = (E_1..E_m) (the paper prints this
    # as a row-vector product with A^{-1}); then E(cfg) = b . xi = sum_j c_j E_j
    pot = make_pot(level=8, S=1)
    B, _, _ = pool_rows(pot)
    rows, _ = og.maxvol(B)
    A = B[rows]
    E_act = np.random.default_rng(2).normal(size=len(rows))
    xi = np.linalg.solve(A, E_act)
    _, _, c = og.grade(B, A)
    assert np.allclose(B @ xi, c @ E_act, rtol=1e-8, atol=1e-8 * np.abs(B @ xi).max())


def test_maxvol_volume_grows_and_converges():
    pot = make_pot(level=8, S=1)
    B, _, _ = pool_rows(pot, n_cfg=60, seed=1)
    Bs = B / np.abs(B).max(axis=0)
    rows = list(og.initial_rows(B))
    vol = abs(np.linalg.det(Bs[rows]))
    for _ in range(50):
        gam, arg, c = og.grade(B, B[rows])
        i = int(np.argmax(gam))
        if gam[i] <= 1.0 + 1e-3:
            break
        k = int(arg[i])
        rows[k] = i
        new = abs(np.linalg.det(Bs[rows]))
        # the determinant grows by exactly |c_k| (matrix determinant lemma)
        assert np.isclose(new / vol, gam[i], rtol=1e-8)
        vol = new
    final, swaps = og.maxvol(B)
    gam, _, _ = og.grade(B, B[final])
    assert gam.max() <= 1.0 + 1e-3 + 1e-9


def _targets(pot_ref, batch, noise_seed=9, noise=1e-3):
    rng = np.random.default_rng(noise_seed)
    E, F, S = [], [], []
    for k in range(len(batch["n_atoms"])):
        pos, sp, cell, pbc = synth.config_of(batch, k)
        r = mtp.evaluate(pot_ref, pos, sp, cell, pbc)
        E.append(r["energy"] + rng.normal(0, noise))
        F.append(r["forces"] + rng.normal(0, noise, r["forces"].shape))
        S.append((r["virial"] if pbc else np.zeros((3, 3))) + rng.normal(0, noise, (3, 3)))
    return {"energy": np.array(E), "forces": np.concatenate(F), "virial": np.array(S)}


def _small_problem(level=8):
    student = make_pot(level=level, S=2, seed=21, xi_scale=1e-3)
    ref = make_pot(level=level, S=2, seed=22, xi_scale=1e-3)
    b = synth.mixed_batch(seed=5, n_configs=4, n_min=6, n_max=14, n_species_model=2)
    assert b["pbc"].any() and not b["pbc"].all()
    return student, b, _targets(ref, b)


@pytest.mark.parametrize("scaling", ol.SCALINGS)
def test_complex_step_gradient_matches_finite_differences(scaling):
    pot, b, tg = _small_problem()
    m = len(pot["xi"])
    idx = [0, 3, m - 1, m, m + 5, m + pot["c"].size - 1]
    g = ol.loss_grad(pot, b, tg, indices=idx, scaling=scaling)
    for t, p in enumerate(idx):
        q1, q2 = dict(pot), dict(pot)
        theta = np.concatenate([pot["xi"], pot["c"].ravel()])
        h = 1e-6 * max(1.0, abs(theta[p]))
        for q, s in ((q1, h), (q2, -h)):
            th = theta.copy()
            th[p] += s
            q["xi"], q["c"] = th[:m], th[m:].reshape(pot["c"].shape)
        fd = (ol.loss(q1, b, tg, scaling=scaling) - ol.loss(q2, b, tg, scaling=scaling)) / (2 * h)
        assert abs(fd - g[t]) <= 1e-6 * max(abs(g).max(), 1e-12), (p, fd, g[t])


def test_loss_is_quadratic_in_xi():
    pot, b, tg = _small_problem()
    d = np.random.default_rng(3).normal(size=len(pot["xi"])) * 1e-3
    vals = []
    for t in range(4):
        q = dict(pot)
        q["xi"] = pot["xi"] + t * d
        vals.append(ol.loss(q, b, tg))
    d2 = np.diff(vals, 2)
    assert np.isclose(d2[0], d2[1], rtol=1e-7)
    assert d2[0] > 0


def test_weighting_scalings_under_replication():
    # "structures": a supercell of the same structure has the same weight;
    # "vibrations": energy and force terms grow with the number of atoms.
    pot = make_pot(level=8, S=1, seed=30, xi_scale=1e-3)
    ref = make_pot(level=8, S=1, seed=31, xi_scale=1e-3)
    one = synth.fcc108(seed=3, a=4.05)
    pos, sp, cell, _ = synth.config_of(one, 0)
    sub = {"n_atoms": np.array([27]), "atom_offsets": np.array([0, 27]),
           "pos": pos[:27] * 0 + synth.supercell(np.eye(3) * 4.05, synth._FCC, (3, 3, 1))[0][:27],
           "species": sp[:27], "cell": np.array([np.diag([12.15, 12.15, 4.05])]), "pbc": np.array([1], np.uint8)}
    sub["pos"] = sub["pos"] + np.random.default_rng(0).normal(0, 0.08, sub["pos"].shape)
    reps = np.array(list(itertools.product(range(1), range(1), range(2))), float) @ sub["cell"][0]
    big = {"n_atoms": np.array([54]), "atom_offsets": np.array([0, 54]),
           "pos": (sub["pos"][None] + reps[:, None]).reshape(-1, 3),
           "species": np.tile(sub["species"], 2),
           "cell": np.array([sub["cell"][0] * np.array([[1], [1], [2]])]), "pbc": np.array([1], np.uint8)}
    t1 = _targets(ref, sub, noise=0.0)
    t2 = {"energy": 2 * t1["energy"], "forces": np.tile(t1["forces"], (2, 1)), "virial": 2 * t1["virial"]}
    for we, wf, ws in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        l1 = ol.loss(pot, sub, t1, we, wf, ws, scaling="structures")
        l2 = ol.loss(pot, big, t2, we, wf, ws, scaling="structures")
        assert np.isclose(l1, l2, rtol=1e-9)
    for we, wf, ws in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        l1 = ol.loss(pot, sub, t1, we, wf, ws, scaling="vibrations")
        l2 = ol.loss(pot, big, t2, we, wf, ws, scaling="vibrations")
        assert np.isclose(l2, 2 * l1, rtol=1e-9)


def test_error_report_definitions():
    batch = {"n_atoms": np.array([1, 2]), "atom_offsets": np.array([0, 1, 3]),
             "pbc": np.array([1, 0], np.uint8)}
    pred = {"energy": np.array([1.0, 4.0]), "forces": np.array([[1.0, 0, 0], [0, 0, 0], [0, 0, 3.0]]),
            "stress": np.array([np.eye(3), np.zeros((3, 3))])}
    ref = {"energy": np.array([0.0, 0.0]), "forces": np.zeros((3, 3)), "stress": np.zeros((2, 3, 3))}
    rep = ol.error_report(batch, pred, ref)
    # energies per atom: 1 and 2 -> RMSE sqrt((1 + 4) / 2)
    assert np.isclose(rep["energy_per_atom"]["rmse"], np.sqrt(2.5))
    assert np.isclose(rep["energy_per_atom"]["mae"], 1.5)
    # forces: config 1 mean square 1/3, config 2 mean square 9/6 -> sqrt((1/3 + 3/2) / 2)
    assert np.isclose(rep["force"]["rmse"], np.sqrt((1 / 3 + 1.5) / 2))
    assert np.isclose(rep["force"]["max"], 3.0)
    # stress: only the periodic config, |sigma|^2 / 9 = 3 / 9
    assert np.isclose(rep["stress"]["rmse"], np.sqrt(3 / 9))


def test_theta_rows_xi_part_is_b_and_c_part_matches_finite_differences():
    """Rows dE_k/dtheta of the nonlinear grade: E is linear in xi, so the xi
    columns are b exactly; the c columns against central differences of E."""
    pot = make_pot(level=8, S=2)
    b = synth.mixed_batch(seed=11, n_configs=3, n_min=6, n_max=14, n_species_model=2)
    m, nc = len(pot["xi"]), pot["c"].size
    idx = list(range(m)) + [m, m + 3, m + nc // 2, m + nc - 1]
    R = og.theta_rows(pot, b, indices=idx)
    for k in range(3):
        ref = mtp.evaluate(pot, *synth.config_of(b, k))
        np.testing.assert_allclose(R[k, :m], ref["b"], rtol=1e-12, atol=1e-12 * np.abs(ref["b"]).max())
        # Euler: E is homogeneous of degree 1 in xi
        assert abs(R[k, :m] @ pot["xi"] - ref["energy"]) <= 1e-12 * max(1.0, abs(ref["energy"]))
    theta = np.concatenate([pot["xi"], pot["c"].ravel()])
    for t, p in enumerate(idx[m:], start=m):
        h = 1e-6 * max(1.0, abs(theta[p]))
        E = []
        for sgn in (1, -1):
            th = theta.copy()
            th[p] += sgn * h
            q = dict(pot, xi=th[:m], c=th[m:].reshape(pot["c"].shape))
            E.append(np.array([mtp.evaluate(q, *synth.config_of(b, k))["energy"] for k in range(3)]))
        fd = (E[0] - E[1]) / (2 * h)
        np.testing.assert_allclose(R[:, t], fd, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(fd).max()))
        assert np.abs(R[:, t]).max() > 0   # the sampled c entries are used by these species pairs


def test_fire_step_special_cases():
    """The FIRE oracle: from rest it is a plain Euler step with the force; a
    velocity against the force is zeroed and the step shrinks; the mixing
    keeps |v| along a force parallel to v."""
    from oracle import relax as orx
    acc = orx.EV_PER_A_AMU_IN_A_PER_FS2
    prm = dict(dt_max=5.0, n_min=1, f_inc=1.1, f_dec=0.5, alpha_start=0.1, f_alpha=0.99)
    x = np.zeros((2, 3)); F = np.array([[1.0, 0, 0], [0, -2.0, 0]]); m = np.array([2.0, 4.0])
    x1, v1, st = orx.fire_step(x, np.zeros((2, 3)), F, m, (0.5, 0.1, 0), **prm)
    np.testing.assert_allclose(v1, 0.5 * acc * F / m[:, None], rtol=1e-15)
    np.testing.assert_allclose(x1, 0.5 * v1, rtol=1e-15)
    assert st == (0.5, 0.1, 1)
    x2, v2, st2 = orx.fire_step(x, -F, F, m, (0.5, 0.05, 7), **prm)
    assert st2 == (0.25, 0.1, 0)
    np.testing.assert_allclose(v2, 0.25 * acc * F / m[:, None], rtol=1e-15)
    v = np.array([[2.0, 0, 0]]); f = np.array([[3.0, 0, 0]])
    _x, v3, st3 = orx.fire_step(np.zeros((1, 3)), v, f, np.array([1e30]), (1.0, 0.1, 5), **prm)
    np.testing.assert_allclose(v3, v, rtol=1e-12)     # mixing along v keeps |v| (the kick is ~0)
    assert st3[0] == 1.1 and abs(st3[1] - 0.099) < 1e-15 and st3[2] == 6
