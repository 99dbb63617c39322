"""Pins of the oracle's normal equations in xi (paper, section 2.2, eq.
Fitting at fixed c) against the loss as the paper defines it and against a
known minimiser."""
import numpy as np
import pytest

import synth
from oracle import fit as of
from oracle import loss as ol
from oracle import mtp

from test_oracle_mtp import make_pot


def _batch(S, seed=11, n=5):
    b = synth.mixed_batch(seed=seed, n_configs=n, n_min=6, n_max=16, n_species_model=S)
    assert b["pbc"].any() and not b["pbc"].all()
    return b


def _predict(pot, batch):
    E, F, W = [], [], []
    for k in range(len(batch["n_atoms"])):
        r = mtp.evaluate(pot, *synth.config_of(batch, k))
        E.append(r["energy"])
        F.append(r["forces"])
        W.append(r["virial"])
    return {"energy": np.array(E), "forces": np.concatenate(F), "virial": np.array(W)}


def _noisy(pred, seed):
    rng = np.random.default_rng(seed)
    return {k: v + rng.normal(0, 0.05, np.shape(v)) for k, v in pred.items()}


@pytest.mark.parametrize("level,S", [(8, 1), (12, 2)])
@pytest.mark.parametrize("scaling", ["molecules", "structures", "vibrations"])
def test_quadratic_form_is_the_loss(level, S, scaling):
    # xi^T H xi - 2 g^T xi + yy equals the loss of eq. Fitting evaluated
    # directly (oracle.loss) at any xi, clusters' stress rows excluded
    pot = make_pot(level=level, S=S)
    b = _batch(S)
    tg = _noisy(_predict(pot, b), 1)
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling=scaling)
    H, g, yy = of.normal_equations(pot, b, tg, **w)
    dd = np.sqrt(np.outer(np.diag(H), np.diag(H)))
    assert np.all(np.abs(H - H.T) <= 1e-13 * dd)
    rng = np.random.default_rng(4)
    for _ in range(3):
        xi = pot["xi"] * (1 + 0.5 * rng.normal(size=pot["xi"].shape))
        q = dict(pot, xi=xi)
        L = ol.loss(q, b, tg, **w)
        Lq = xi @ H @ xi - 2 * g @ xi + yy
        assert abs(Lq - L) <= 1e-9 * abs(L)


@pytest.mark.parametrize("level,S", [(8, 1), (12, 2)])
def test_noiseless_targets_recover_xi(level, S):
    # targets from a reference potential with the same c: the minimiser is
    # the reference xi, recovered to about cond(D H D) * eps
    pot = make_pot(level=level, S=S)
    b = _batch(S, seed=12, n=8)
    ref = dict(pot, xi=pot["xi"] * (1 + 0.3 * np.random.default_rng(5).normal(size=pot["xi"].shape)))
    tg = _predict(ref, b)
    H, g, yy = of.normal_equations(pot, b, tg)
    xi = of.solve(H, g)
    d = 1 / np.sqrt(np.diag(H))
    cond = np.linalg.cond(H * d[:, None] * d[None, :])
    err = np.max(np.abs((xi - ref["xi"]) / d)) / np.max(np.abs(ref["xi"] / d))
    assert err <= max(1e-12, 1e-14 * cond), (err, cond)
    # the residual vanishes: L(xi*) = yy - g^T xi* = 0 up to rounding
    assert abs(yy - g @ xi) <= 1e-8 * yy


def test_loss_gradient_vanishes_at_the_solution():
    # dL/dxi by complex steps of the loss itself (oracle.loss_grad) is zero at
    # the normal-equation solution and not at the starting xi
    pot = make_pot(level=8, S=1)
    b = _batch(1)
    tg = _noisy(_predict(pot, b), 2)
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations")
    H, g, _ = of.normal_equations(pot, b, tg, **w)
    xi = of.solve(H, g)
    m = len(xi)
    g0 = ol.loss_grad(pot, b, tg, indices=range(m), **w)
    g1 = ol.loss_grad(dict(pot, xi=xi), b, tg, indices=range(m), **w)
    d = 1 / np.sqrt(np.diag(H))
    # compare in the scaled variables xi' = xi / d (gradient d * dL/dxi)
    assert np.max(np.abs(d * g1)) <= 1e-9 * np.max(np.abs(d * g0))


def test_rows_and_weights_layout():
    # energies first, force components atom-major, virials configuration-major
    pot = make_pot(level=8, S=1)
    b = _batch(1, n=4)
    K, N = 4, int(b["n_atoms"].sum())
    J = of.jacobian(pot, b)
    assert J.shape == (K + 3 * N + 9 * K, len(pot["xi"]))
    pred = _predict(pot, b)
    np.testing.assert_allclose(J @ pot["xi"], of.targets_vector(b, pred), rtol=1e-12,
                               atol=1e-12 * np.abs(J @ pot["xi"]).max())
    w = of.row_weights(b, 2.0, 0.5, 0.25, "vibrations")
    n = b["n_atoms"]
    np.testing.assert_allclose(w[:K], 2.0 / n)
    assert np.all(w[K:K + 3 * N] == 0.5)
    for k in range(K):
        v = w[K + 3 * N + 9 * k:K + 3 * N + 9 * (k + 1)]
        assert np.all(v == (0.25 / n[k] if b["pbc"][k] else 0.0))
