"""Pins of two oracle helpers that the full-size GPU tests and the MaxVol
tests rely on.

* ``mtp.evaluate_sampled`` (site energies of some atoms and exact forces on
  others, section 2.1) must equal the full evaluation on those atoms: a force
  needs dV_i/dr_ik of every atom i that sees atom k, so a dropped neighbour
  contribution, a wrong sign of the reverse share or a missed self-image
  shows up as a force difference.
* ``grade.initial_rows`` (the starting rows of MaxVol, section 2.3) must be the
  pivot rows of Gaussian elimination with partial pivoting, written out here
  as a plain loop (largest entry of the current column among the rows not yet
  chosen, lowest index on ties), not taken from a library.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import basis as ob
from oracle import grade as og
from oracle import mtp


def make_pot(level=12, S=3, n_q=8, seed=11):
    funcs = list(ob.basis(level))
    moments = ob.moments_used(level)
    n_mu = 1 + max(mu for mu, _ in moments)
    c, xi = synth.draw_model(seed, n_mu, S, n_q, len(funcs))
    return dict(level=level, n_species=S, n_q=n_q, r_min=2.0, r_cut=5.0, moments=moments,
                graphs=list(ob.connected_contractions(level)), basis=funcs, c=c, xi=xi)


def _configs():
    batch = synth.mixed_batch(seed=21, n_configs=12, n_min=8, n_max=40, n_species_model=3)
    out = []
    kinds = {True: None, False: None}
    for k in range(12):
        cfg = synth.config_of(batch, k)
        if kinds[cfg[3]] is None or len(out) < 3:
            out.append(cfg)
            kinds[cfg[3]] = k
    assert any(c[3] for c in out) and any(not c[3] for c in out)
    # a periodic cell narrower than 2 R_cut: atoms see their own images
    out.append((np.array([[0.1, 0.2, 0.3], [1.4, 1.3, 1.2]]), np.array([0, 2]), np.eye(3) * 2.8, True))
    # one atom in a simple cubic cell: every neighbour is a self-image
    out.append((np.zeros((1, 3)), np.array([1]), np.eye(3) * 2.6, True))
    return out


@pytest.mark.parametrize("case", range(5))
def test_evaluate_sampled_equals_full_evaluation(case):
    pot = make_pot()
    pos, sp, cell, pbc = _configs()[case]
    n = len(pos)
    full = mtp.evaluate(pot, pos, sp, cell, pbc)
    rng = np.random.default_rng(case)
    e_atoms = np.sort(rng.choice(n, size=min(n, 5), replace=False))
    f_atoms = np.sort(rng.choice(n, size=min(n, 4), replace=False))
    site, forces = mtp.evaluate_sampled(pot, pos, sp, cell, pbc, e_atoms, f_atoms)
    s_scale = max(1.0, np.abs(full["site"]).max())
    # per-pair gradients are of the order of the site energies per Angstrom;
    # forces that cancel (a one-atom cell) keep their rounding
    f_scale = max(1.0, np.abs(full["forces"]).max(), s_scale)
    assert np.abs(site - full["site"][e_atoms]).max() <= 1e-13 * s_scale
    assert np.abs(forces - full["forces"][f_atoms]).max() <= 1e-13 * f_scale
    # the forces are not dominated by any single centre's share: every atom
    # that sees a force atom contributes (dropping one moves the force)
    if n > 2:
        assert np.abs(full["forces"][f_atoms]).max() > 1e-6 * f_scale


def test_evaluate_sampled_force_atoms_outside_energy_atoms():
    pot = make_pot(level=8, S=2)
    pos, sp, cell, pbc = synth.config_of(synth.mixed_batch(seed=5, n_configs=1, n_min=60, n_max=60,
                                                          n_species_model=2), 0)
    full = mtp.evaluate(pot, pos, sp, cell, pbc)
    site, forces = mtp.evaluate_sampled(pot, pos, sp, cell, pbc, [0], [len(pos) - 1, 7])
    assert abs(site[0] - full["site"][0]) <= 1e-13 * max(1.0, abs(full["site"][0]))
    assert np.abs(forces - full["forces"][[len(pos) - 1, 7]]).max() <= 1e-13 * np.abs(full["forces"]).max()


def _gepp_pivot_rows(B):
    """Gaussian elimination with partial pivoting on the columns of B in
    order; returns the pivot rows, ascending."""
    W = np.array(B, dtype=np.float64)
    K, m = W.shape
    chosen = []
    free = list(range(K))
    for t in range(m):
        best = free[0]
        for r in free[1:]:
            if abs(W[r, t]) > abs(W[best, t]):
                best = r
        chosen.append(best)
        free.remove(best)
        for r in free:
            l = W[r, t] / W[best, t]
            assert abs(l) <= 1.0          # partial pivoting bounds every multiplier
            W[r, t:] -= l * W[best, t:]
    return sorted(chosen)


@pytest.mark.parametrize("K,m,seed", [(36, 12, 0), (50, 20, 1), (20, 20, 2), (64, 9, 3)])
def test_initial_rows_are_partial_pivoting_rows(K, m, seed):
    rng = np.random.default_rng(seed)
    scales = 10.0 ** rng.uniform(-3, 3, size=m)
    B = rng.normal(size=(K, m)) * scales
    rows = og.initial_rows(B)
    assert len(rows) == m and len(set(rows.tolist())) == m
    assert rows.tolist() == _gepp_pivot_rows(B / np.abs(B).max(axis=0))
    # the chosen submatrix is well inside the pool's rank: nonsingular
    assert abs(np.linalg.det(B[rows] / np.abs(B[rows]).max(axis=0))) > 1e-12


def test_initial_rows_on_descriptor_rows():
    pot = make_pot(level=8, S=2)
    batch = synth.mixed_batch(seed=9, n_configs=30, n_min=8, n_max=24, n_species_model=2)
    b = np.array([mtp.evaluate(pot, *synth.config_of(batch, k))["b"] for k in range(30)])
    rows = og.initial_rows(b)
    assert rows.tolist() == _gepp_pivot_rows(b / np.abs(b).max(axis=0))


def test_initial_rows_rejects_a_short_pool():
    with pytest.raises(ValueError):
        og.initial_rows(np.ones((3, 4)))
