"""Oracle: extrapolation grade and MaxVol active-set selection (test infrastructure).

Follows the paper, section 2.3 "Active learning: query strategy":

* eq. matrix-B: row k of B is b(cfg_k), b_alpha(cfg) = sum_i B_alpha(n_i).
* The active set is m rows of B; A is that m x m submatrix.
* For a configuration with row b: (c_1 .. c_m) = b A^{-1},
  gamma = max_j |c_j|, and if gamma > 1 the row k = argmax_j |c_j| of A
  is the one to replace (the MaxVol step of Goreinov et al., cited there).

Readings where the paper is silent: ties in argmax go to the lowest index;
the MaxVol iteration over a pool stops when no entry of B_pool A^{-1}
exceeds 1 + delta (delta = 1e-3) or after 100 m swaps; its start is the row
set chosen by LU with partial pivoting of the column-equilibrated pool.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def grade(b, A):
    """gamma and argmax for rows b [K, m] against the active-set matrix A [m, m].

    c = b A^{-1} is found by solving A^T c^T = b^T with LAPACK (column
    equilibration of A does not change c: (b D)(A D)^{-1} = b A^{-1})."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    A = np.asarray(A, dtype=np.float64)
    scale = 1.0 / np.max(np.abs(A), axis=0)
    c = np.linalg.solve((A * scale).T, (b * scale).T).T
    ac = np.abs(c)
    return ac.max(axis=1), ac.argmax(axis=1), c


def initial_rows(B_pool):
    """m row indices of the pool picked by LU with partial pivoting."""
    B = np.asarray(B_pool, dtype=np.float64)
    K, m = B.shape
    if K < m:
        raise ValueError("pool has fewer rows than the basis size")
    Bs = B / np.max(np.abs(B), axis=0)
    P, _L, _U = scipy.linalg.lu(Bs)         # Bs = P L U
    perm = np.argmax(P, axis=0)             # row of Bs that lands in position t
    return np.sort(perm[:m])


def maxvol(B_pool, delta=1e-3, max_swaps=None, start=None):
    """Row indices of a dominant m x m submatrix of B_pool and the swap count.

    Each step replaces row j of A by pool row i at the largest |C_ij| of
    C = B_pool A^{-1}; |det A| grows by that factor every step.  start: the
    starting rows (default: initial_rows)."""
    B = np.asarray(B_pool, dtype=np.float64)
    K, m = B.shape
    rows = list(initial_rows(B)) if start is None else [int(r) for r in start]
    if max_swaps is None:
        max_swaps = 100 * m
    swaps = 0
    while swaps < max_swaps:
        A = B[rows]
        _, _, C = grade(B, A)
        ac = np.abs(C)
        i, j = np.unravel_index(np.argmax(ac), ac.shape)
        if ac[i, j] <= 1.0 + delta:
            break
        rows[j] = int(i)
        swaps += 1
    return np.array(rows, dtype=np.int64), swaps


def theta_rows(pot, batch, indices=None, h=1e-30):
    """Rows of the nonlinear grade: dE_k/dtheta for every configuration k of
    the batch, theta = [xi, c.ravel()] (section 2.3: the matrix B built from
    the derivatives of the energy in all parameters, linearised at the current
    theta; its xi part is b).  Columns are the flat theta indices requested
    (all when None).  Each column is one complex-step evaluation (Squire and
    Trapp, 1998): dE_k/dtheta_p = Im E_k(theta + i h e_p) / h, exact to
    rounding since E is real-analytic in theta."""
    from . import mtp
    import synth
    m = len(pot["xi"])
    nc = pot["c"].size
    idx = list(range(m + nc)) if indices is None else list(indices)
    K = len(batch["n_atoms"])
    R = np.zeros((K, len(idx)))
    for t, p in enumerate(idx):
        q = dict(pot)
        xi = pot["xi"].astype(np.complex128)
        c = pot["c"].astype(np.complex128).ravel()
        if p < m:
            xi[p] += 1j * h
        else:
            c[p - m] += 1j * h
        q["xi"] = xi
        q["c"] = c.reshape(pot["c"].shape)
        for k in range(K):
            R[k, t] = np.imag(mtp.evaluate(q, *synth.config_of(batch, k))["energy"]) / h
    return R
