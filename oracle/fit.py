"""Oracle: the training problem in xi at fixed c as linear least squares (test infrastructure).

Paper, section 2.2, eq. Fitting, with the per-configuration weights of the
scalings (eqs. train-structures, train-vibrations; see oracle.loss).  The site
energy is a linear combination of the basis functions with coefficients xi
(section 2.1), so energies, forces and virials are linear in xi at fixed
radial coefficients c, and the loss restricted to xi is a weighted linear
least-squares problem:

    L(xi) = sum_r w_r (J xi - y)_r^2 = xi^T H xi - 2 g^T xi + yy,
    H = J^T W J,  g = J^T W y,  yy = y^T W y,  H xi* = g.

Rows r: the K energies, then the 3 N force components (atom-major), then the
9 K virial components (configuration-major), the layout the library's
normal-equation entry point documents.  Column alpha of J is the oracle
evaluation of the potential with xi = e_alpha (energies, forces, virials).
Clusters have no stress term (weight 0).  H is badly scaled (its diagonal
spans many decades across basis functions of different degree), so the solve
scales it to unit diagonal: (D H D) z = D g, xi = D z with D = diag(H)^(-1/2),
D H D handed to numpy.linalg.solve (LAPACK LU with partial pivoting).
"""
from __future__ import annotations

import numpy as np

import synth
from . import mtp
from .loss import scaled_weights


def n_rows(batch):
    K = len(batch["n_atoms"])
    return K + 3 * int(batch["n_atoms"].sum()) + 9 * K


def row_weights(batch, w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations"):
    K = len(batch["n_atoms"])
    N = int(batch["n_atoms"].sum())
    w = np.zeros(n_rows(batch))
    offs = batch["atom_offsets"]
    for k in range(K):
        n = int(batch["n_atoms"][k])
        if n == 0:
            continue
        we, wf, ws = scaled_weights(w_e, w_f, w_s, n, scaling)
        w[k] = we
        w[K + 3 * offs[k]:K + 3 * offs[k + 1]] = wf
        if batch["pbc"][k]:
            w[K + 3 * N + 9 * k:K + 3 * N + 9 * (k + 1)] = ws
    return w


def targets_vector(batch, targets):
    return np.concatenate([np.asarray(targets["energy"], dtype=np.float64).ravel(),
                           np.asarray(targets["forces"], dtype=np.float64).ravel(),
                           np.asarray(targets["virial"], dtype=np.float64).ravel()])


def jacobian(pot, batch):
    """J [R, m]: column alpha = energies, forces, virials with xi = e_alpha."""
    m = len(pot["xi"])
    K = len(batch["n_atoms"])
    N = int(batch["n_atoms"].sum())
    offs = batch["atom_offsets"]
    J = np.zeros((n_rows(batch), m))
    for a in range(m):
        q = dict(pot)
        q["xi"] = np.zeros(m)
        q["xi"][a] = 1.0
        for k in range(K):
            r = mtp.evaluate(q, *synth.config_of(batch, k))
            J[k, a] = r["energy"]
            J[K + 3 * offs[k]:K + 3 * offs[k + 1], a] = np.asarray(r["forces"]).ravel()
            J[K + 3 * N + 9 * k:K + 3 * N + 9 * (k + 1), a] = np.asarray(r["virial"]).ravel()
    return J


def normal_equations(pot, batch, targets, w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations", J=None):
    """H [m, m], g [m], yy of the loss in xi at the potential's c."""
    if J is None:
        J = jacobian(pot, batch)
    w = row_weights(batch, w_e, w_f, w_s, scaling)
    y = targets_vector(batch, targets)
    y = np.where(w != 0.0, y, 0.0)
    WJ = J * w[:, None]
    return J.T @ WJ, WJ.T @ y, float(y @ (w * y))


def solve(H, g):
    d = 1.0 / np.sqrt(np.diag(H))
    return d * np.linalg.solve(H * d[:, None] * d[None, :], d * g)
