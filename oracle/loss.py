"""Oracle: training loss, its parameter gradient and error metrics (test infrastructure).

Follows the paper, section 2.2 "Training on a quantum-mechanical database":

* eq. Fitting: sum_k [ w_e (E_k - E^qm_k)^2 + w_f sum_i |f_i - f^qm_i|^2
  + w_s |sigma_k - sigma^qm_k|^2 ], |sigma|^2 the Frobenius norm.
* weighting "molecules": eq. Fitting as written (the paper pairs it with
  w_s = 0; the weights are taken as given);
  "structures" (eq. train-structures): w_e / N^2, w_f / N, w_s / N^2;
  "vibrations" (eq. train-vibrations, the default): w_e / N, w_f, w_s / N.
* eqs. E_RMSE, F_RMSE, S_RMSE for the error report.

Readings: the stress in eq. Fitting is taken as the extensive virial stress
W = dE/d eps = volume * sigma (eV).  The paper's rationale for the scalings
(a larger cell of the same structure keeps the same relative weight of
energy and stress under "structures") holds only for an extensive stress: with
W, the "structures" loss of a supercell equals that of the cell, and every
"vibrations" term grows with N.  Free clusters have no stress term.  The gradient with respect to theta = (xi, c) is computed by
the complex-step method (Squire and Trapp, 1998): L is real-analytic in
theta, so dL/dtheta_p = Im L(theta + i h e_p) / h with h = 1e-30, exact to
rounding (no subtractive cancellation).  Every square in the loss is written
as x * x, never |x|^2, so the complex extension stays analytic.
"""
from __future__ import annotations

import numpy as np

import synth
from . import mtp

SCALINGS = ("molecules", "structures", "vibrations")


def scaled_weights(w_e, w_f, w_s, n, scaling):
    if scaling == "molecules":
        return w_e, w_f, w_s
    if scaling == "structures":
        return w_e / n ** 2, w_f / n, w_s / n ** 2
    if scaling == "vibrations":
        return w_e / n, w_f, w_s / n
    raise ValueError(scaling)


def predictions(pot, batch):
    """Per config E, F and the virial W (None for clusters)."""
    out = []
    for k in range(len(batch["n_atoms"])):
        pos, sp, cell, pbc = synth.config_of(batch, k)
        r = mtp.evaluate(pot, pos, sp, cell, pbc)
        out.append((r["energy"], r["forces"], r["virial"] if pbc else None))
    return out


def loss(pot, batch, targets, w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations"):
    """targets: dict with energy [K], forces [N, 3], virial [K, 3, 3] (eV)."""
    total = 0.0
    offs = batch["atom_offsets"]
    for k, (E, F, S) in enumerate(predictions(pot, batch)):
        n = int(batch["n_atoms"][k])
        we, wf, ws = scaled_weights(w_e, w_f, w_s, n, scaling)
        dE = E - targets["energy"][k]
        dF = F - targets["forces"][offs[k]:offs[k + 1]]
        total = total + we * dE * dE + wf * np.sum(dF * dF)
        if S is not None:
            dS = S - targets["virial"][k]
            total = total + ws * np.sum(dS * dS)
    return total


def loss_grad(pot, batch, targets, indices=None, h=1e-30, **kw):
    """dL/dtheta at the requested flat indices of theta = [xi, c.ravel()]
    (all when indices is None), by the complex-step method."""
    m = len(pot["xi"])
    nc = pot["c"].size
    if indices is None:
        indices = range(m + nc)
    g = np.zeros(len(list(indices)))
    for t, p in enumerate(indices):
        q = dict(pot)
        xi = pot["xi"].astype(np.complex128)
        c = pot["c"].astype(np.complex128).ravel()
        if p < m:
            xi[p] += 1j * h
        else:
            c[p - m] += 1j * h
        q["xi"] = xi
        q["c"] = c.reshape(pot["c"].shape)
        g[t] = np.imag(loss(q, batch, targets, **kw)) / h
    return g


def error_report(batch, pred, ref):
    """RMSE / MAE / max of energy per atom, force components and stress
    components (eqs. E_RMSE, F_RMSE, S_RMSE and the matching MAE and max).

    pred and ref are dicts: energy [K], forces [N, 3], stress [K, 3, 3]
    (stress rows of clusters are ignored)."""
    n = batch["n_atoms"].astype(np.float64)
    offs = batch["atom_offsets"]
    K = len(n)
    de = (np.asarray(pred["energy"]) - np.asarray(ref["energy"])) / n
    dF = np.asarray(pred["forces"]) - np.asarray(ref["forces"])
    rep = {"energy_per_atom": {"rmse": float(np.sqrt(np.mean(de * de))),
                               "mae": float(np.mean(np.abs(de))),
                               "max": float(np.max(np.abs(de)))}}
    # per-configuration means over 3 N_k components, then over configurations
    ms = np.array([np.mean(dF[offs[k]:offs[k + 1]] ** 2) for k in range(K)])
    ma = np.array([np.mean(np.abs(dF[offs[k]:offs[k + 1]])) for k in range(K)])
    rep["force"] = {"rmse": float(np.sqrt(np.mean(ms))), "mae": float(np.mean(ma)),
                    "max": float(np.max(np.abs(dF)))}
    pbc = batch["pbc"].astype(bool)
    if pbc.any() and "stress" in pred:
        dS = (np.asarray(pred["stress"]) - np.asarray(ref["stress"]))[pbc].reshape(-1, 9)
        rep["stress"] = {"rmse": float(np.sqrt(np.mean(np.sum(dS * dS, axis=1) / 9.0))),
                         "mae": float(np.mean(np.abs(dS))), "max": float(np.max(np.abs(dS)))}
    return rep
