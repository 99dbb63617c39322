"""Training of a moment tensor potential (paper, section 2.2).

The loss of eq. Fitting is minimised over theta = (xi, c) with L-BFGS; every
loss and gradient comes from the library (mtp_loss_grad), so the host only
runs the optimiser's two-loop recursion on the parameter vector.  Between
L-BFGS rounds xi can be refitted exactly at the current c from the normal
equations (the loss is linear least squares in xi: mtp_normal_equations,
mtp_solve_normal).  `ensemble` trains several potentials from seeded
perturbations of the starting radial coefficients; the spread of their
predictions is the usual uncertainty estimate of an ensemble.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize

from .model import Batch, Potential

DEFAULT_WEIGHTS = {"w_e": 1.0, "w_f": 0.01, "w_s": 0.001, "scaling": "vibrations"}


def fit(P: Potential, batch: Batch, E_t, F_t, W_t, rounds=2, iters=200, refit_xi=True, weights=None,
        precision="fp64"):
    """Trains P in place on one batch with targets E_t [K], F_t [N,3], W_t
    [K,3,3] (virials, eV).  Each round refits xi by the normal equations
    (when refit_xi) and then runs at most `iters` L-BFGS iterations over all
    of theta.  Returns {"loss": final loss, "history": the loss at every
    evaluation, "rounds": [(loss after the xi refit, loss after L-BFGS)]}."""
    w = dict(DEFAULT_WEIGHTS if weights is None else weights)
    c0, xi0 = P.get_params()
    m = len(xi0)
    history = []

    def loss_and_grad(theta):
        P.set_params(c=theta[m:], xi=theta[:m])
        loss, grad = P.loss_grad(batch, E_t, F_t, W_t, precision=precision, **w)
        value = float(loss.item())
        history.append(value)
        return value, grad.cpu().numpy()

    theta = np.concatenate([xi0, c0])
    summary = []
    for _ in range(rounds):
        if refit_xi:
            P.set_params(c=theta[m:], xi=theta[:m])
            theta[:m] = P.fit_xi(batch, E_t, F_t, W_t, precision="fp64", **w).cpu().numpy()
        after_refit = loss_and_grad(theta)[0]
        res = scipy.optimize.minimize(loss_and_grad, theta, jac=True, method="L-BFGS-B",
                                      options={"maxiter": iters})
        theta = res.x
        summary.append((after_refit, float(res.fun)))
    final = loss_and_grad(theta)[0]   # installs theta and records its loss
    return {"loss": final, "history": history, "rounds": summary}


def ensemble(path, n, batch: Batch, E_t, F_t, W_t, seed=0, c_sigma=0.05, device=0, **fit_kwargs):
    """n potentials loaded from `path`, each starting from its radial
    coefficients times (1 + N(0, c_sigma^2)) drawn from seed + k, trained by
    fit().  Returns the trained potentials and their fit summaries."""
    members, results = [], []
    for k in range(n):
        P = Potential(path, device=device)
        c, xi = P.get_params()
        rng = np.random.default_rng(seed + k)
        P.set_params(c=c * (1.0 + c_sigma * rng.normal(size=c.shape)), xi=xi)
        results.append(fit(P, batch, E_t, F_t, W_t, **fit_kwargs))
        members.append(P)
    return members, results
