"""Oracle: one FIRE relaxation step (test infrastructure).

The relaxations of the paper's active learning (section 2.3) take a
configuration to a minimum of the potential.  FIRE is the method of Bitzek,
Koskinen, Gaehler, Moseler and Gumbsch, Phys. Rev. Lett. 97, 170201 (2006):
with the power P = F . v of the whole configuration, the velocities are mixed
towards the force while P >= 0, v <- (1 - alpha) v + alpha |v| F/|F|, and the
step grows (dt <- min(f_inc dt, dt_max), alpha <- f_alpha alpha) once more
than n_min such steps have passed in a row; when P < 0 the velocities are
zeroed, dt <- f_dec dt and alpha returns to alpha_start.  The motion is a
semi-implicit Euler step, v += dt F / m, x += dt v.

Units: Angstrom, fs, eV, atomic mass units (1 eV/(A amu) = 1/103.642696562
A/fs^2).
"""
from __future__ import annotations

import numpy as np

EV_PER_A_AMU_IN_A_PER_FS2 = 1.0 / 103.642696562


def fire_step(pos, vel, forces, masses, state, dt_max, n_min, f_inc, f_dec, alpha_start, f_alpha):
    """One step of one configuration.  pos, vel, forces [n, 3]; masses [n]
    (amu, per atom); state (dt, alpha, n_pos).  Returns the new pos, vel and
    state."""
    dt, alpha, n_pos = state
    P = float(np.sum(forces * vel))
    if P >= 0.0:
        vn = np.sqrt(np.sum(vel * vel))
        fn = np.sqrt(np.sum(forces * forces))
        v = (1.0 - alpha) * vel + (alpha * vn / fn if fn > 0 else 0.0) * forces
        if n_pos > n_min:
            dt = min(dt * f_inc, dt_max)
            alpha = alpha * f_alpha
        n_pos = n_pos + 1
    else:
        v = np.zeros_like(vel)
        dt = dt * f_dec
        alpha = alpha_start
        n_pos = 0
    v = v + dt * EV_PER_A_AMU_IN_A_PER_FS2 * forces / masses[:, None]
    return pos + dt * v, v, (dt, alpha, n_pos)
