"""Writes the seeded, calibrated potential files under tests/golden/potentials.

Test infrastructure: uses the oracle only.  Run from the repository root:
    python -m oracle.make_potentials [name ...]

Each potential is the basis of its level (oracle.basis) with parameters
drawn by synth.draw_model (c ~ N(0, 0.1^2), xi ~ N(0, 1)).  With raw-Angstrom
moments those draws give site energies of 1e3..1e7 eV, so xi is calibrated:
xi_alpha <- xi_alpha / (sqrt(m) s_alpha), s_alpha the RMS over a calibration
set of atoms of B_alpha(n_i) computed by the FP64 oracle (s_alpha = 1 where
it is 0).  This keeps the function space and the draw and makes site
energies O(1) eV.  The uncalibrated draw is written beside it as *_raw.mtp.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

import synth
from . import basis as obasis
from . import mtp
from .potential import write_potential

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "tests", "golden", "potentials")

# name: (level, species, N_Q, R_min, R_cut, model seed, calibration set)
SPECS = {
    "lev8_s1": (8, 1, 8, 2.0, 5.0, 101, ("fcc108",)),
    "lev12_s2": (12, 2, 8, 2.0, 5.0, 107, ("mixed", 11, 32, 8, 64)),
    "lev16_s2": (16, 2, 8, 2.0, 5.0, 102, ("bcc_alloy", 2048)),
    "lev16_s3": (16, 3, 8, 2.0, 5.0, 103, ("mixed", 1, 64, 8, 256)),
    "lev20_s3": (20, 3, 8, 2.0, 5.0, 104, ("mixed", 2, 64, 32, 128)),
    "lev20_s3_ref": (20, 3, 8, 2.0, 5.0, 105, ("mixed", 2, 64, 32, 128)),
    "lev24_s3": (24, 3, 8, 2.0, 5.0, 106, ("fcc_alloy", 128)),
}


def calibration_B(pot, calib, max_atoms=2048):
    rng = np.random.default_rng(12345)
    rows = []
    if calib[0] == "fcc108":
        b = synth.fcc108(seed=0)
    elif calib[0] == "bcc_alloy":
        b = synth.bcc_alloy(seed=0)
    elif calib[0] == "fcc_alloy":
        b = synth.fcc_alloy(seed=0)
    elif calib[0] == "mixed":
        _, seed, n_cfg, n_min, n_max = calib
        b = synth.mixed_batch(seed=seed, n_configs=n_cfg, n_min=n_min, n_max=n_max,
                              n_species_model=pot["n_species"])
    else:
        raise ValueError(calib)
    total = int(b["n_atoms"].sum())
    budget = min(total, calib[1] if calib[0] in ("bcc_alloy", "fcc_alloy") else max_atoms)
    take = np.sort(rng.choice(total, size=budget, replace=False)) if budget < total else np.arange(total)
    offs = b["atom_offsets"]
    for k in range(len(b["n_atoms"])):
        sel = take[(take >= offs[k]) & (take < offs[k + 1])] - offs[k]
        if len(sel) == 0:
            continue
        pos, sp, cell, pbc = synth.config_of(b, k)
        # full 3^nu tensors: fewer centres per call at high levels
        step = 256 if pot["level"] <= 20 else 8
        for s in range(0, len(sel), step):
            _, B, _ = mtp._eval_centers(pot, pos, sp, cell, pbc, sel[s:s + step], want_grad=False)
            rows.append(B)
    return np.concatenate(rows)


def make(name):
    level, S, n_q, r_min, r_cut, seed, calib = SPECS[name]
    t0 = time.time()
    graphs = list(obasis.connected_contractions(level))
    funcs = list(obasis.basis(level))
    moments = obasis.moments_used(level)
    n_mu = 1 + max(mu for mu, _ in moments)
    c, xi = synth.draw_model(seed, n_mu, S, n_q, len(funcs))
    pot = dict(level=level, n_species=S, n_q=n_q, r_min=r_min, r_cut=r_cut,
               moments=moments, graphs=graphs, basis=funcs, c=c, xi=xi)
    os.makedirs(OUT, exist_ok=True)
    write_potential(os.path.join(OUT, name + "_raw.mtp"), pot)
    B = calibration_B(pot, calib)
    s = np.sqrt(np.mean(B * B, axis=0))
    s[s == 0.0] = 1.0
    pot["xi"] = xi / (np.sqrt(len(funcs)) * s)
    write_potential(os.path.join(OUT, name + ".mtp"), pot)
    print(f"{name}: m={len(funcs)} graphs={len(graphs)} calib_atoms={len(B)} "
          f"({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(SPECS)):
        make(n)
