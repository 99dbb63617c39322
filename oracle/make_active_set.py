"""Writes the seeded active set of the level-16, 3-species potential.

Test infrastructure: uses the oracle only.  Run from the repository root:
    python -m oracle.make_active_set

Pool: 4 m configurations from the mixed generator (seed 5, 8..256 atoms);
rows b(cfg) = sum_i B(n_i) from the FP64 oracle (eq. matrix-B); the active
set is the MaxVol selection of m rows (oracle.grade.maxvol).  Output:
tests/golden/active_lev16_s3.npz with A [m, m] (rows in selection order,
columns in the potential file's basis order) and the pool indices.
"""
from __future__ import annotations

import os
import time

import numpy as np

import synth
from . import mtp
from .grade import maxvol
from .potential import read_potential

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POT = os.path.join(ROOT, "tests", "golden", "potentials", "lev16_s3.mtp")
OUT = os.path.join(ROOT, "tests", "golden", "active_lev16_s3.npz")


def main():
    pot = read_potential(POT)
    m = len(pot["xi"])
    pool = synth.mixed_batch(seed=5, n_configs=4 * m, n_min=8, n_max=256, n_species_model=3)
    t0 = time.time()
    rows = []
    for k in range(4 * m):
        pos, sp, cell, pbc = synth.config_of(pool, k)
        _, B, _ = mtp._eval_centers(pot, pos, sp, cell, pbc, np.arange(len(pos)), want_grad=False)
        rows.append(B.sum(axis=0))
    Bp = np.array(rows)
    sel, swaps = maxvol(Bp)
    np.savez(OUT, A=Bp[sel], pool_rows=sel, pool_seed=5, pool_size=4 * m)
    print(f"active set: m={m}, pool={4 * m}, swaps={swaps}, {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
