"""Seeded synthetic inputs shared by the oracle tests and the product path.

This module builds geometry and draws random numbers only; it holds none of
the potential's arithmetic.  The workloads stand in for the paper's own
systems (a 108-atom fcc Al box in Example 2, small fcc/bcc/hcp alloy cells
in Example 3, a bcc metal in Example 1); no dataset is read.

Draw order inside one generator call is fixed: geometry -> displacements ->
species.  Model parameters are drawn by ``draw_model`` from their own seed.

A batch is a dict of numpy arrays:
    n_atoms      int64 [n_cfg]
    atom_offsets int64 [n_cfg + 1]
    pos          float64 [N, 3]   (Angstrom)
    species      int32 [N]
    cell         float64 [n_cfg, 3, 3]  (rows are lattice vectors; zero for clusters)
    pbc          uint8 [n_cfg]    (1 periodic in 3D, 0 free cluster)
"""
from __future__ import annotations

import itertools

import numpy as np

SQRT83 = np.sqrt(8.0 / 3.0)

# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------

_FCC = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
_BCC = np.array([[0, 0, 0], [.5, .5, .5]], dtype=np.float64)
_HCP = np.array([[0, 0, 0], [1 / 3, 1 / 3, .5]], dtype=np.float64)


def unit_cell(kind, nn_dist):
    """(cell rows, fractional basis) of a lattice with nearest-neighbour
    distance nn_dist."""
    if kind == "fcc":
        a = nn_dist * np.sqrt(2.0)
        return np.eye(3) * a, _FCC
    if kind == "bcc":
        a = nn_dist * 2.0 / np.sqrt(3.0)
        return np.eye(3) * a, _BCC
    if kind == "hcp":
        a = nn_dist
        cell = np.array([[a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0], [0, 0, a * SQRT83]])
        return cell, _HCP
    raise ValueError(kind)


def supercell(cell, basis, reps):
    """Tile a unit cell reps = (n1, n2, n3) times.  Returns (pos, cell)."""
    n1, n2, n3 = reps
    grid = np.array(list(itertools.product(range(n1), range(n2), range(n3))), dtype=np.float64)
    frac = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return frac @ cell, cell * np.array(reps, dtype=np.float64)[:, None]


def cubic_box(kind, n, a):
    """n x n x n conventional cubic cells of fcc or bcc with lattice constant a."""
    basis = {"fcc": _FCC, "bcc": _BCC}[kind]
    return supercell(np.eye(3) * a, basis, (n, n, n))


# --------------------------------------------------------------------------
# distances (geometry only; used to enforce the minimal distance)
# --------------------------------------------------------------------------

def _shift_vectors(cell, pbc, cutoff):
    if not pbc:
        return np.zeros((1, 3))
    vol = abs(np.linalg.det(cell))
    rng = []
    for k in range(3):
        l, m = (k + 1) % 3, (k + 2) % 3
        spacing = vol / np.linalg.norm(np.cross(cell[l], cell[m]))
        # after reduction to the nearest image a fractional offset is within
        # [-1/2, 1/2], so |t| <= cutoff / spacing + 1/2 covers every image
        n = int(np.ceil(cutoff / spacing + 0.5))
        rng.append(range(-n, n + 1))
    return np.array(list(itertools.product(*rng)), dtype=np.float64) @ cell


def close_pairs(pos, cell, pbc, cutoff):
    """All pairs (i, j), i < j, of distinct atoms with some image closer than
    cutoff.  Brute force for small systems, binning for large periodic ones."""
    N = len(pos)
    if N < 2:
        return np.zeros((0, 2), dtype=np.int64)
    if pbc and N > 4096:
        return _close_pairs_binned(pos, cell, cutoff)
    inv = np.linalg.inv(cell) if pbc else None
    shifts = _shift_vectors(cell, pbc, cutoff)
    iu, ju = np.triu_indices(N, k=1)
    out = []
    step = max(1, 2_000_000 // max(1, len(shifts)))
    for s in range(0, len(iu), step):
        i, j = iu[s:s + step], ju[s:s + step]
        d = pos[j] - pos[i]
        if pbc:
            d = d - np.rint(d @ inv) @ cell
        r2 = np.full(len(i), np.inf)
        for sh in shifts:
            e = d + sh
            r2 = np.minimum(r2, np.einsum("pa,pa->p", e, e))
        close = r2 < cutoff * cutoff
        out.append(np.stack([i[close], j[close]], axis=1))
    return np.concatenate(out).astype(np.int64).reshape(-1, 2)


def _close_pairs_binned(pos, cell, cutoff, subset=None):
    inv = np.linalg.inv(cell)
    frac = (pos @ inv) % 1.0
    vol = abs(np.linalg.det(cell))
    nb = []
    for k in range(3):
        l, m = (k + 1) % 3, (k + 2) % 3
        spacing = vol / np.linalg.norm(np.cross(cell[l], cell[m]))
        nb.append(max(1, int(spacing // cutoff)))
    nb = np.array(nb)
    if np.any(nb < 3):
        raise ValueError("cell too small for binning")
    b3 = np.minimum((frac * nb).astype(np.int64), nb - 1)
    flat = (b3[:, 0] * nb[1] + b3[:, 1]) * nb[2] + b3[:, 2]
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=int(np.prod(nb)))
    occ = counts.max()
    table = -np.ones((int(np.prod(nb)), occ), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    sorted_flat = flat[order]
    rank = np.arange(len(order)) - starts[sorted_flat]
    table[sorted_flat, rank] = order
    pairs = []
    rows = np.arange(len(pos)) if subset is None else np.asarray(subset, dtype=np.int64)
    for off in itertools.product((-1, 0, 1), repeat=3):
        nbin = (b3[rows] + np.array(off)) % nb
        nflat = (nbin[:, 0] * nb[1] + nbin[:, 1]) * nb[2] + nbin[:, 2]
        cand = table[nflat]                                  # [rows, occ]
        i_idx = np.repeat(rows[:, None], occ, axis=1)
        ok = (cand >= 0) & (cand != i_idx)
        ii, jj = np.minimum(i_idx[ok], cand[ok]), np.maximum(i_idx[ok], cand[ok])
        d = pos[jj] - pos[ii]
        d = d - np.rint(d @ inv) @ cell
        close = np.einsum("pa,pa->p", d, d) < cutoff * cutoff
        pairs.append(np.stack([ii[close], jj[close]], axis=1))
    p = np.unique(np.concatenate(pairs), axis=0)
    return p


def min_distance(pos, cell, pbc, probe=6.0):
    """Smallest interatomic distance (over images), or inf if none below probe."""
    pairs = close_pairs(pos, cell, pbc, probe)
    if len(pairs) == 0:
        return np.inf
    inv = np.linalg.inv(cell) if pbc else None
    d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
    if pbc:
        d = d - np.rint(d @ inv) @ cell
        shifts = _shift_vectors(cell, pbc, probe)
        r = np.sqrt(np.min(np.einsum("tpa,tpa->tp", d[None] + shifts[:, None], d[None] + shifts[:, None]), axis=0))
    else:
        r = np.sqrt(np.einsum("pa,pa->p", d, d))
    return float(r.min())


# --------------------------------------------------------------------------
# displacements with a minimal distance
# --------------------------------------------------------------------------

def displace(rng, ideal, cell, pbc, sigma, r_min, max_redraws=100):
    """Gaussian displacements N(0, sigma^2) per Cartesian component.

    Then, while some pair of distinct atoms is closer than r_min, redraw (from
    the same stream, in ascending atom order) the displacement of the higher
    index atom of every such pair; an atom redrawn max_redraws times returns
    to its ideal site and is not moved again (the other atom of a pair is
    redrawn instead).  Returns (pos, n_redraws).
    """
    N = len(ideal)
    disp = rng.normal(0.0, sigma, size=(N, 3))
    count = np.zeros(N, dtype=np.int64)
    frozen = np.zeros(N, dtype=bool)
    total = 0
    pairs = close_pairs(ideal + disp, cell, pbc, r_min)
    while True:
        pos = ideal + disp
        if len(pairs) == 0:
            return pos, total
        movers = set()
        for i, j in pairs:
            movers.add(int(j) if not frozen[j] else int(i))
        for k in sorted(movers):
            if frozen[k]:
                continue
            count[k] += 1
            total += 1
            if count[k] >= max_redraws:
                disp[k] = 0.0
                frozen[k] = True
            else:
                disp[k] = rng.normal(0.0, sigma, size=3)
        # only pairs that touch an atom involved in a close pair can change
        pos = ideal + disp
        touched = np.unique(pairs.ravel())
        pairs = _close_pairs_of(pos, cell, pbc, r_min, touched)


def _close_pairs_of(pos, cell, pbc, cutoff, atoms):
    """Pairs (i, j), i < j, closer than cutoff with i or j in ``atoms``."""
    N = len(pos)
    atoms = np.asarray(atoms, dtype=np.int64)
    if len(atoms) == 0:
        return np.zeros((0, 2), dtype=np.int64)
    if pbc and N > 4096:
        return _close_pairs_binned(pos, cell, cutoff, subset=atoms)
    inv = np.linalg.inv(cell) if pbc else None
    shifts = _shift_vectors(cell, pbc, cutoff)
    d = pos[None, :, :] - pos[atoms][:, None, :]           # [A, N, 3]
    if pbc:
        d = d - np.rint(d @ inv) @ cell
    r2 = np.full(d.shape[:2], np.inf)
    for sh in shifts:
        e = d + sh
        r2 = np.minimum(r2, np.einsum("anx,anx->an", e, e))
    r2[np.arange(len(atoms)), atoms] = np.inf
    a_idx, j_idx = np.nonzero(r2 < cutoff * cutoff)
    i_g = atoms[a_idx]
    p = np.stack([np.minimum(i_g, j_idx), np.maximum(i_g, j_idx)], axis=1)
    return np.unique(p, axis=0).astype(np.int64)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def _batch(cfgs):
    n = np.array([len(c[0]) for c in cfgs], dtype=np.int64)
    return {
        "n_atoms": n,
        "atom_offsets": np.concatenate([[0], np.cumsum(n)]).astype(np.int64),
        "pos": np.concatenate([c[0] for c in cfgs]).astype(np.float64).reshape(-1, 3),
        "species": np.concatenate([c[1] for c in cfgs]).astype(np.int32),
        "cell": np.stack([c[2] for c in cfgs]).astype(np.float64),
        "pbc": np.array([c[3] for c in cfgs], dtype=np.uint8),
    }


def config_of(batch, k):
    """(pos, species, cell, pbc) of configuration k of a batch."""
    a, b = batch["atom_offsets"][k], batch["atom_offsets"][k + 1]
    return batch["pos"][a:b], batch["species"][a:b], batch["cell"][k], bool(batch["pbc"][k])


def subset(batch, idx):
    return _batch([config_of(batch, int(k)) for k in idx])


def fcc108(seed=0, a=4.05, sigma=0.1, r_min=2.0):
    """108-atom periodic fcc box, 3x3x3 cells (one species)."""
    rng = np.random.default_rng(seed)
    ideal, cell = cubic_box("fcc", 3, a)
    pos, _ = displace(rng, ideal, cell, True, sigma, r_min)
    return _batch([(pos, np.zeros(len(pos), np.int32), cell, 1)])


def bcc_alloy(seed=0, n=20, a=3.2, sigma=0.15, r_min=2.0, n_species=2):
    """n^3-cell periodic bcc box with an exact equal split of species."""
    rng = np.random.default_rng(seed)
    ideal, cell = cubic_box("bcc", n, a)
    pos, _ = displace(rng, ideal, cell, True, sigma, r_min)
    N = len(pos)
    sp = np.repeat(np.arange(n_species, dtype=np.int32), -(-N // n_species))[:N]
    sp = sp[rng.permutation(N)]
    return _batch([(pos, sp, cell, 1)])


def fcc_alloy(seed=0, n=40, a=3.6, sigma=0.2, r_min=2.0, n_species=3):
    """n^3-cell periodic disordered fcc alloy, equal species fractions."""
    return _cubic_alloy("fcc", seed, n, a, sigma, r_min, n_species)


def _cubic_alloy(kind, seed, n, a, sigma, r_min, n_species):
    rng = np.random.default_rng(seed)
    ideal, cell = cubic_box(kind, n, a)
    pos, _ = displace(rng, ideal, cell, True, sigma, r_min)
    N = len(pos)
    sp = np.repeat(np.arange(n_species, dtype=np.int32), -(-N // n_species))[:N]
    sp = sp[rng.permutation(N)]
    return _batch([(pos, sp, cell, 1)])


def md_jitter(seed, n_atoms, n_steps, sigma=0.002):
    """Per-step Gaussian jitter for the repeated-evaluation workload."""
    rng = np.random.default_rng(seed)
    for _ in range(n_steps):
        yield rng.normal(0.0, sigma, size=(n_atoms, 3))


def _reps_for(n_sites_cell, n_atoms):
    best = None
    for reps in itertools.product(range(1, 13), repeat=3):
        if not (reps[0] <= reps[1] <= reps[2]):
            continue
        tot = n_sites_cell * reps[0] * reps[1] * reps[2]
        if tot < n_atoms:
            continue
        key = (tot, reps[2] / reps[0])
        if best is None or key < best[0]:
            best = (key, reps)
    return best[1]


def mixed_batch(seed=0, n_configs=4096, n_min=8, n_max=256, n_species_model=3,
                nn_range=(2.6, 3.0), sigma_range=(0.05, 0.3), r_min=2.0):
    """Many small configurations of uneven size: random fcc/bcc/hcp periodic
    cells (vacancies removed at random down to N) and free fragments (the N
    sites nearest a random centre), Gaussian displacements, 1..3 species."""
    rng = np.random.default_rng(seed)
    cfgs = []
    kinds = ("fcc", "bcc", "hcp")
    for _ in range(n_configs):
        N = int(rng.integers(n_min, n_max + 1))
        kind = kinds[int(rng.integers(0, 3))]
        nn = float(rng.uniform(*nn_range))
        periodic = bool(rng.integers(0, 2))
        sigma = float(rng.uniform(*sigma_range))
        ucell, ubasis = unit_cell(kind, nn)
        if periodic:
            reps = _reps_for(len(ubasis), N)
            ideal, cell = supercell(ucell, ubasis, reps)
            keep = np.sort(rng.permutation(len(ideal))[:N])
            ideal = ideal[keep]
        else:
            k = int(np.ceil((4 * N / len(ubasis)) ** (1 / 3))) + 2
            block, bcell = supercell(ucell, ubasis, (k, k, k))
            centre = (np.array([0.5, 0.5, 0.5]) + rng.uniform(-0.5, 0.5, 3) / k) @ bcell
            d = np.linalg.norm(block - centre, axis=1)
            ideal = block[np.sort(np.argsort(d, kind="stable")[:N])]
            ideal = ideal - centre
            cell = np.zeros((3, 3))
        pos, _ = displace(rng, ideal, cell, periodic, sigma, r_min)
        s = int(rng.integers(1, n_species_model + 1))
        present = np.sort(rng.choice(n_species_model, size=s, replace=False))
        sp = rng.choice(present, size=N).astype(np.int32)
        cfgs.append((pos, sp, cell, int(periodic)))
    return _batch(cfgs)


def draw_model(seed, n_mu, n_species, n_q, m, c_sigma=0.1):
    """Uncalibrated parameters: c ~ N(0, c_sigma^2) [n_mu, S, S, N_Q] then
    xi ~ N(0, 1) [m], in that order."""
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, c_sigma, size=(n_mu, n_species, n_species, n_q))
    xi = rng.normal(0.0, 1.0, size=m)
    return c, xi
