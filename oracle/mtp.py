"""Oracle: plain FP64 evaluation of a Moment Tensor Potential (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module.  It shares no code with the HIP product path.  Every tensor is held
as a full 3^nu array and every contraction is an ``np.einsum`` over those
arrays, written straight from the definitions of the paper, section 2.1:

* eq. E_MTP: E(cfg) = sum_i V(n_i).
* eq. V_MTP: V(n_i) = sum_alpha xi_alpha B_alpha(n_i).
* moments:  M_{mu,nu}(n_i) = sum_j f_mu(|r_ij|, z_i, z_j) r_ij^{(x) nu},
  with r_ij pointing from atom i to atom j (an image of j for periodic cells).
* eq. f_mu: f_mu = sum_{beta=1..N_Q} c^{(beta)}_{mu,z_i,z_j} Q^{(beta)}(|r_ij|).
* eq. radial-basis: Q^{(beta)}(r) = phi^{(beta)}(r) (R_cut - r)^2 for
  r < R_cut, else 0.

Readings where the paper is silent:

* phi^{(beta)} = T_{beta-1}(x), Chebyshev polynomials of the first kind of
  x = (2r - R_min - R_cut) / (R_cut - R_min), the affine map of
  [R_min, R_cut] onto [-1, 1] (beta = 1..N_Q, so T_0 .. T_{N_Q-1}).  The
  polynomial is evaluated as written also for r < R_min.
* The neighbourhood of atom i holds every atom j and every periodic image of
  every atom (atom i's own images included) with 0 < |r_ij| < R_cut.
* Forces are F = -dE/dx.  The virial W_ab = dE/d eps_ab for the homogeneous
  strain r -> (I + eps) r; it equals sum over pairs of g_a r_b where
  g = dV_i/dr_ij.  Stress is sigma = W / volume for periodic cells.

The code is dtype-generic so that the loss gradient can be checked by the
complex-step method (complex c and xi flow through unchanged).
"""
from __future__ import annotations

import itertools
import string

import numpy as np

_LETTERS = string.ascii_lowercase + string.ascii_uppercase.replace("Z", "")


# --------------------------------------------------------------------------
# neighbourhoods
# --------------------------------------------------------------------------

def image_shifts(cell, pbc, r_cut):
    """Integer lattice shifts, relative to the nearest image, that can reach
    within r_cut.  Free clusters use only 0."""
    if not pbc:
        return np.zeros((1, 3), dtype=np.int64)
    cell = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(cell))
    ranges = []
    for k in range(3):
        l, m = (k + 1) % 3, (k + 2) % 3
        spacing = vol / np.linalg.norm(np.cross(cell[l], cell[m]))
        # offsets are first reduced to the nearest image (fractional part in
        # [-1/2, 1/2]); an image within r_cut then has |n| <= r_cut/spacing + 1/2
        n = int(np.ceil(r_cut / spacing + 0.5))
        ranges.append(range(-n, n + 1))
    return np.array(list(itertools.product(*ranges)), dtype=np.int64)


def neighbour_pairs(pos, cell, pbc, r_cut, centers):
    """Brute force over all atoms and images.

    Returns (center_slot, j, rvec): for every pair, the position of its
    centre atom in ``centers``, the home index j of the neighbour and the
    vector r_ij = x_j + n.L - x_i.  Pairs are grouped by centre, in order.
    """
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    shifts = image_shifts(cell, pbc, r_cut)
    inv = np.linalg.inv(cell) if pbc else None
    out_c, out_j, out_r = [], [], []
    for slot, i in enumerate(centers):
        d = pos - pos[i]
        if pbc:
            n0 = -np.rint(d @ inv)
            base = d + n0 @ cell
        else:
            n0 = np.zeros_like(d)
            base = d
        r = base[None, :, :] + (shifts @ cell if pbc else np.zeros((1, 3)))[:, None, :]
        dist = np.sqrt(np.einsum("tja,tja->tj", r, r))
        mask = (dist < r_cut) & (dist > 0.0)
        t_idx, j_idx = np.nonzero(mask)
        # keep a deterministic order: by neighbour, then image
        order = np.lexsort((t_idx, j_idx))
        t_idx, j_idx = t_idx[order], j_idx[order]
        out_c.append(np.full(len(j_idx), slot, dtype=np.int64))
        out_j.append(j_idx.astype(np.int64))
        out_r.append(r[t_idx, j_idx])
    if not out_c:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3))
    return np.concatenate(out_c), np.concatenate(out_j), np.concatenate(out_r)


# --------------------------------------------------------------------------
# radial part (eqs. f_mu and radial-basis)
# --------------------------------------------------------------------------

def chebyshev(x, n):
    """T_0..T_{n-1} at x and their x-derivatives, by the three-term recurrence."""
    T = [np.ones_like(x), x]
    dT = [np.zeros_like(x), np.ones_like(x)]
    for k in range(1, n - 1):
        T.append(2.0 * x * T[k] - T[k - 1])
        dT.append(2.0 * T[k] + 2.0 * x * dT[k] - dT[k - 1])
    return np.stack(T[:n], axis=-1), np.stack(dT[:n], axis=-1)


def radial_basis(r, r_min, r_cut, n_q):
    """Q^{(beta)}(r), beta = 1..N_Q, and dQ/dr, shape [..., N_Q]."""
    r = np.asarray(r, dtype=np.float64)
    x = (2.0 * r - r_min - r_cut) / (r_cut - r_min)
    T, dT = chebyshev(x, n_q)
    inside = (r < r_cut)[..., None]
    s = (r_cut - r)[..., None]
    Q = np.where(inside, T * s * s, 0.0)
    dQ = np.where(inside, dT * (2.0 / (r_cut - r_min)) * s * s - 2.0 * T * s, 0.0)
    return Q, dQ


# --------------------------------------------------------------------------
# tensors and contractions
# --------------------------------------------------------------------------

def outer_powers(rvec, nu_max):
    """r^{(x) nu} for nu = 0..nu_max as arrays [P] + [3]*nu."""
    P = rvec.shape[0]
    out = [np.ones(P)]
    for _ in range(nu_max):
        prev = out[-1]
        out.append(prev[..., None] * rvec.reshape((P,) + (1,) * (prev.ndim - 1) + (3,)))
    return out


def _graph_subscripts(graph):
    """Per-vertex index letters: an edge of multiplicity k gives k letters
    shared by its two end vertices."""
    labels, edges = graph
    subs = [[] for _ in labels]
    t = 0
    for u, v, k in edges:
        for _ in range(k):
            ch = _LETTERS[t]
            t += 1
            subs[u].append(ch)
            subs[v].append(ch)
    for lab, s in zip(labels, subs):
        assert len(s) == lab[1], "vertex degree must equal the moment rank"
    return ["".join(s) for s in subs]


def graph_value(graph, M):
    """Value of one connected contraction for a batch of atoms.
    M maps (mu, nu) -> array [A] + [3]*nu."""
    labels, _ = graph
    subs = _graph_subscripts(graph)
    spec = ",".join("Z" + s for s in subs) + "->Z"
    return np.einsum(spec, *[M[l] for l in labels], optimize="greedy")


def graph_value_grad(graph, M, vertex):
    """d(graph value)/d(tensor of one vertex), as a full tensor [A] + [3]*nu
    (the vertex's own tensor left out of the product, its indices left open)."""
    labels, _ = graph
    subs = _graph_subscripts(graph)
    others = [i for i in range(len(labels)) if i != vertex]
    if not others:  # a lone scalar moment
        return np.ones(M[labels[vertex]].shape[0], dtype=M[labels[vertex]].dtype)
    spec = ",".join("Z" + subs[i] for i in others) + "->Z" + subs[vertex]
    return np.einsum(spec, *[M[labels[i]] for i in others], optimize="greedy")


def _contract_all_but(D, rvec, nu, slot):
    """Contract a per-pair tensor D [P]+[3]*nu with r on every axis but one."""
    P = rvec.shape[0]
    Dm = D.reshape(P, 3 ** slot, 3, 3 ** (nu - slot - 1))
    left = outer_powers(rvec, slot)[slot].reshape(P, 3 ** slot)
    right = outer_powers(rvec, nu - slot - 1)[nu - slot - 1].reshape(P, 3 ** (nu - slot - 1))
    return np.einsum("plmr,pl,pr->pm", Dm, left, right)


# --------------------------------------------------------------------------
# evaluation
# --------------------------------------------------------------------------

def _eval_centers(pot, pos, species, cell, pbc, centers, want_grad=True):
    """Site quantities for a list of centre atoms.

    Returns V [A], B [A, m] and, when want_grad, the pair list
    (slot, j, rvec) and the pair gradients g = dV_i/dr_ij [P, 3].
    """
    c = pot["c"]
    xi = pot["xi"]
    r_min, r_cut, n_q = pot["r_min"], pot["r_cut"], pot["n_q"]
    moments = pot["moments"]
    graphs = pot["graphs"]
    funcs = pot["basis"]
    A = len(centers)
    slot, j, rvec, r, f, df = _pair_radial(pot, pos, species, cell, pbc, centers)
    R = outer_powers(rvec, max(nu for _, nu in moments))
    dtype = np.result_type(f, xi)
    M = _moments(pot, slot, f, R, A)
    G = np.stack([graph_value(g, M) for g in graphs], axis=1) if A else np.zeros((0, len(graphs)), dtype)
    B = np.stack([np.prod(G[:, list(fac)], axis=1) for fac in funcs], axis=1)
    V = B @ xi
    if not want_grad:
        return V, B, None
    # dV/dG: product rule over the factors of every basis function
    dVdG = np.zeros_like(G)
    for a, fac in enumerate(funcs):
        for pos_k in range(len(fac)):
            rest = list(fac[:pos_k]) + list(fac[pos_k + 1:])
            dVdG[:, fac[pos_k]] += xi[a] * np.prod(G[:, rest], axis=1)
    # dV/dM as full tensors
    D = {m: np.zeros_like(M[m]) for m in moments}
    for gi, g in enumerate(graphs):
        for v, lab in enumerate(g[0]):
            D[lab] = D[lab] + dVdG[:, gi].reshape((-1,) + (1,) * lab[1]) * graph_value_grad(g, M, v)
    # pair gradients g = dV_i/dr_ij
    P = len(slot)
    grad = np.zeros((P, 3), dtype=dtype)
    rhat = rvec / r[:, None] if P else rvec
    for mu, nu in moments:
        Dp = D[(mu, nu)][slot]                   # [P] + [3]*nu
        radial_term = np.einsum("pk,pk->p", Dp.reshape(P, 3 ** nu), R[nu].reshape(P, 3 ** nu))
        grad = grad + (df[:, mu] * radial_term)[:, None] * rhat
        for s in range(nu):
            grad = grad + f[:, mu][:, None] * _contract_all_but(Dp, rvec, nu, s)
    return V, B, (slot, j, rvec, grad)


def evaluate(pot, pos, species, cell, pbc, chunk=256):
    """E, forces, virial, site energies and descriptors b for one config.

    Returns a dict with
        energy  : E (eq. E_MTP)
        forces  : [N, 3], F = -dE/dx
        virial  : [3, 3], W = dE/deps (symmetric)
        site    : [N], V(n_i)
        B       : [N, m], B_alpha(n_i)
        b       : [m], b_alpha(cfg) = sum_i B_alpha(n_i)  (eq. matrix-B)
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    m = len(pot["basis"])
    dtype = np.result_type(pot["c"], pot["xi"])
    F = np.zeros((N, 3), dtype=dtype)
    W = np.zeros((3, 3), dtype=dtype)
    V = np.zeros(N, dtype=dtype)
    B = np.zeros((N, m), dtype=dtype)
    for start in range(0, N, chunk):
        centers = np.arange(start, min(N, start + chunk))
        v, b, (slot, j, rvec, g) = _eval_centers(pot, pos, species, cell, pbc, centers)
        V[centers] = v
        B[centers] = b
        np.add.at(F, centers[slot], g)
        np.add.at(F, j, -g)
        W = W + np.einsum("pa,pb->ab", g, rvec)
    return {"energy": V.sum(), "forces": F, "virial": W, "site": V, "B": B, "b": B.sum(axis=0)}


def evaluate_sampled(pot, pos, species, cell, pbc, energy_atoms, force_atoms, chunk=64):
    """Site energies for ``energy_atoms`` and exact forces for ``force_atoms``.

    A force on atom k needs dV_i/dr_ik of every atom i that has k as a
    neighbour, so the neighbourhoods of all atoms within R_cut of a force
    atom are evaluated in full.
    """
    pos = np.asarray(pos, dtype=np.float64)
    force_atoms = np.asarray(force_atoms, dtype=np.int64)
    energy_atoms = np.asarray(energy_atoms, dtype=np.int64)
    # atoms that see a force atom = neighbours of the force atoms (symmetric relation)
    _, jn, _ = neighbour_pairs(pos, cell, pbc, pot["r_cut"], force_atoms)
    centers = np.unique(np.concatenate([energy_atoms, force_atoms, jn]))
    site = {}
    Fk = {int(k): np.zeros(3) for k in force_atoms}
    want = set(int(k) for k in force_atoms)
    for start in range(0, len(centers), chunk):
        cs = centers[start:start + chunk]
        v, _b, (slot, j, rvec, g) = _eval_centers(pot, pos, species, cell, pbc, cs)
        for a, i in enumerate(cs):
            site[int(i)] = v[a]
        for p in range(len(slot)):
            i = int(cs[slot[p]])
            if i in want:
                Fk[i] = Fk[i] + g[p]
            jj = int(j[p])
            if jj in want:
                Fk[jj] = Fk[jj] - g[p]
    return (np.array([site[int(i)] for i in energy_atoms]),
            np.array([Fk[int(k)] for k in force_atoms]))


def stress(virial, cell):
    """sigma = W / volume (eV / A^3) for a periodic cell."""
    return np.asarray(virial) / abs(np.linalg.det(np.asarray(cell, dtype=np.float64)))



def _pair_radial(pot, pos, species, cell, pbc, centers):
    """Pairs of the centre atoms with r = |r_ij|, f_mu and df_mu/dr per pair."""
    species = np.asarray(species)
    slot, j, rvec = neighbour_pairs(pos, cell, pbc, pot["r_cut"], centers)
    r = np.sqrt(np.einsum("pa,pa->p", rvec, rvec))
    Q, dQ = radial_basis(r, pot["r_min"], pot["r_cut"], pot["n_q"])
    zi = species[np.asarray(centers, dtype=np.int64)[slot]]
    coef = pot["c"][:, zi, species[j], :]        # [n_mu, P, N_Q]
    f = np.einsum("mpb,pb->pm", coef, Q)
    df = np.einsum("mpb,pb->pm", coef, dQ)
    return slot, j, rvec, r, f, df


def _moments(pot, slot, f, R, A):
    """M_{mu,nu} = sum over a centre's pairs of f_mu r^{(x) nu}."""
    M = {}
    for mu, nu in pot["moments"]:
        acc = np.zeros((A,) + (3,) * nu, dtype=np.result_type(f))
        np.add.at(acc, slot, f[:, mu].reshape((-1,) + (1,) * nu) * R[nu])
        M[(mu, nu)] = acc
    return M


def site_moments(pot, pos, species, cell, pbc, centers):
    """Full moment tensors M_{mu,nu} of the given centre atoms, as a dict
    (mu, nu) -> [A] + [3]*nu (the first stage of the evaluation)."""
    slot, _j, rvec, _r, f, _df = _pair_radial(pot, pos, species, cell, pbc, centers)
    R = outer_powers(rvec, max(nu for _, nu in pot["moments"]))
    return _moments(pot, slot, f, R, len(centers))
