"""MTP basis: moments, connected contractions and basis functions.

The definitions follow the paper, section 2.1: a moment M_{mu,nu} has level
2 + 4 mu + nu (eq. LevelMTD); levels add under products and contractions;
every contraction of moments that yields a scalar is a basis function, and
an MTP of level lev_max holds all of them with level <= lev_max (the nine
functions of eq. MTPbasisLevel8 for lev_max = 8).

A connected contraction is a connected multigraph: one vertex per moment,
vertex degree equal to its rank nu, no self-loops, edge multiplicity k
meaning k contracted index pairs.  A basis function is a product of
connected contractions.  Moments are fully symmetric tensors, so a
contraction depends only on its multigraph up to isomorphism.

Canonical form (shared with the loader in the C++ library): over every
permutation of the vertices, the lexicographically smallest tuple
    (mu_0, nu_0, ..., mu_{n-1}, nu_{n-1}, k_01, k_02, ..., k_{n-2,n-1}).
"""
from __future__ import annotations

import itertools
from functools import lru_cache


def level_of(mu, nu):
    return 2 + 4 * mu + nu


def canonical(labels, adj):
    """labels: list of (mu, nu); adj: dense symmetric multiplicity matrix."""
    n = len(labels)
    best = None
    for perm in itertools.permutations(range(n)):
        key = tuple(x for v in perm for x in labels[v]) + tuple(
            adj[perm[a]][perm[b]] for a in range(n) for b in range(a + 1, n))
        if best is None or key < best:
            best = key
    return best


def decode(key):
    """Canonical key -> (labels, edges) with edges (u, v, k), u < v."""
    n = 0
    while 2 * n + n * (n - 1) // 2 < len(key):
        n += 1
    labels = [(key[2 * v], key[2 * v + 1]) for v in range(n)]
    edges = []
    t = 2 * n
    for a in range(n):
        for b in range(a + 1, n):
            if key[t]:
                edges.append((a, b, key[t]))
            t += 1
    return labels, edges


def key_level(key):
    labels, _ = decode(key)
    return sum(level_of(mu, nu) for mu, nu in labels)


def _multigraphs(deg):
    """Every loopless multigraph with the given degree sequence (as a dense
    multiplicity matrix), each exactly once: the first vertex with open
    degree spreads all of it over later vertices, one multiplicity per
    later vertex, bounded by their open degrees."""
    n = len(deg)
    adj = [[0] * n for _ in range(n)]
    rem = list(deg)

    def spread(a, b, left):
        # give vertex a's remaining `left` edges to vertices b, b+1, ...
        if left == 0:
            yield from rec()
            return
        if b >= n:
            return
        if sum(rem[c] for c in range(b, n)) < left:
            return
        for k in range(min(left, rem[b]), -1, -1):
            rem[b] -= k
            adj[a][b] = adj[b][a] = k
            yield from spread(a, b + 1, left - k)
            rem[b] += k
            adj[a][b] = adj[b][a] = 0

    def rec():
        a = next((v for v in range(n) if rem[v] > 0), None)
        if a is None:
            yield [row[:] for row in adj]
            return
        left = rem[a]
        rem[a] = 0
        yield from spread(a, a + 1, left)
        rem[a] = left

    yield from rec()


def _connected(adj):
    n = len(adj)
    seen, todo = {0}, [0]
    while todo:
        a = todo.pop()
        for b in range(n):
            if adj[a][b] and b not in seen:
                seen.add(b)
                todo.append(b)
    return len(seen) == n


def _label_multisets(types, n, budget):
    """Non-decreasing n-tuples of vertex types whose levels sum to at most
    budget (types sorted by (mu, nu), so a type's level grows with nu within
    one mu and the scan over later types can stop per mu)."""
    lev = [level_of(*t) for t in types]
    cheapest = min(lev)
    out = []

    def rec(start, chosen, total):
        if len(chosen) == n:
            out.append(tuple(chosen))
            return
        left = n - len(chosen) - 1
        for t in range(start, len(types)):
            if total + lev[t] + left * cheapest > budget:
                continue
            chosen.append(types[t])
            rec(t, chosen, total + lev[t])
            chosen.pop()

    rec(0, [], 0)
    return out


@lru_cache(maxsize=None)
def contractions(lev_max):
    """Canonical keys of all connected contractions with level <= lev_max,
    sorted by (level, key)."""
    keys = set()
    for mu in range(lev_max):
        if level_of(mu, 0) <= lev_max:
            keys.add((mu, 0))
    vertex_types = sorted((mu, nu) for mu in range(lev_max) for nu in range(1, lev_max)
                          if level_of(mu, nu) <= lev_max)
    n = 2
    while 4 * n - 2 <= lev_max:      # n vertices need >= n-1 edges: level >= 4n - 2
        for labels in _label_multisets(vertex_types, n, lev_max):
            deg = [nu for _, nu in labels]
            if sum(deg) % 2:
                continue
            for adj in _multigraphs(deg):
                if _connected(adj):
                    keys.add(canonical(list(labels), adj))
        n += 1
    return tuple(sorted(keys, key=lambda k: (key_level(k), k)))


@lru_cache(maxsize=None)
def functions(lev_max):
    """Basis functions as sorted tuples of contraction indices, sorted by
    (level, tuple)."""
    keys = contractions(lev_max)
    lev = [key_level(k) for k in keys]
    out = []
    stack = [((), 0, 0)]
    while stack:
        chosen, start, total = stack.pop()
        if chosen:
            out.append(chosen)
        for g in range(start, len(keys)):
            if total + lev[g] <= lev_max:
                stack.append((chosen + (g,), g, total + lev[g]))
    return tuple(sorted(out, key=lambda f: (sum(lev[g] for g in f), f)))


def moments(lev_max):
    """Sorted (mu, nu) of the moments the basis uses."""
    s = set()
    for k in contractions(lev_max):
        s.update(map(tuple, decode(k)[0]))
    return sorted(s)
