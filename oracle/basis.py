"""Oracle: enumeration of the MTP basis (test infrastructure, not the product).

This module is part of the plain FP64 CPU oracle. Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the HIP product
path never does.

What it follows (paper, section 2.1 "Moment Tensor Potential"):

* eq. LevelMTD: a moment M_{mu,nu} has level 2 + 4 mu + nu.
* The level of a product or contraction of moments is the sum of the levels.
* Every contraction of one or more moments that yields a scalar is a basis
  function; the basis holds all of them with level <= lev_max.
* eq. MTPbasisLevel8 lists the nine functions of lev_max = 8.

Reading of the definition (the paper lists only lev_max = 8): a *connected
contraction* is a connected multigraph whose vertices are moments (mu, nu),
where the degree of a vertex equals its rank nu, with no self-loops (a trace
of one moment only re-weights the radial part, which f_mu already spans).
An edge of multiplicity k between two vertices contracts k index pairs of
the two tensors.  Because every moment is a fully symmetric tensor, the value
of a contraction depends only on the multigraph up to a label-preserving
isomorphism.  A basis function is a product (multiset) of one or more
connected contractions.  There is no constant term.  This reproduces the
nine level-8 functions exactly.

Graph encoding used throughout the oracle:
    labels : tuple of (mu, nu) sorted ascending, one per vertex
    edges  : tuple of (u, v, k), u < v, k >= 1 the multiplicity
"""
from __future__ import annotations

import itertools
from functools import lru_cache


def moment_level(mu: int, nu: int) -> int:
    """Level of M_{mu,nu} (eq. LevelMTD)."""
    return 2 + 4 * mu + nu


def graph_level(graph) -> int:
    """Level of a contraction: the sum of the levels of its moments."""
    labels, _ = graph
    return sum(moment_level(mu, nu) for mu, nu in labels)


def basis_function_level(factors) -> int:
    """Level of a product of contractions: levels add."""
    return sum(graph_level(g) for g in factors)


def _is_connected(n, edges) -> bool:
    if n == 1:
        return True
    adj = {i: set() for i in range(n)}
    for u, v, _k in edges:
        adj[u].add(v)
        adj[v].add(u)
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == n


def _canonical(labels, mult) -> tuple:
    """Canonical form of a labelled multigraph.

    labels is sorted; only permutations inside runs of equal labels keep it
    sorted, so the minimum over those permutations of the upper-triangle
    multiplicity tuple is a complete isomorphism invariant.
    """
    n = len(labels)
    groups = []
    start = 0
    for i in range(1, n + 1):
        if i == n or labels[i] != labels[start]:
            groups.append(list(range(start, i)))
            start = i
    best = None
    for parts in itertools.product(*[itertools.permutations(g) for g in groups]):
        perm = [p for part in parts for p in part]  # new position -> old vertex
        key = tuple(mult[perm[a]][perm[b]] for a in range(n) for b in range(a + 1, n))
        if best is None or key < best:
            best = key
    return best


def _graph_from_key(labels, key):
    n = len(labels)
    edges = []
    t = 0
    for a in range(n):
        for b in range(a + 1, n):
            if key[t]:
                edges.append((a, b, key[t]))
            t += 1
    return (tuple(labels), tuple(edges))


def _adjacency_fillings(degrees):
    """All symmetric zero-diagonal non-negative integer matrices with the
    given row sums, yielded as dense lists."""
    n = len(degrees)
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    mult = [[0] * n for _ in range(n)]
    rem = list(degrees)

    def rec(t):
        if t == len(pairs):
            if all(r == 0 for r in rem):
                yield [row[:] for row in mult]
            return
        a, b = pairs[t]
        # once all pairs involving a are assigned, rem[a] must be zero
        last_for_a = all(p[0] != a for p in pairs[t + 1:])
        hi = min(rem[a], rem[b])
        lo = rem[a] if last_for_a else 0
        if lo > hi:
            return
        for k in range(lo, hi + 1):
            mult[a][b] = mult[b][a] = k
            rem[a] -= k
            rem[b] -= k
            yield from rec(t + 1)
            rem[a] += k
            rem[b] += k
        mult[a][b] = mult[b][a] = 0

    yield from rec(0)


@lru_cache(maxsize=None)
def connected_contractions(lev_max: int):
    """All connected contractions with level <= lev_max, each exactly once,
    sorted by (level, labels, edges)."""
    out = set()
    # single vertex: a scalar moment M_{mu,0}
    mu = 0
    while moment_level(mu, 0) <= lev_max:
        out.add((((mu, 0),), ()))
        mu += 1
    # n >= 2 vertices: every vertex has nu >= 1; connected needs at least
    # n - 1 edges, so sum(nu) >= 2(n - 1) and level >= 4n - 2.
    n = 2
    while 4 * n - 2 <= lev_max:
        moments = [(m, v) for m in range(lev_max) for v in range(1, lev_max)
                   if moment_level(m, v) <= lev_max]
        for labels in itertools.combinations_with_replacement(sorted(moments), n):
            lev = sum(moment_level(m, v) for m, v in labels)
            if lev > lev_max:
                continue
            degrees = [v for _m, v in labels]
            if sum(degrees) % 2 or sum(degrees) < 2 * (n - 1):
                continue
            if max(degrees) > sum(degrees) - max(degrees):
                continue  # no self-loops: a vertex cannot out-degree the rest
            for mult in _adjacency_fillings(degrees):
                edges = [(a, b, mult[a][b]) for a in range(n) for b in range(a + 1, n) if mult[a][b]]
                if not _is_connected(n, edges):
                    continue
                out.add(_graph_from_key(labels, _canonical(labels, mult)))
        n += 1
    return tuple(sorted(out, key=lambda g: (graph_level(g), g[0], g[1])))


@lru_cache(maxsize=None)
def basis(lev_max: int):
    """The basis of lev_max: a tuple of basis functions, each a sorted tuple
    of indices into connected_contractions(lev_max) (with repetition for
    powers).  Sorted by (level, factor indices)."""
    graphs = connected_contractions(lev_max)
    levels = [graph_level(g) for g in graphs]
    funcs = []

    def rec(start, chosen, lev):
        if chosen:
            funcs.append(tuple(chosen))
        for gi in range(start, len(graphs)):
            if lev + levels[gi] <= lev_max:
                chosen.append(gi)
                rec(gi, chosen, lev + levels[gi])
                chosen.pop()

    rec(0, [], 0)
    funcs.sort(key=lambda f: (sum(levels[i] for i in f), f))
    return tuple(funcs)


def moments_used(lev_max: int):
    """Sorted list of the (mu, nu) moments that occur in the basis."""
    s = set()
    for labels, _ in connected_contractions(lev_max):
        s.update(labels)
    return sorted(s)
