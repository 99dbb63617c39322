"""Tables of the table-driven contraction (host side, no GPU): the per-graph
tries built by the kernel generator must reproduce, by the walk the kernels
make, every connected contraction written as its sum of weighted component
products, and its derivative in each component; every index in the tables
must stay inside the arrays the kernels read."""
import numpy as np
import pytest

from paper_2007_08555_amd import codegen as cg


def walk_value(nodes, coefs, a, b, level, depth, M):
    s = 0.0
    for n in range(a, b):
        k, c0, c1 = nodes[n]
        if level == depth:
            s += coefs[c0] * M[k]
        else:
            s += M[k] * walk_value(nodes, coefs, c0, c1, level + 1, depth, M)
    return s


def walk_reverse(nodes, coefs, a, b, level, depth, P, M, G):
    s = 0.0
    for n in range(a, b):
        k, c0, c1 = nodes[n]
        sub = coefs[c0] if level == depth else walk_reverse(nodes, coefs, c0, c1, level + 1, depth, P * M[k], M, G)
        G[k] += P * sub
        s += M[k] * sub
    return s


@pytest.mark.parametrize("level", [8, 12, 16])
def test_trie_walk_reproduces_terms(level):
    s = cg.Schedule(level)
    nodes, coefs, roots = cg.build_tries(s)
    rng = np.random.default_rng(level)
    M = rng.normal(size=s.C)
    dg = rng.normal(size=len(s.terms))
    G = np.zeros(s.C)
    G_ref = np.zeros(s.C)
    seen = set()
    for depth, lst in roots.items():
        for g, r0, r1 in lst:
            seen.add(g)
            terms = s.terms[g]
            direct = sum(c * np.prod([M[k] for k in idx]) for c, idx in terms)
            assert np.isclose(walk_value(nodes, coefs, r0, r1, 1, depth, M), direct, rtol=1e-12, atol=1e-12)
            walk_reverse(nodes, coefs, r0, r1, 1, depth, dg[g], M, G)
            for c, idx in terms:
                for t in range(len(idx)):
                    rest = idx[:t] + idx[t + 1:]
                    G_ref[idx[t]] += dg[g] * c * np.prod([M[k] for k in rest])
    assert seen == set(range(len(s.terms)))
    assert np.allclose(G, G_ref, rtol=1e-11, atol=1e-11 * np.abs(G_ref).max())


@pytest.mark.parametrize("level", [20, 24])
def test_tables_stay_in_bounds(level):
    s = cg.Schedule(level)
    nodes, coefs, roots = cg.build_tries(s)
    nodes = np.array(nodes)
    assert nodes[:, 0].min() >= 0 and nodes[:, 0].max() < s.C
    n_terms = sum(len(t) for t in s.terms)
    assert len(coefs) == n_terms and all(float(c) == c for c in coefs)
    # every node is reached exactly once from the roots, children ranges
    # inside the node array, leaves at the graph's depth
    reached = np.zeros(len(nodes), int)
    for depth, lst in roots.items():
        for g, r0, r1 in lst:
            assert 0 <= g < len(s.terms) and len(s.terms[g][0][1]) == depth
            stack = [(r0, r1, 1)]
            while stack:
                a, b, lev = stack.pop()
                assert 0 <= a < b <= len(nodes)
                reached[a:b] += 1
                for n in range(a, b):
                    if lev == depth:
                        assert 0 <= nodes[n, 1] < len(coefs)
                    else:
                        stack.append((nodes[n, 1], nodes[n, 2], lev + 1))
    assert (reached == 1).all()
    assert max(len(f) for f in s.funcs) <= 12 and max(roots) <= 6


def test_split_kernel_tables_level20():
    """The split kernels' tables: every root has a share in [0, TABLE_WAVES)
    and the shares' trie sizes are balanced; a node's local slot s >= 0 names
    its own component in its graph's slot list, and the slot lists hold
    distinct components."""
    import re
    src, _meta = cg.generate_table(20)

    def arr(name):
        m = re.search(r"__device__ const int " + name + r"\[\][^=]*= \{([^}]*)\}", src)
        return [int(x) for x in m.group(1).split(",") if x.strip()]

    node = np.array(arr("kNode")).reshape(-1, 4)
    roots = np.array(arr("kRoots")).reshape(-1, 4)
    slot_k = np.array(arr("kSlotK")).reshape(-1, cg.table_slots(20))
    assert cg.table_slots(20, fp64=True) <= cg.table_slots(20) and cg.table_slots(20, fp64=False) <= cg.table_slots(20)
    begin = [int(x) for x in re.search(r"constexpr int b\[\] = \{([^}]*)\}", src).group(1).split(",")]
    load = np.zeros(cg.TABLE_WAVES)
    for d in range(1, len(begin) - 1):
        for g, r0, r1, w in roots[begin[d]:begin[d + 1]]:
            assert 0 <= w < cg.TABLE_WAVES
            ks = [k for k in slot_k[g] if k >= 0]
            assert len(ks) == len(set(ks))
            stack, n = [(r0, r1, 1)], 0
            while stack:
                a, b, level = stack.pop()
                for t in range(a, b):
                    n += 1
                    k, c0, c1, s = node[t]
                    if s >= 0:
                        assert slot_k[g, s] == k
                    else:
                        assert k not in ks
                    if level < d:
                        stack.append((c0, c1, level + 1))
            load[w] += n
    assert load.max() <= 1.05 * load.mean()
