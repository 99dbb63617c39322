"""Pins of the oracle's basis enumeration against the paper (section 2.1)."""
import os
import re

import pytest

from oracle import basis as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [l.split() for l in fh if l.strip() and not l.startswith("#")]


def _moment_terms(expr):
    """(mu, nu, power) for every M_{mu,nu}^power in a printed expression."""
    return [(int(a), int(b), int(p) if p else 1)
            for a, b, p in re.findall(r"M_\{(\d+),(\d+)\}(?:\^(\d+))?", expr)]


def test_levels_printed_in_paper():
    rows = _lines("levels.txt")
    assert len(rows) == 10
    for expr, lev in rows:
        got = sum(p * ob.moment_level(mu, nu) for mu, nu, p in _moment_terms(expr))
        assert got == int(lev), expr


def test_printed_contractions_are_basis_members():
    # (M11 . M01), (M12 : M02), ((M03 M02) . M01) are connected contractions
    g1 = (((0, 1), (1, 1)), ((0, 1, 1),))
    g2 = (((0, 2), (1, 2)), ((0, 1, 2),))
    g3 = (((0, 1), (0, 2), (0, 3)), ((0, 2, 1), (1, 2, 2)))
    assert g1 in ob.connected_contractions(10) and ob.graph_level(g1) == 10
    assert g2 in ob.connected_contractions(12) and ob.graph_level(g2) == 12
    assert g3 in ob.connected_contractions(12) and ob.graph_level(g3) == 12
    assert g1 not in ob.connected_contractions(8)


_FACTOR = {
    "M00": (((0, 0),), ()),
    "M10": (((1, 0),), ()),
    "M01.M01": (((0, 1), (0, 1)), ((0, 1, 1),)),
    "M02:M02": (((0, 2), (0, 2)), ((0, 1, 2),)),
}


def test_level8_basis_is_the_papers():
    rows = _lines("basis_lev8.txt")
    want = sorted((int(lev), tuple(sorted(map(str, f.split("*"))))) for _n, lev, f in rows)
    graphs = ob.connected_contractions(8)
    name = {g: k for k, g in _FACTOR.items()}
    got = sorted((ob.basis_function_level([graphs[i] for i in fn]),
                  tuple(sorted(name[graphs[i]] for i in fn))) for fn in ob.basis(8))
    assert got == want
    assert len(ob.basis(8)) == 9


def test_basis_is_closed_and_unique():
    L = 12
    graphs = ob.connected_contractions(L)
    assert len(set(graphs)) == len(graphs)
    for labels, edges in graphs:
        deg = [0] * len(labels)
        for u, v, k in edges:
            assert u != v and k >= 1
            deg[u] += k
            deg[v] += k
        assert deg == [nu for _mu, nu in labels]
        assert ob.graph_level((labels, edges)) <= L
    funcs = ob.basis(L)
    assert len(set(funcs)) == len(funcs)
    # every product of graphs within the level bound is present
    levels = [ob.graph_level(g) for g in graphs]
    for a in range(len(graphs)):
        for b in range(a, len(graphs)):
            if levels[a] + levels[b] <= L:
                assert (a, b) in funcs


def test_levels_are_even_and_monotone_counts():
    prev = 0
    for L in (2, 4, 6, 8, 10, 12):
        n = len(ob.basis(L))
        assert n > prev
        prev = n
        assert len(ob.basis(L + 1)) == n  # an odd bound adds nothing: levels are even


@pytest.mark.slow
def test_counts_level16():
    # regression numbers of this reading (not printed in the paper)
    assert len(ob.connected_contractions(16)) == 41
    assert len(ob.basis(16)) == 116
