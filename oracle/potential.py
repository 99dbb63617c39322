"""Oracle: reader/writer of the MTP potential text file (test infrastructure).

The file holds the functional form of an MTP (paper, section 2.1: lev_max,
N_Q, R_min, R_cut, the list of basis contractions) and its parameters
theta = {xi, c} (eqs. V_MTP and f_mu).  The product library has its own,
independent parser of the same format.

Format (whitespace separated, '#' starts a comment line):

    mtp355 1
    level <lev_max>
    species_count <S>
    radial_basis_size <N_Q>
    min_dist <R_min>
    max_dist <R_cut>
    moments <n>                 then n lines "mu nu"
    contractions <n>            then n lines
        "<nv> <moment index> x nv <ne> (<u> <v> <k>) x ne"
    basis <m>                   then m lines "<nf> <contraction index> x nf"
    radial_coeffs <n_mu*S*S*N_Q>   values, layout c[mu][z_i][z_j][beta]
    xi <m>                      values
"""
from __future__ import annotations

import numpy as np


def write_potential(path, pot):
    lines = ["mtp355 1",
             f"level {pot['level']}",
             f"species_count {pot['n_species']}",
             f"radial_basis_size {pot['n_q']}",
             f"min_dist {pot['r_min']!r}",
             f"max_dist {pot['r_cut']!r}"]
    moments = pot["moments"]
    lines.append(f"moments {len(moments)}")
    lines += [f"{mu} {nu}" for mu, nu in moments]
    index = {m: i for i, m in enumerate(moments)}
    lines.append(f"contractions {len(pot['graphs'])}")
    for labels, edges in pot["graphs"]:
        parts = [str(len(labels))] + [str(index[l]) for l in labels] + [str(len(edges))]
        for u, v, k in edges:
            parts += [str(u), str(v), str(k)]
        lines.append(" ".join(parts))
    lines.append(f"basis {len(pot['basis'])}")
    lines += [" ".join([str(len(f))] + [str(g) for g in f]) for f in pot["basis"]]
    c = np.asarray(pot["c"], dtype=np.float64).ravel()
    lines.append(f"radial_coeffs {c.size}")
    lines += [repr(float(v)) for v in c]
    xi = np.asarray(pot["xi"], dtype=np.float64).ravel()
    lines.append(f"xi {xi.size}")
    lines += [repr(float(v)) for v in xi]
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def read_potential(path):
    with open(path) as fh:
        toks = [t for line in fh if not line.lstrip().startswith("#") for t in line.split()]
    pos = 0

    def take():
        nonlocal pos
        pos += 1
        return toks[pos - 1]

    def expect(word):
        got = take()
        if got != word:
            raise ValueError(f"{path}: expected '{word}', found '{got}'")

    expect("mtp355")
    if take() != "1":
        raise ValueError(f"{path}: unsupported format version")
    pot = {}
    expect("level"); pot["level"] = int(take())
    expect("species_count"); pot["n_species"] = int(take())
    expect("radial_basis_size"); pot["n_q"] = int(take())
    expect("min_dist"); pot["r_min"] = float(take())
    expect("max_dist"); pot["r_cut"] = float(take())
    expect("moments")
    moments = [(int(take()), int(take())) for _ in range(int(take()))]
    pot["moments"] = moments
    expect("contractions")
    graphs = []
    for _ in range(int(take())):
        nv = int(take())
        labels = tuple(moments[int(take())] for _ in range(nv))
        ne = int(take())
        edges = tuple((int(take()), int(take()), int(take())) for _ in range(ne))
        graphs.append((labels, edges))
    pot["graphs"] = graphs
    expect("basis")
    pot["basis"] = [tuple(int(take()) for _ in range(int(take()))) for _ in range(int(take()))]
    expect("radial_coeffs")
    n_mu = 1 + max(mu for mu, _ in moments)
    nc = int(take())
    if nc != n_mu * pot["n_species"] ** 2 * pot["n_q"]:
        raise ValueError(f"{path}: radial_coeffs count {nc} does not match the moments")
    pot["c"] = np.array([float(take()) for _ in range(nc)]).reshape(
        n_mu, pot["n_species"], pot["n_species"], pot["n_q"])
    expect("xi")
    nx = int(take())
    if nx != len(pot["basis"]):
        raise ValueError(f"{path}: xi count {nx} != basis size {len(pot['basis'])}")
    pot["xi"] = np.array([float(take()) for _ in range(nx)])
    return pot


def n_mu(pot) -> int:
    return 1 + max(mu for mu, _ in pot["moments"])
