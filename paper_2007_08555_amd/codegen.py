"""Generates the HIP evaluation kernel of one MTP basis (build step).

For a basis of level lev_max (paper, section 2.1) the generator emits one
straight-line kernel per atom that

1. accumulates the moments M_{mu,nu} over the atom's pairs, held as the
   symmetric components M[a,b,c] (a + b + c = nu; the entry of the full
   tensor at any index tuple with a x's, b y's and c z's),
2. evaluates every connected contraction as a sum of products of those
   components, forms the basis functions B_alpha (products of contractions)
   and V = sum_alpha xi_alpha B_alpha (eq. V_MTP),
3. runs the same straight-line code in reverse to get G = dV/dM, and
4. for every pair forms g = dV/dr_ij from G, f_mu and df_mu/dr, writes it
   for the force gather and accumulates the virial sum g (x) r.

A contraction of symmetric tensors over an edge of multiplicity k sums over
the k contracted index pairs; grouping the index tuples by their counts
(kx, ky, kz) turns it into a sum over compositions of k with weight
k! / (kx! ky! kz!).  A vertex reads the component given by the sum of the
compositions of its incident edges.

All array indices are compile-time constants, so M and G live in registers.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from collections import defaultdict

from . import basis as pb


def components(nu):
    """(a, b, c) with a + b + c = nu in a fixed order."""
    return [(a, b, nu - a - b) for a in range(nu, -1, -1) for b in range(nu - a, -1, -1)]


def multinomial(a, b, c):
    return math.factorial(a + b + c) // (math.factorial(a) * math.factorial(b) * math.factorial(c))


class Schedule:
    """Component layout, contraction terms and basis products of one level."""

    def __init__(self, lev_max):
        self.level = lev_max
        self.keys = list(pb.contractions(lev_max))
        self.funcs = list(pb.functions(lev_max))
        self.moments = pb.moments(lev_max)
        self.n_mu = 1 + max(mu for mu, _ in self.moments)
        self.nu_max = max(nu for _, nu in self.moments)
        self.comp = {}
        for mu, nu in self.moments:
            for abc in components(nu):
                self.comp[(mu, nu, abc)] = len(self.comp)
        self.C = len(self.comp)
        self.graphs = [pb.decode(k) for k in self.keys]
        self.terms = [self._terms(labels, edges) for labels, edges in self.graphs]

    def _terms(self, labels, edges):
        """Sum over the index assignments of a graph as weighted products of
        components: edges are taken one at a time, each spreading its k
        contracted index pairs over the axes (composition (kx, ky, kz) with
        weight k! / (kx! ky! kz!)) and adding them to both endpoints' counts;
        assignments that reach the same per-vertex counts are merged."""
        if not edges:
            (mu, nu), = labels
            return [(1, (self.comp[(mu, 0, (0, 0, 0))],))]
        states = {tuple((0, 0, 0) for _ in labels): 1}
        for u, v, k in edges:
            spread = [(abc, multinomial(*abc)) for abc in components(k)]
            nxt = defaultdict(int)
            for st, coef in states.items():
                for abc, w in spread:
                    cnt = list(st)
                    cnt[u] = tuple(x + y for x, y in zip(cnt[u], abc))
                    cnt[v] = tuple(x + y for x, y in zip(cnt[v], abc))
                    nxt[tuple(cnt)] += coef * w
            states = nxt
        acc = defaultdict(int)
        for cnt, coef in states.items():
            idx = tuple(sorted(self.comp[(mu, nu, cnt[x])] for x, (mu, nu) in enumerate(labels)))
            acc[idx] += coef
        return sorted((c, idx) for idx, c in acc.items())

    # ------------------------------------------------------------------
    def nus_used(self):
        return sorted({nu for _, nu in self.moments})

    def mus_of_nu(self, nu):
        return [mu for mu, n in self.moments if n == nu]

    def metadata(self):
        return {"level": self.level, "m": len(self.funcs), "graphs": len(self.keys),
                "C": self.C, "n_mu": self.n_mu, "nu_max": self.nu_max,
                "terms": sum(len(t) for t in self.terms)}


def _prod(factors):
    return " * ".join(factors) if factors else "T(1)"


def _const(v):
    return f"T({float(v)!r})"


def _mono_steps(s):
    """Per degree nu, the statements defining its monomials from degree nu - 1."""
    steps = {}
    mono = {(0, 0, 0): "T(1)"}
    for nu in range(1, s.nu_max + 1):
        lines = []
        for a, b, c in components(nu):
            if a:
                src, v = (a - 1, b, c), "x"
            elif b:
                src, v = (a, b - 1, c), "y"
            else:
                src, v = (a, b, c - 1), "z"
            name = f"m{a}_{b}_{c}"
            rhs = v if src == (0, 0, 0) else f"{mono[src]} * {v}"
            lines.append((f"const T {name} = {rhs};", src != (0, 0, 0)))
            mono[(a, b, c)] = name
        steps[nu] = lines
    return steps, mono


def emit_pair_forward(s, comp_mode, nus=None, kmap=None):
    """Monomials of the pair vector, degree by degree, each followed by the
    moment components that use it (only two degrees are live at once).
    Restricted to the degrees in nus (all when None); kmap maps a component
    index to its register slot in M."""
    out = []
    ops = 0
    steps, mono = _mono_steps(s)
    by_nu = defaultdict(list)
    for (mu, nu, abc), k in s.comp.items():
        if nus is None or nu in nus:
            by_nu[nu].append((mu, abc, k if kmap is None else kmap[k]))
    top = s.nu_max if nus is None else max(nus)
    for nu in range(0, top + 1):
        for line, counted in steps.get(nu, []):
            out.append(line)
            ops += 1 if counted else 0
        for mu, abc, k in by_nu.get(nu, []):
            term = f"f[{mu}]" if nu == 0 else f"f[{mu}] * {mono[abc]}"
            if comp_mode:
                out.append(f"if constexpr (COMP) mtp::two_sum_acc(M[{k}], Mlo[{k}], {term}); else M[{k}] += {term};")
            else:
                out.append(f"M[{k}] += {term};")
            ops += 2 if nu else 1
    return out, ops


REVERSE_TEMPLATE = r"""
// Reverse sweep, pass {pidx}: G = dV/dM for the components of degrees {nus}
// from the moments they pair with and dV/dg of the graphs they occur in.
template <typename T>
__global__ void __launch_bounds__(BLOCK){attr} contract_rev_{tag}_kernel(const mtp::EvalArgs<T> args) {{
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  T M[C];
{load_m}
{load_dg}
#define MTP_OUT_G(k_, v_) args.G[(size_t)(k_) * args.stride + i] = (v_)
#define MTP_FENCE_M() do {{ {fence} }} while (0)
{body}
#undef MTP_FENCE_M
#undef MTP_OUT_G
}}
"""


TGRAPH_TEMPLATE = r"""
// Loss path, graph pass {pidx}: values and tangents (along dM) of the
// connected graphs {graphs}, from the moments they use.
template <typename R>
__global__ void __launch_bounds__(BLOCK) tgraph_{tag}_kernel(const mtp::EvalArgs<R> args, const mtp::LossArgs<R> la) {{
  using T = mtp::Dual<R>;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  T M[C];
{load_m}
{body}
{store_g}
}}
"""

TBASIS_TEMPLATE = r"""
// Loss path: basis functions, V and dV/dg on dual numbers from the graph
// values and tangents; writes a_k B_alpha + tangent of B_alpha and dV/dg.
template <typename R>
__global__ void __launch_bounds__(BLOCK) tbasis_kernel(const mtp::EvalArgs<R> args, const mtp::LossArgs<R> la) {{
  using T = mtp::Dual<R>;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  const R* __restrict__ xi = args.xi;
  const R aw = la.a_atom[i];
{load_g}
#define MTP_OUT_B(a_, v_) la.xi_terms[(size_t)(a_) * args.stride + i] = aw * (v_).v + (v_).d
{body}
#undef MTP_OUT_B
{store_dg}
  (void)V;
}}
"""

TREV_TEMPLATE = r"""
// Loss path, reverse pass {pidx}: tangent of G = dV/dM for the components of
// degrees {nus}, from the moments they pair with and dV/dg on dual numbers.
template <typename R>
__global__ void __launch_bounds__(BLOCK) trev_{tag}_kernel(const mtp::EvalArgs<R> args, const mtp::LossArgs<R> la) {{
  using T = mtp::Dual<R>;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  T M[C];
{load_m}
{load_dg}
#define MTP_OUT_G(k_, v_) la.dG[(size_t)(k_) * args.stride + i] = (v_).d
#define MTP_FENCE_M() do {{ {fence} }} while (0)
{body}
#undef MTP_FENCE_M
#undef MTP_OUT_G
}}
"""


def graph_groups(s, budget):
    """Connected graphs grouped (in order of their first moment component)
    so that each group reads at most `budget` moment components."""
    sets = [set(k for c, idx in t for k in idx) for t in s.terms]
    order = sorted(range(len(sets)), key=lambda g: (min(sets[g]) if sets[g] else 0, len(sets[g]), g))
    out, cur, used = [], [], set()
    for g in order:
        if cur and len(used | sets[g]) > budget:
            out.append(cur)
            cur, used = [], set()
        cur.append(g)
        used |= sets[g]
    if cur:
        out.append(cur)
    return out


MOMENTS_TEMPLATE = r"""
// Moments pass {pidx}: the components of degrees {nus} of one atom, summed
// over its pairs and written to args.M; {split} thread(s) per atom, each over
// every {split}-th pair, partial sums combined across those lanes.
template <typename T, bool COMP, int NQ, bool PR64>
__device__ __forceinline__ void moments_{tag}_body(const mtp::EvalArgs<T>& args) {{
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* cs = reinterpret_cast<T*>(smem_raw);
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) cs[t + t / args.nq] = args.c[t];
  __syncthreads();
  constexpr int SPLIT = {split};
  const int tid = blockIdx.x * BLOCK + threadIdx.x;
  const int i = tid / SPLIT;
  const int h = tid - i * SPLIT;
  if (i >= args.n_atoms) return;
  const int S = args.n_species;
  const int nq = args.nq;
  // c in LDS with one pad slot after every (z_i, z_j) block of N_Q values, so
  // that lanes of different species pairs read different banks
  const int nqp = nq + 1;
  const int mu_stride = S * S * nqp;
  const int zi = clamp_species(args.species[i], S);
  const int cnt = args.nbr_count[i];
  const T rmin = args.rmin, rcut = args.rcut;
  constexpr int CP = {ncomp};
  constexpr int NMP = {nmu};
  constexpr int kIdx[CP] = {{ {comp_list} }};
  T M[CP];
  T Mlo[COMP ? CP : 1];
#pragma unroll
  for (int k = 0; k < CP; ++k) M[k] = T(0);
#pragma unroll
  for (int k = 0; k < (COMP ? CP : 1); ++k) Mlo[k] = T(0);
  // pair p + SPLIT is loaded while pair p is processed
  T xn = T(0), yn = T(0), zn = T(0), un = T(0), sn = T(0);
  int zjn = 0;
  if (h < cnt) {{
    const mtp::PairVec<T> q = mtp::load_pair<T, PR64>(args, (size_t)h * args.stride + i);
    xn = q.x; yn = q.y; zn = q.z; un = q.u; sn = q.s; zjn = q.zj;
  }}
#pragma unroll 1
  for (int p = h; p < cnt; p += SPLIT) {{
    const T x = xn, y = yn, z = zn, u = un, sc = sn;
    const int zj = zjn;
    if (p + SPLIT < cnt) {{
      const size_t en = (size_t)(p + SPLIT) * args.stride + i;
      const mtp::PairVec<T> q = mtp::load_pair<T, PR64>(args, en);
      xn = q.x; yn = q.y; zn = q.z; un = q.u; sn = q.s; zjn = q.zj;
    }}
    T f[NMP], df[NMP];
    if constexpr (PR64) {{
      // radial arguments formed in FP64 (load_pair)
      mtp::radial_us<T, NMP, false, NQ>(cs, (zi * S + zj) * nqp, mu_stride, nq, u, sc, T(0), f, df);
    }} else {{
      (void)u; (void)sc;
      const T r = sqrt(x * x + y * y + z * z);
      mtp::radial<T, NMP, false, NQ>(cs, (zi * S + zj) * nqp, mu_stride, nq, r, rmin, rcut, f, df);
    }}
{body}
  }}
  if constexpr (COMP) {{
#pragma unroll
    for (int k = 0; k < CP; ++k) M[k] += Mlo[k];
  }}
  if constexpr (SPLIT > 1) {{
    // one component at a time (the empty asm ties each sum to the next
    // component), so that the lane moves of all components are not in
    // flight at once
#pragma unroll
    for (int k = 0; k < CP; ++k) {{
      M[k] = mtp::group_sum<SPLIT>(M[k]);
      if (k + 1 < CP) asm volatile("" : "+v"(M[k]), "+v"(M[k + 1]));
    }}
  }}
  if (h != 0) return;
#pragma unroll
  for (int k = 0; k < CP; ++k) args.M[(size_t)kIdx[k] * args.stride + i] = M[k];
}}

template <typename T, int NQ, bool PR64>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
moments_{tag}_kernel(const mtp::EvalArgs<T> args) {{
  moments_{tag}_body<T, false, NQ, PR64>(args);
}}

// compensated sums hold two registers per component: one wavefront per SIMD
// (the register file of two would spill)
template <typename T, int NQ, bool PR64>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(1)))
moments_{tag}_ckernel(const mtp::EvalArgs<T> args) {{
  moments_{tag}_body<T, true, NQ, PR64>(args);
}}
"""


def emit_contraction(s):
    """Forward contraction, basis values, V, and the reverse sweep into G."""
    out = []
    ops = 0
    # forward: graph values
    for g, terms in enumerate(s.terms):
        out.append(f"T g{g} = T(0);")
        for coef, idx in terms:
            fac = [f"M[{k}]" for k in idx]
            expr = _prod(fac)
            if coef != 1:
                expr = f"{_const(coef)} * {expr}"
            out.append(f"g{g} += {expr};")
            ops += len(idx) + (1 if coef != 1 else 0)
    # basis functions and V
    out.append("T V = T(0);")
    for a, fn in enumerate(s.funcs):
        out.append(f"{{ const T b = {_prod([f'g{g}' for g in fn])}; V += xi[{a}] * b; MTP_OUT_B({a}, b); }}")
        ops += len(fn) - 1 + 2
    # dV/dg
    dg = defaultdict(list)
    for a, fn in enumerate(s.funcs):
        counts = defaultdict(int)
        for g in fn:
            counts[g] += 1
        for g, n in counts.items():
            rest = list(fn)
            rest.remove(g)
            expr = _prod([f"g{h}" for h in rest])
            if n > 1:
                expr = f"T({float(n)!r}) * {expr}"
            dg[g].append(f"xi[{a}] * {expr}")
            ops += len(rest) + 1 + (1 if n > 1 else 0)
    for g in range(len(s.terms)):
        out.append(f"const T dg{g} = " + (" + ".join(dg[g]) if dg[g] else "T(0)") + ";")
    # keep the products of the forward sweep from being reused (and held in
    # registers) by the reverse sweep: M is reloaded (or made opaque to the
    # optimiser) here, so that it is dead while B, V and dV/dg are formed
    out.append("MTP_RELOAD_M();")
    # reverse of the graph terms, gathered per component so that each
    # G[k] is complete when written and nothing but M stays live
    contrib = defaultdict(lambda: defaultdict(list))
    for g, terms in enumerate(s.terms):
        for coef, idx in terms:
            for k in set(idx):
                cnt = idx.count(k)
                rest = list(idx)
                rest.remove(k)
                contrib[k][g].append((coef * cnt, rest))
    for k in range(s.C):
        if not contrib[k]:
            out.append(f"MTP_OUT_G({k}, T(0));")
            continue
        parts = []
        for g, lst in sorted(contrib[k].items()):
            inner = []
            for c, rest in lst:
                expr = _prod([f"M[{q}]" for q in rest])
                if c != 1:
                    expr = f"{_const(c)} * {expr}" if rest else _const(c)
                    ops += 1
                inner.append(expr)
                ops += max(len(rest) - 1, 0) + 1
            parts.append(f"dg{g} * (" + " + ".join(inner) + ")")
            ops += 1
        out.append(f"MTP_OUT_G({k}, " + " + ".join(parts) + ");")
        # one fence per component keeps each G[k]'s products from being
        # interleaved with the next ones (FP64 then needs no scratch)
        out.append("mtp::opaque(M);")
    return out, ops


def emit_reverse_pass(s, ks):
    """Reverse sweep restricted to the components ks: G[k] = sum over graph
    terms holding M[k] of dV/dg times the product of the other factors.
    Returns the lines and the sets of M components and graphs it reads."""
    contrib = defaultdict(lambda: defaultdict(list))
    for g, terms in enumerate(s.terms):
        for coef, idx in terms:
            for k in set(idx):
                cnt = idx.count(k)
                rest = list(idx)
                rest.remove(k)
                contrib[k][g].append((coef * cnt, rest))
    out, m_used, g_used = [], set(), set()
    for k in ks:
        if not contrib[k]:
            out.append(f"MTP_OUT_G({k}, T(0));")
            continue
        parts = []
        for g, lst in sorted(contrib[k].items()):
            g_used.add(g)
            inner = []
            for c, rest in lst:
                m_used.update(rest)
                expr = _prod([f"M[{q}]" for q in rest])
                if c != 1:
                    expr = f"{_const(c)} * {expr}" if rest else _const(c)
                inner.append(expr)
            parts.append(f"dg{g} * (" + " + ".join(inner) + ")")
        out.append(f"MTP_OUT_G({k}, " + " + ".join(parts) + ");")
        out.append("MTP_FENCE_M();")
    return out, sorted(m_used), sorted(g_used)


def emit_pair_backward(s, nus=None, gmap=None, nmu=None):
    """g = dV/dr_ij for one pair from G, f, df and the monomials, restricted
    to the components of the degrees in nus (all when None); gmap maps a
    component index to its register slot in G.

    G[k] is the derivative with respect to the component itself, a plain sum
    over pairs of f_mu x^a y^b z^c, so d/dr of one pair's share is
    df_mu x^a y^b z^c r/|r| + f_mu grad(x^a y^b z^c)."""
    out = []
    ops = 0
    steps, mono = _mono_steps(s)
    nm = "NMU" if nmu is None else str(nmu)
    out.append(f"T D[{nm}];")
    out.append(f"#pragma unroll\nfor (int q = 0; q < {nm}; ++q) D[q] = T(0);")
    out.append("T gx = T(0), gy = T(0), gz = T(0);")
    used = set(s.nus_used()) if nus is None else set(nus)
    gmap = gmap or {k: k for k in range(s.C)}
    top = max(used)
    for nu in range(0, top + 1):
        for line, counted in steps.get(nu, []):
            out.append(line)
            ops += 1 if counted else 0
        if nu not in used:
            continue
        mus = s.mus_of_nu(nu)
        for a, b, c in components(nu):
            ks = [gmap[s.comp[(mu, nu, (a, b, c))]] for mu in mus]
            if nu == 0:
                for mu, k in zip(mus, ks):
                    out.append(f"D[{mu}] += G[{k}];")
                    ops += 1
                continue
            out.append("{")
            mono_abc = mono[(a, b, c)]
            for mu, k in zip(mus, ks):
                out.append(f"D[{mu}] += G[{k}] * {mono_abc};")
                ops += 2
            out.append("const T h = " + " + ".join(f"f[{mu}] * G[{k}]" for mu, k in zip(mus, ks)) + ";")
            ops += 2 * len(ks) - 1
            for axis, e, src in (("gx", a, (a - 1, b, c)), ("gy", b, (a, b - 1, c)), ("gz", c, (a, b, c - 1))):
                if e:
                    lower = mono[src]
                    fac = "h" if e == 1 else f"{_const(e)} * h"
                    out.append(f"{axis} += {fac} * {lower};" if lower != "T(1)" else f"{axis} += {fac};")
                    ops += 2 + (1 if e != 1 else 0)
            out.append("}")
    out.append("T rad = T(0);")
    out.append(f"#pragma unroll\nfor (int q = 0; q < {nm}; ++q) rad += df[q] * D[q];")
    out.append("const T ri = rad * inv_r;")
    out.append("gx += ri * x; gy += ri * y; gz += ri * z;")
    ops += 2 * s.n_mu + 1 + 6
    return out, ops


def _nu_bits(nus):
    return sum(1 << n for n in nus)


def _adjoint_launches(tags_nus, split):
    """Launch lines of the adjoint passes [(tag, degrees)]: a preamble that
    finds the last pass the caller needs (nu_need, a bit mask of degrees: the
    later passes would only add zeros) and the degrees nu_run of the passes
    that run, then the launches.  The final pass of the split sums the
    per-atom virial and own force itself; when an earlier pass is the last
    that runs, those sums follow as a kernel of their own (in the earlier
    passes they would spill)."""
    n = len(tags_nus)
    pre = [f"constexpr unsigned kAdjNu[{n}] = {{ {', '.join(f'{_nu_bits(nus)}u' for _, nus in tags_nus)} }};",
           f"int last_adj = {n - 1};",
           "while (last_adj > 0 && !(nu_need & kAdjNu[last_adj])) --last_adj;",
           "unsigned nu_run = 0;",
           "for (int k = 0; k <= last_adj; ++k) nu_run |= kAdjNu[k];",
           "(void)nu_run;"]
    grid = _grid(split)
    adj = []
    for k, (tag, _) in enumerate(tags_nus):
        first = "true" if k == 0 else "false"
        if k == n - 1:
            adj.append(f"if (last_adj == {k}) hipLaunchKernelGGL((adjoint_{tag}_kernel<T, {first}, true, NQ>), "
                       f"{grid}, dim3(BLOCK), smem, s, args);")
        else:
            adj.append(f"if (last_adj >= {k}) hipLaunchKernelGGL((adjoint_{tag}_kernel<T, {first}, false, NQ>), "
                       f"{grid}, dim3(BLOCK), smem, s, args);")
            adj.append(f"if (last_adj == {k}) hipLaunchKernelGGL((mtp::adjoint_sums_kernel<T>), "
                       "dim3((args.n_atoms + 255) / 256), dim3(256), 0, s, args);")
    return pre, adj


def _grid(split):
    """Launch grid of a per-pair pass with `split` threads per atom."""
    return "grid" if split == 1 else f"dim3((args.n_atoms * {split} + BLOCK - 1) / BLOCK)"


def adjoint_passes(s, budget):
    """Degrees grouped into passes of at most `budget` components (a degree
    is never split); one pass when everything fits."""
    per_nu = defaultdict(list)
    for (mu, nu, abc), k in s.comp.items():
        per_nu[nu].append(k)
    passes, cur, n = [], [], 0
    for nu in sorted(per_nu):
        if cur and n + len(per_nu[nu]) > budget:
            passes.append(cur)
            cur, n = [], 0
        cur.append(nu)
        n += len(per_nu[nu])
    passes.append(cur)
    return [(p, sorted(k for nu in p for k in per_nu[nu])) for p in passes]


FUSED_TEMPLATE = r"""
// Moments, contractions and reverse sweep of one atom in one kernel: all C
// moment components summed in registers over the atom's pairs (and written
// out only when STORE_M, for the loss and normal-equation paths that reread
// them), then the graph values, B, V, dV/dg and G = dV/dM (written out for
// the adjoint passes).  Up to 512 registers per lane (VGPRs and AGPRs), one
// wavefront per SIMD.
template <typename T, bool WANT_B, bool STORE_M, int NQ>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(1, 1)))
fused_{tag}_kernel(const mtp::EvalArgs<T> args) {{
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* cs = reinterpret_cast<T*>(smem_raw);
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) cs[t + t / args.nq] = args.c[t];
  __syncthreads();
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  const int S = args.n_species;
  const int nq = args.nq;
  // c in LDS with one pad slot after every (z_i, z_j) block of N_Q values, so
  // that lanes of different species pairs read different banks
  const int nqp = nq + 1;
  const int mu_stride = S * S * nqp;
  const int zi = clamp_species(args.species[i], S);
  const int cnt = args.nbr_count[i];
  const T rmin = args.rmin, rcut = args.rcut;
  constexpr bool COMP = false;
  T M[C];
  T Mlo[1];
  (void)Mlo;
#pragma unroll
  for (int k = 0; k < C; ++k) M[k] = T(0);
  T xn = T(0), yn = T(0), zn = T(0);
  int zjn = 0;
  if (cnt > 0) {{
    const mtp::PairRec<T> q = args.pr[i];
    xn = q.x; yn = q.y; zn = q.z; zjn = q.zj;
  }}
#pragma unroll 1
  for (int p = 0; p < cnt; ++p) {{
    const T x = xn, y = yn, z = zn;
    const int zj = zjn;
    if (p + 1 < cnt) {{
      const size_t en = (size_t)(p + 1) * args.stride + i;
      const mtp::PairRec<T> q = args.pr[en];
      xn = q.x; yn = q.y; zn = q.z; zjn = q.zj;
    }}
    const T r = sqrt(x * x + y * y + z * z);
    T f[NMU], df[NMU];
    mtp::radial<T, NMU, false, NQ>(cs, (zi * S + zj) * nqp, mu_stride, nq, r, rmin, rcut, f, df);
{moments}
  }}
  if constexpr (STORE_M) {{
#pragma unroll
    for (int k = 0; k < C; ++k) args.M[(size_t)k * args.stride + i] = M[k];
  }}
  const T* __restrict__ xi = args.xi;
#define MTP_OUT_B(a_, v_) do {{ if (WANT_B) args.B[(size_t)(a_) * args.b_stride + i] = (v_); }} while (0)
#define MTP_OUT_G(k_, v_) args.G[(size_t)(k_) * args.stride + i] = (v_)
#define MTP_RELOAD_M() mtp::opaque(M)
{contraction}
#undef MTP_RELOAD_M
#undef MTP_OUT_G
#undef MTP_OUT_B
  args.site[i] = V;
}}
"""


ADJOINT_TEMPLATE = r"""
// Adjoint pass {pidx} over the pairs of one atom, components of degrees {nus}:
// its share of g = dV_i/dr_ij from G, f_mu and df_mu/dr, stored (first pass)
// or added (later passes) per pair for the force and virial gather; the
// last pass also sums the atom's own share of its force, sum_p g_p, in FP64,
// so that the gather only has to fetch the reverse pairs' g.  {split}
// thread(s) per atom, each over every {split}-th pair (the per-atom sums are
// combined across those lanes).
template <typename T, bool FIRST, bool LAST, int NQ>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
adjoint_{tag}_kernel(const mtp::EvalArgs<T> args) {{
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* cs = reinterpret_cast<T*>(smem_raw);
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) cs[t + t / args.nq] = args.c[t];
  __syncthreads();
  constexpr int SPLIT = {split};
  const int tid = blockIdx.x * BLOCK + threadIdx.x;
  const int i = tid / SPLIT;
  const int h = tid - i * SPLIT;
  if (i >= args.n_atoms) return;
  const int S = args.n_species;
  const int nq = args.nq;
  // c in LDS with one pad slot after every (z_i, z_j) block of N_Q values, so
  // that lanes of different species pairs read different banks
  const int nqp = nq + 1;
  const int mu_stride = S * S * nqp;
  const int zi = clamp_species(args.species[i], S);
  const int cnt = args.nbr_count[i];
  const T rmin = args.rmin, rcut = args.rcut;
  constexpr int CP = {ncomp};
  constexpr int kIdx[CP] = {{ {comp_list} }};
  T G[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) G[k] = args.G[(size_t)kIdx[k] * args.stride + i];
  // the last pass also sums the per-atom virial sum_p g_p (x) r_p and sum_p g_p
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  T w0 = T(0), w1 = T(0), w2 = T(0), w3 = T(0), w4 = T(0), w5 = T(0), w6 = T(0), w7 = T(0), w8 = T(0);
  // pair p + SPLIT (and its partial g) is loaded while pair p is processed
  T xn = T(0), yn = T(0), zn = T(0), g0n = T(0), g1n = T(0), g2n = T(0);
  int zjn = 0;
  if (h < cnt) {{
    const size_t e0 = (size_t)h * args.stride + i;
    const mtp::PairRec<T> q = args.pr[e0];
    xn = q.x; yn = q.y; zn = q.z; zjn = q.zj;
    if (!FIRST) {{ g0n = args.g[3 * e0]; g1n = args.g[3 * e0 + 1]; g2n = args.g[3 * e0 + 2]; }}
  }}
#pragma unroll 1
  for (int p = h; p < cnt; p += SPLIT) {{
    const size_t e = (size_t)p * args.stride + i;
    const T x = xn, y = yn, z = zn;
    const int zj = zjn;
    const T gp0 = g0n, gp1 = g1n, gp2 = g2n;
    if (p + SPLIT < cnt) {{
      const size_t en = e + (size_t)SPLIT * args.stride;
      const mtp::PairRec<T> q = args.pr[en];
      xn = q.x; yn = q.y; zn = q.z; zjn = q.zj;
      if (!FIRST) {{ g0n = args.g[3 * en]; g1n = args.g[3 * en + 1]; g2n = args.g[3 * en + 2]; }}
    }}
    const T r = sqrt(x * x + y * y + z * z);
    const T inv_r = T(1) / r;
    T f[{nmu}], df[{nmu}];
    mtp::radial<T, {nmu}, true, NQ>(cs, (zi * S + zj) * nqp, mu_stride, nq, r, rmin, rcut, f, df);
{body}
    const T tx = FIRST ? gx : gp0 + gx, ty = FIRST ? gy : gp1 + gy, tz = FIRST ? gz : gp2 + gz;
    args.g[3 * e] = tx;
    args.g[3 * e + 1] = ty;
    args.g[3 * e + 2] = tz;
    if constexpr (LAST) {{
      w0 += tx * x; w1 += tx * y; w2 += tx * z;
      w3 += ty * x; w4 += ty * y; w5 += ty * z;
      w6 += tz * x; w7 += tz * y; w8 += tz * z;
      o0 += (double)tx; o1 += (double)ty; o2 += (double)tz;
    }}
  }}
  if constexpr (LAST && SPLIT > 1) {{
    w0 = mtp::group_sum<SPLIT>(w0); w1 = mtp::group_sum<SPLIT>(w1); w2 = mtp::group_sum<SPLIT>(w2);
    w3 = mtp::group_sum<SPLIT>(w3); w4 = mtp::group_sum<SPLIT>(w4); w5 = mtp::group_sum<SPLIT>(w5);
    w6 = mtp::group_sum<SPLIT>(w6); w7 = mtp::group_sum<SPLIT>(w7); w8 = mtp::group_sum<SPLIT>(w8);
    o0 = mtp::group_sum<SPLIT>(o0); o1 = mtp::group_sum<SPLIT>(o1); o2 = mtp::group_sum<SPLIT>(o2);
  }}
  if (LAST && h == 0) {{
    T* wv = args.atom_virial + i;
    const size_t st = args.stride;
    wv[0] = w0; wv[st] = w1; wv[2 * st] = w2; wv[3 * st] = w3; wv[4 * st] = w4;
    wv[5 * st] = w5; wv[6 * st] = w6; wv[7 * st] = w7; wv[8 * st] = w8;
    double* ow = args.own + i;
    ow[0] = o0; ow[st] = o1; ow[2 * st] = o2;
  }}
}}
"""


def _dual_mono_steps(s, top):
    """Statements defining monomials m and their tangents dm along (dx, dy, dz)
    for degrees 1..top, grouped by degree."""
    steps = {}
    mono = {(0, 0, 0): ("T(1)", "T(0)")}
    for nu in range(1, top + 1):
        lines = []
        for a, b, c in components(nu):
            if a:
                src, v, dv = (a - 1, b, c), "x", "dx"
            elif b:
                src, v, dv = (a, b - 1, c), "y", "dy"
            else:
                src, v, dv = (a, b, c - 1), "z", "dz"
            m, dm = f"m{a}_{b}_{c}", f"dm{a}_{b}_{c}"
            if src == (0, 0, 0):
                lines.append(f"const T {m} = {v}; const T {dm} = {dv};")
            else:
                ms, dms = mono[src]
                lines.append(f"const T {m} = {ms} * {v}; const T {dm} = {dms} * {v} + {ms} * {dv};")
            mono[(a, b, c)] = (m, dm)
        steps[nu] = lines
    return steps, mono


def emit_tangent_moments(s, nus, gmap):
    """dM_k += df_mu (r.dr / r) m_k + f_mu dm_k for the components of degrees nus."""
    out = []
    top = max(nus)
    steps, mono = _dual_mono_steps(s, top)
    out.append("const T rdot = (x * dx + y * dy + z * dz) * inv_r;")
    for nu in range(0, top + 1):
        out += steps.get(nu, [])
        if nu not in nus:
            continue
        for mu in s.mus_of_nu(nu):
            for abc in components(nu):
                j = gmap[s.comp[(mu, nu, abc)]]
                if nu == 0:
                    out.append(f"DM[{j}] += df[{mu}] * rdot;")
                else:
                    m, dm = mono[abc]
                    out.append(f"DM[{j}] += df[{mu}] * rdot * {m} + f[{mu}] * {dm};")
    return out


def emit_cgrad_pass(s, nus, gmap):
    """Per pair: s1_mu += H m, s2_mu += G m, s3_mu += G dm over the components of
    degrees nus (H = a G + dG)."""
    out = []
    top = max(nus)
    steps, mono = _dual_mono_steps(s, top)
    out.append("const T rdot = (x * dx + y * dy + z * dz) * inv_r;")
    out.append("T s1[NMU], s2[NMU], s3[NMU];")
    out.append("#pragma unroll\nfor (int q = 0; q < NMU; ++q) { s1[q] = T(0); s2[q] = T(0); s3[q] = T(0); }")
    for nu in range(0, top + 1):
        out += steps.get(nu, [])
        if nu not in nus:
            continue
        for mu in s.mus_of_nu(nu):
            for abc in components(nu):
                j = gmap[s.comp[(mu, nu, abc)]]
                if nu == 0:
                    out.append(f"s1[{mu}] += H[{j}]; s2[{mu}] += G[{j}];")
                else:
                    m, dm = mono[abc]
                    out.append(f"s1[{mu}] += H[{j}] * {m}; s2[{mu}] += G[{j}] * {m}; s3[{mu}] += G[{j}] * {dm};")
    return out


def pass_mus(s, nus):
    return sorted({mu for mu, nu in s.moments if nu in nus})


LOSS_PASS_HEAD = r"""
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* cs = reinterpret_cast<T*>(smem_raw);
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) cs[t + t / args.nq] = args.c[t];
  __syncthreads();
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  const int S = args.n_species;
  const int nq = args.nq;
  // c in LDS with one pad slot after every (z_i, z_j) block of N_Q values, so
  // that lanes of different species pairs read different banks
  const int nqp = nq + 1;
  const int mu_stride = S * S * nqp;
  const int zi = clamp_species(args.species[i], S);
  const int cnt = args.nbr_count[i];
  const T rmin = args.rmin, rcut = args.rcut;
  const size_t n = args.stride;
  const T ux = la.u[3 * (size_t)i], uy = la.u[3 * (size_t)i + 1], uz = la.u[3 * (size_t)i + 2];
  const T e00 = la.eps_atom[0 * n + i], e01 = la.eps_atom[1 * n + i], e02 = la.eps_atom[2 * n + i];
  const T e10 = la.eps_atom[3 * n + i], e11 = la.eps_atom[4 * n + i], e12 = la.eps_atom[5 * n + i];
  const T e20 = la.eps_atom[6 * n + i], e21 = la.eps_atom[7 * n + i], e22 = la.eps_atom[8 * n + i];
"""

LOSS_PAIR_HEAD = r"""
    const size_t e = (size_t)p * args.stride + i;
    const mtp::PairRec<T> q = args.pr[e];
    const T x = q.x, y = q.y, z = q.z;
    const int zj = q.zj;
    const int j = la.nbr[(size_t)p * args.stride + i];
    // delta r_ij = u_j - u_i + eps r_ij
    const T dx = la.u[3 * (size_t)j] - ux + (e00 * x + e01 * y + e02 * z);
    const T dy = la.u[3 * (size_t)j + 1] - uy + (e10 * x + e11 * y + e12 * z);
    const T dz = la.u[3 * (size_t)j + 2] - uz + (e20 * x + e21 * y + e22 * z);
    const T r = sqrt(x * x + y * y + z * z);
    const T inv_r = T(1) / r;
    T f[NMU], df[NMU];
    mtp::radial<T, NMU, true>(cs, (zi * S + zj) * nqp, mu_stride, nq, r, rmin, rcut, f, df);
"""


def emit_loss_kernels(s, budget):
    """Sources of the loss-gradient kernels and the body of their launcher."""
    src, launch = [], []
    passes = adjoint_passes(s, budget)
    ind = lambda lines, k: "\n".join(" " * k + l for l in lines)
    for pidx, (nus, comps) in enumerate(passes):
        gmap = {k: j for j, k in enumerate(comps)}
        body = emit_tangent_moments(s, nus, gmap)
        src.append(f"""
// Tangent of the moments of degrees {nus} along delta r (loss gradient).
template <typename T>
__global__ void __launch_bounds__(BLOCK) tmom_p{pidx}_kernel(const mtp::EvalArgs<T> args, const mtp::LossArgs<T> la) {{{LOSS_PASS_HEAD}
  constexpr int CP = {len(comps)};
  constexpr int kIdx[CP] = {{ {", ".join(map(str, comps))} }};
  T DM[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) DM[k] = T(0);
#pragma unroll 1
  for (int p = 0; p < cnt; ++p) {{{LOSS_PAIR_HEAD}
{ind(body, 4)}
  }}
#pragma unroll
  for (int k = 0; k < CP; ++k) la.dM[(size_t)kIdx[k] * args.stride + i] = DM[k];
}}
""")
        launch.append(f"  hipLaunchKernelGGL((tmom_p{pidx}_kernel<T>), grid, dim3(BLOCK), smem, s, args, la);")
    launch.append("  hipLaunchKernelGGL((tangent_contract_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);")
    for pidx, (nus, comps) in enumerate(passes):
        gmap = {k: j for j, k in enumerate(comps)}
        body = emit_cgrad_pass(s, nus, gmap)
        mus = pass_mus(s, nus)
        if pidx == 0:
            store = "\n".join(f"    la.pa[(size_t){mu} * n_slots + e] = {'s1[%d] + s3[%d]' % (mu, mu) if mu in mus else 'T(0)'};\n"
                              f"    la.pb[(size_t){mu} * n_slots + e] = {'s2[%d] * rdot' % mu if mu in mus else 'T(0)'};"
                              for mu in range(s.n_mu))
        else:
            store = "\n".join(f"    la.pa[(size_t){mu} * n_slots + e] += s1[{mu}] + s3[{mu}];\n"
                              f"    la.pb[(size_t){mu} * n_slots + e] += s2[{mu}] * rdot;" for mu in mus)
        src.append(f"""
// Radial sensitivities of the pairs from the components of degrees {nus}:
// coefficients of Q_beta and dQ_beta/dr in dL/dc (loss gradient).
template <typename T>
__global__ void __launch_bounds__(BLOCK) cgrad_p{pidx}_kernel(const mtp::EvalArgs<T> args, const mtp::LossArgs<T> la) {{{LOSS_PASS_HEAD}
  const T aw = la.a_atom[i];
  const size_t n_slots = (size_t)la.K * args.stride;
  constexpr int CP = {len(comps)};
  constexpr int kIdx[CP] = {{ {", ".join(map(str, comps))} }};
  T G[CP], H[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) {{
    G[k] = args.G[(size_t)kIdx[k] * args.stride + i];
    H[k] = aw * G[k] + la.dG[(size_t)kIdx[k] * args.stride + i];
  }}
#pragma unroll 1
  for (int p = 0; p < cnt; ++p) {{{LOSS_PAIR_HEAD}
{ind(body, 4)}
{store}
  }}
}}
""")
        launch.append(f"  hipLaunchKernelGGL((cgrad_p{pidx}_kernel<T>), grid, dim3(BLOCK), smem, s, args, la);")
    launch.append("  hipLaunchKernelGGL((creduce_kernel<T>), grid, dim3(BLOCK * kCredSplit), "
                  "creduce_smem(args.n_c, args.nq), s, args, la);")
    # the gradient in the positions (when la.hvp is given): the tangent of the
    # pair gradients along delta r, on dual numbers (twice the registers of
    # the adjoint: passes of at most 40 components)
    import re as _re
    launch.append("  if (la.hvp) {")
    for pidx, (nus, comps) in enumerate(adjoint_passes(s, 40)):
        gmap = {k: j for j, k in enumerate(comps)}
        nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
        body, _ = emit_pair_backward(s, nus=nus, gmap=gmap, nmu=nmu)
        body = [_re.sub(r"\bT\b", "DT", l) for l in body]
        src.append(TADJ_TEMPLATE.format(
            pidx=pidx, nus=nus, head=LOSS_PASS_HEAD, ncomp=len(comps), comp_list=", ".join(map(str, comps)),
            nmu=nmu, body=ind(body, 4), store=TADJ_FIRST if pidx == 0 else TADJ_ADD))
        launch.append(f"    hipLaunchKernelGGL((tadj_p{pidx}_kernel<T>), grid, dim3(BLOCK), smem, s, args, la);")
    launch.append("  }")
    return "\n".join(src), "\n".join(launch)


TADJ_TEMPLATE = r"""
// Loss gradient in the positions, pass {pidx} (components of degrees {nus}):
// per pair, the tangent along delta r of this pass's share of g = dV_i/dr_ij
// (G with its tangent dG from the loss path, the pair vector with tangent
// delta r, in dual numbers), stored (first pass, with eps^T g) or added to
// la.hvp.
template <typename T>
__global__ void __launch_bounds__(BLOCK) tadj_p{pidx}_kernel(const mtp::EvalArgs<T> args, const mtp::LossArgs<T> la) {{{head}
  using DT = mtp::Dual<T>;
  constexpr int CP = {ncomp};
  constexpr int kIdx[CP] = {{ {comp_list} }};
  DT G[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k)
    G[k] = DT(args.G[(size_t)kIdx[k] * args.stride + i], la.dG[(size_t)kIdx[k] * args.stride + i]);
#pragma unroll 1
  for (int p = 0; p < cnt; ++p) {{
    const size_t e = (size_t)p * args.stride + i;
    const mtp::PairRec<T> q = args.pr[e];
    const int zj = q.zj;
    const int j = la.nbr[e];
    // delta r_ij = u_j - u_i + eps r_ij
    const T dx = la.u[3 * (size_t)j] - ux + (e00 * q.x + e01 * q.y + e02 * q.z);
    const T dy = la.u[3 * (size_t)j + 1] - uy + (e10 * q.x + e11 * q.y + e12 * q.z);
    const T dz = la.u[3 * (size_t)j + 2] - uz + (e20 * q.x + e21 * q.y + e22 * q.z);
    const DT x = DT(q.x, dx), y = DT(q.y, dy), z = DT(q.z, dz);
    const DT r = mtp::dsqrt(x * x + y * y + z * z);
    const DT inv_r = DT(T(1)) / r;
    DT f[{nmu}], df[{nmu}];
    mtp::radial<DT, {nmu}, true, 0, T>(cs, (zi * S + zj) * nqp, mu_stride, nq, r, DT(rmin), DT(rcut), f, df);
{body}
    T cx = gx.d, cy = gy.d, cz = gz.d;
{store}
  }}
}}
"""

TADJ_FIRST = r"""    {{
      // the stress term's explicit dependence on r_ij: eps^T g
      const T g0 = args.g[3 * e], g1 = args.g[3 * e + 1], g2 = args.g[3 * e + 2];
      cx += e00 * g0 + e10 * g1 + e20 * g2;
      cy += e01 * g0 + e11 * g1 + e21 * g2;
      cz += e02 * g0 + e12 * g1 + e22 * g2;
    }}
    la.hvp[3 * e] = cx;
    la.hvp[3 * e + 1] = cy;
    la.hvp[3 * e + 2] = cz;""".replace("{{", "{").replace("}}", "}")

TADJ_ADD = r"""    la.hvp[3 * e] += cx;
    la.hvp[3 * e + 1] += cy;
    la.hvp[3 * e + 2] += cz;"""


CREDUCE_TEMPLATE = r"""
// dL/dc[mu][z_i][z_j][beta] = sum over pairs of species (z_i, z_j) of
// pa_mu Q_beta(r) + pb_mu dQ_beta/dr.  Four lanes per atom, each over every
// fourth pair in order, for one z_j at a time; the four partial sums are
// combined by DPP quad moves, then per workgroup in a fixed order (for each
// entry, the atoms of that z_i in atom order: bitwise repeatable), then per
// workgroup (BLOCK atoms) to cpart.  LDS: creduce_smem.
constexpr int kCredSplit = 4;
template <typename T>
__global__ void __launch_bounds__(BLOCK * kCredSplit) creduce_kernel(const mtp::EvalArgs<T> args,
                                                                     const mtp::LossArgs<T> la) {{
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int S = args.n_species;
  const int nq = args.nq;
  double* acc_blk = reinterpret_cast<double*>(smem_raw);
  double* tile = acc_blk + args.n_c;
  int* zt = reinterpret_cast<int*>(tile + (size_t)NMU * nq * BLOCK);
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) acc_blk[t] = 0.0;
  const int a = threadIdx.x / kCredSplit, h = threadIdx.x % kCredSplit;
  const int i = blockIdx.x * BLOCK + a;
  const size_t n_slots = (size_t)la.K * args.stride;
  const bool active = i < args.n_atoms;
  const int zi = active ? clamp_species(args.species[i], S) : -1;
  const int cnt = active ? args.nbr_count[i] : 0;
  if (h == 0) zt[a] = zi;
  const T span_inv = T(1) / (args.rcut - args.rmin);
  for (int zj = 0; zj < S; ++zj) {{
    T acc[NMU][16];
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu)
#pragma unroll
      for (int b = 0; b < 16; ++b) acc[mu][b] = T(0);
    for (int p = h; p < cnt; p += kCredSplit) {{
      const size_t e = (size_t)p * args.stride + i;
      const mtp::PairRec<T> pq = args.pr[e];
      if (pq.zj != zj) continue;
      const T x = pq.x, y = pq.y, z = pq.z;
      const T r = sqrt(x * x + y * y + z * z);
      const T q = (T(2) * r - args.rmin - args.rcut) * span_inv;
      const T dqdr = T(2) * span_inv;
      const T sc = args.rcut - r;
      T pa[NMU], pb[NMU];
#pragma unroll
      for (int mu = 0; mu < NMU; ++mu) {{
        pa[mu] = la.pa[(size_t)mu * n_slots + e];
        pb[mu] = la.pb[(size_t)mu * n_slots + e];
      }}
      T t0 = T(1), t1 = q, d0 = T(0), d1 = T(1);
#pragma unroll
      for (int b = 0; b < 16; ++b) {{
        if (b < nq) {{
          const T tb = b == 0 ? t0 : t1;
          const T db = b == 0 ? d0 : d1;
          const T Qb = tb * sc * sc;
          const T dQb = db * dqdr * sc * sc - T(2) * tb * sc;
#pragma unroll
          for (int mu = 0; mu < NMU; ++mu) acc[mu][b] += pa[mu] * Qb + pb[mu] * dQb;
          if (b >= 1) {{
            const T t2 = T(2) * q * t1 - t0;
            const T d2 = T(2) * t1 + T(2) * q * d1 - d0;
            t0 = t1; t1 = t2; d0 = d1; d1 = d2;
          }}
        }}
      }}
    }}
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu)
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (b < nq) {{
          const double v = mtp::group_sum<kCredSplit>((double)acc[mu][b]);
          if (h == 0) tile[(size_t)(mu * nq + b) * BLOCK + a] = v;
        }}
    __syncthreads();
    for (int t = threadIdx.x; t < NMU * S * nq; t += blockDim.x) {{
      const int b = t % nq, zz = (t / nq) % S, mu = t / (nq * S);
      const double* row = tile + (size_t)(mu * nq + b) * BLOCK;
      double v = 0.0;
      for (int l = 0; l < BLOCK; ++l) v += zt[l] == zz ? row[l] : 0.0;
      acc_blk[((mu * S + zz) * S + zj) * nq + b] += v;
    }}
    __syncthreads();
  }}
  for (int t = threadIdx.x; t < args.n_c; t += blockDim.x) la.cpart[(size_t)blockIdx.x * args.n_c + t] = acc_blk[t];
}}

// LDS bytes of creduce_kernel
inline size_t creduce_smem(int n_c, int nq) {{
  return (size_t)(n_c + NMU * nq * BLOCK) * sizeof(double) + BLOCK * sizeof(int);
}}
"""


KERNEL_TEMPLATE = r"""// Generated by paper_2007_08555_amd/codegen.py for the MTP basis of level {level}
// ({m} basis functions, {ngraphs} connected contractions, {C} moment components).
// Do not edit: regenerate with the package build step.
#include "mtp_device.h"
#include "mtp_variant.h"

namespace {{
namespace {ns} {{

constexpr int C = {C};
constexpr int NMU = {n_mu};
constexpr int BLOCK = {block};

__device__ __forceinline__ int clamp_species(int z, int S) {{ return z < 0 ? 0 : (z >= S ? S - 1 : z); }}

#if MTP_PART == 1 || MTP_PART == 2
{moments_kernels}
// Forward contractions of one atom's moments: graph values, V, optional B,
// and dV/dg of every connected graph g (to args.D).
template <typename T, bool WANT_B>
__global__ void __launch_bounds__(BLOCK) contract_fwd_kernel(const mtp::EvalArgs<T> args) {{
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= args.n_atoms) return;
  const T* __restrict__ xi = args.xi;
  T M[C];
  if (args.M32) {{   // mixed precision: FP32 moments, widened
#pragma unroll
    for (int k = 0; k < C; ++k) M[k] = static_cast<T>(args.M32[(size_t)k * args.stride + i]);
  }} else {{
#pragma unroll
    for (int k = 0; k < C; ++k) M[k] = args.M[(size_t)k * args.stride + i];
  }}
#define MTP_OUT_B(a_, v_) do {{ if (WANT_B) args.B[(size_t)(a_) * args.b_stride + i] = (v_); }} while (0)
{contraction_fwd}
#undef MTP_OUT_B
{store_dg}
  args.site[i] = V;
}}

#endif  // parts 1, 2

#if MTP_PART == 3
{loss_kernels}
{creduce}

template <typename T>
hipError_t launch_loss_t(const void* a, const void* l, hipStream_t s) {{
  const auto& args = *static_cast<const mtp::EvalArgs<T>*>(a);
  const auto& la = *static_cast<const mtp::LossArgs<T>*>(l);
  if (args.n_atoms <= 0) return hipSuccess;
  const dim3 grid((args.n_atoms + BLOCK - 1) / BLOCK);
  const size_t smem = (size_t)(args.n_c + args.n_c / args.nq) * sizeof(T);   // c, padded
{launch_loss}
  return hipGetLastError();
}}
#endif  // part 3

#if MTP_PART == 1 || MTP_PART == 2
template <typename T, bool COMP, bool WANT_B, int NQ, bool PR64 = false>
hipError_t launch_t(const void* a, unsigned flags, int schedule, hipStream_t s) {{
  const auto& args = *static_cast<const mtp::EvalArgs<T>*>(a);
  const bool reuse_moments = (flags & mtp::kEvalReuseMoments) != 0;
  const bool store_moments = (flags & mtp::kEvalStoreMoments) != 0;
  const bool moments_only = (flags & mtp::kEvalMomentsOnly) != 0;
  // degrees whose adjoint the caller needs (all unless kEvalNuMask)
  const unsigned nu_need = (flags & mtp::kEvalNuMask) ? (flags >> mtp::kEvalNuShift) : ~0u;
  (void)store_moments;
  (void)moments_only;
  if (args.n_atoms <= 0) return hipSuccess;
  const dim3 grid((args.n_atoms + BLOCK - 1) / BLOCK);
  const size_t smem = (size_t)(args.n_c + args.n_c / args.nq) * sizeof(T);   // c, padded
#if MTP_PART == 1
{launch_body64}
#else
{launch_body32}
#endif
  return hipGetLastError();
}}
#endif  // parts 1, 2

}}  // namespace {ns}
}}  // namespace

// Entry points of the parts (compiled as separate translation units).
namespace mtp_gen_{ns} {{
hipError_t eval64(unsigned flags, int schedule, const void* a, hipStream_t s);
hipError_t eval32(int precision, unsigned flags, int schedule, const void* a, hipStream_t s);
hipError_t loss(int precision, const void* a, const void* l, hipStream_t s);
#if MTP_PART == 1
hipError_t eval64(unsigned flags, int schedule, const void* a, hipStream_t s) {{
  using namespace {ns};
  const bool want_b = (flags & mtp::kEvalWantB) != 0;
  // the pair kernels come with the radial basis size 8 fixed (unrolled) and
  // with a run-time size
  if (static_cast<const mtp::EvalArgs<double>*>(a)->nq == 8)
    return want_b ? launch_t<double, false, true, 8>(a, flags, schedule, s)
                  : launch_t<double, false, false, 8>(a, flags, schedule, s);
  return want_b ? launch_t<double, false, true, 0>(a, flags, schedule, s)
                : launch_t<double, false, false, 0>(a, flags, schedule, s);
}}
#elif MTP_PART == 2
hipError_t eval32(int precision, unsigned flags, int schedule, const void* a, hipStream_t s) {{
  using namespace {ns};
  const bool want_b = (flags & mtp::kEvalWantB) != 0;
  if (precision == 3)   // mixed precision: FP32 moments from the FP64 pair records
    return (flags & mtp::kEvalMomentsOnly) ? launch_t<float, false, false, 0, true>(a, flags, schedule, s)
                                           : hipErrorInvalidValue;
  if (static_cast<const mtp::EvalArgs<float>*>(a)->nq == 8) {{
    if (precision == 2)
      return want_b ? launch_t<float, true, true, 8>(a, flags, schedule, s)
                    : launch_t<float, true, false, 8>(a, flags, schedule, s);
    return want_b ? launch_t<float, false, true, 8>(a, flags, schedule, s)
                  : launch_t<float, false, false, 8>(a, flags, schedule, s);
  }}
  if (precision == 2)
    return want_b ? launch_t<float, true, true, 0>(a, flags, schedule, s) : launch_t<float, true, false, 0>(a, flags, schedule, s);
  return want_b ? launch_t<float, false, true, 0>(a, flags, schedule, s) : launch_t<float, false, false, 0>(a, flags, schedule, s);
}}
#elif MTP_PART == 3
hipError_t loss(int precision, const void* a, const void* l, hipStream_t s) {{
  using namespace {ns};
  return precision == 0 ? launch_loss_t<double>(a, l, s) : launch_loss_t<float>(a, l, s);
}}
#endif
}}  // namespace mtp_gen_{ns}

#if MTP_PART == 0
namespace {{
namespace {ns} {{
hipError_t launch(int precision, unsigned flags, int schedule, const void* a, hipStream_t s) {{
  if (precision == 0) return mtp_gen_{ns}::eval64(flags, schedule, a, s);
  if (precision >= 1 && precision <= 3) return mtp_gen_{ns}::eval32(precision, flags, schedule, a, s);
  return hipErrorInvalidValue;
}}

hipError_t launch_loss(int precision, const void* a, const void* l, hipStream_t s) {{
  return mtp_gen_{ns}::loss(precision, a, l, s);
}}

const int kMoments[] = {{ {moments} }};
const int kGraphKeyOffsets[] = {{ {graph_offsets} }};
const int kGraphKeys[] = {{ {graph_keys} }};
const int kFuncOffsets[] = {{ {func_offsets} }};
const int kFuncFactors[] = {{ {func_factors} }};

}}  // namespace {ns}
}}  // namespace

// The table entry holds a host function pointer, so it exists only in the
// host compilation pass.
#if !defined(__HIP_DEVICE_COMPILE__)
extern const mtp::BasisVariant {ns}_variant = {{
  "{ns}", {level}, {n_moments}, {ns}::kMoments, {ngraphs}, {ns}::kGraphKeyOffsets, {ns}::kGraphKeys,
  {m}, {ns}::kFuncOffsets, {ns}::kFuncFactors, {C}, {n_mu}, {nu_max},
  {flops_pair_fwd}, {flops_pair_bwd}, {flops_atom}, {ns}::launch, {ns}::launch_loss, {ns}::BLOCK, {n_sched} }};
#endif
#endif  // part 0
"""


# FP64 schedules: how the per-atom work is cut into passes that fit the
# register file (moments and adjoint: components per pass; reverse sweep:
# degree groups).  Fewer passes recompute less per pair; more passes need
# fewer registers per wavefront and so run more wavefronts per SIMD.  The
# library times them on the caller's batch (mtp_autotune) and keeps the
# fastest; schedule 0 is the default.
SCHEDULES_F64 = [
    {"mom": 85, "rev": [(0, 1, 2), (3, 4), (5, 6)], "adj": 90},
    {"mom": 85, "rev": [(0, 1), (2,), (3, 4), (5, 6)], "adj": 90},
    {"mom": 50, "rev": [(0,), (1,), (2,), (3,), (4,), (5,), (6,)], "adj": 50},
    # moments, contractions and reverse sweep in one kernel (M, dV/dg never
    # leave the registers), then the adjoint passes
    {"fused": True, "adj": 90},
    # schedule 0 with two and four threads per atom in the moments and adjoint
    # passes (each over every second / fourth pair): more wavefronts in flight
    {"mom": 85, "rev": [(0, 1, 2), (3, 4), (5, 6)], "adj": 90, "split": 2},
    {"mom": 85, "rev": [(0, 1, 2), (3, 4), (5, 6)], "adj": 90, "split": 4},
    # the fused schedule with two threads per atom in its adjoint passes
    {"fused": True, "adj": 90, "split": 2},
]
SCHEDULE_F32 = {"mom": 10 ** 9, "rev": [tuple(range(64))], "adj": 10 ** 9}


def generate(lev_max, block=64):
    s = Schedule(lev_max)
    ns = f"lev{lev_max}"
    fwd, ops_f = emit_pair_forward(s, comp_mode=True)
    # moments passes: FP64 accumulators of all 130 components of level 16 do
    # not fit the register file next to the pair's temporaries, so FP64 sums
    # the degrees in two groups (each pass recomputes r and f_mu)
    comp_nu = {k: nu for (mu, nu, abc), k in s.comp.items()}
    con, ops_c = emit_contraction(s)
    bwd, ops_b = emit_pair_backward(s)
    loss_src, loss_launch = emit_loss_kernels(s, budget=45)
    kern_src, sched_launch = {"f32": [], "f64": []}, {}
    plans = [("f32", 0, SCHEDULE_F32)] + [("f64", k, sch) for k, sch in enumerate(SCHEDULES_F64)]
    for prec, sidx, sch in plans:
        mom_lines, rev_lines, adj_lines = [], [], []
        if sch.get("fused"):
            tag = f"{prec}s{sidx}"
            kern_src[prec].append(FUSED_TEMPLATE.format(
                tag=tag, moments="\n".join(" " * 4 + l for l in fwd), contraction="\n".join("  " + l for l in con)))
            passes = adjoint_passes(s, sch["adj"])
            for pidx, (nus, comps) in enumerate(passes):
                ptag = f"{prec}s{sidx}_p{pidx}"
                gmap = {k: j for j, k in enumerate(comps)}
                nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
                body, _ = emit_pair_backward(s, nus=nus, gmap=gmap, nmu=nmu)
                kern_src[prec].append(ADJOINT_TEMPLATE.format(split=sch.get("split", 1), pidx=pidx, nus=nus, tag=ptag, ncomp=len(comps), nmu=nmu,
                                                              comp_list=", ".join(map(str, comps)),
                                                              body="\n".join(" " * 4 + l for l in body)))
            pre, adj_lines = _adjoint_launches([(f"{prec}s{sidx}_p{pidx}", nus) for pidx, (nus, _) in enumerate(passes)],
                                               sch.get("split", 1))
            # the reread of stored moments (normal equations) runs the
            # contraction of schedule 0 from them
            rev0 = [l for l in sched_launch[(prec, 0)] if "hipLaunchKernelGGL((contract_rev_" in l]
            body = (["if (moments_only) return hipErrorInvalidValue;   // the moments stay in registers"] + pre +
                    ["if (reuse_moments) {",
                     "  hipLaunchKernelGGL((contract_fwd_kernel<T, WANT_B>), grid, dim3(BLOCK), 0, s, args);"] +
                    ["  " + l for l in rev0] +
                    ["} else if (store_moments) {",
                     f"  hipLaunchKernelGGL((fused_{tag}_kernel<T, WANT_B, true, NQ>), grid, dim3(BLOCK), smem, s, args);",
                     "} else {",
                     f"  hipLaunchKernelGGL((fused_{tag}_kernel<T, WANT_B, false, NQ>), grid, dim3(BLOCK), smem, s, args);",
                     "}"] + adj_lines)
            sched_launch[(prec, sidx)] = body
            continue
        # moments passes: each recomputes r and f_mu for the degrees it sums
        for pidx, (nus, comps) in enumerate(adjoint_passes(s, sch["mom"])):
            tag = f"{prec}s{sidx}_p{pidx}"
            kmap = {k: j for j, k in enumerate(comps)}
            body, _ = emit_pair_forward(s, comp_mode=True, nus=set(nus), kmap=kmap)
            nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
            kern_src[prec].append(MOMENTS_TEMPLATE.format(split=sch.get("split", 1), pidx=pidx, nus=nus, tag=tag, ncomp=len(comps), nmu=nmu,
                                                    comp_list=", ".join(map(str, comps)),
                                                    body="\n".join(" " * 4 + l for l in body)))
            # (the moments passes measured no faster with the unrolled radial basis)
            mom_lines.append(_moments_launch(tag, sch.get('split', 1)))
        # reverse sweep passes by degree groups: each pass holds only the
        # moments and dV/dg its components need
        groups = [tuple(n for n in grp if n <= s.nu_max) for grp in sch["rev"]]
        groups = [grp for grp in groups if any(comp_nu[k] in grp for k in range(s.C))]
        covered = {n for grp in groups for n in grp}
        groups += [(n,) for n in sorted(set(comp_nu.values()) - covered)]   # higher levels: one pass per degree
        for pidx, grp in enumerate(groups):
            tag = f"{prec}s{sidx}_p{pidx}"
            ks = [k for k in range(s.C) if comp_nu[k] in grp]
            body, m_used, g_used = emit_reverse_pass(s, ks)
            kern_src[prec].append(REVERSE_TEMPLATE.format(
                pidx=pidx, nus=list(grp), tag=tag,
                # FP64 passes: two wavefronts per SIMD (a pass just above 256
                # registers spills a few words rather than halving occupancy)
                attr=" __attribute__((amdgpu_waves_per_eu(2)))" if prec == "f64" else "",
                load_m="\n".join(["  if (args.M32) {  // mixed precision: FP32 moments, widened"] +
                                 [f"    M[{q}] = static_cast<T>(args.M32[(size_t){q} * args.stride + i]);" for q in m_used] +
                                 ["  } else {"] +
                                 [f"    M[{q}] = args.M[(size_t){q} * args.stride + i];" for q in m_used] + ["  }"]),
                load_dg="\n".join(f"  const T dg{g} = args.D[(size_t){g} * args.stride + i];" for g in g_used),
                fence=" ".join(f'asm volatile("" : "+v"(M[{q}]));' for q in m_used),
                body="\n".join("  " + l for l in body)))
            rev_lines.append(f"if (nu_run & {_nu_bits(grp)}u) "
                             f"hipLaunchKernelGGL((contract_rev_{tag}_kernel<T>), grid, dim3(BLOCK), 0, s, args);")
        # adjoint passes
        passes = adjoint_passes(s, sch["adj"])
        for pidx, (nus, comps) in enumerate(passes):
            tag = f"{prec}s{sidx}_p{pidx}"
            gmap = {k: j for j, k in enumerate(comps)}
            nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
            body, _ = emit_pair_backward(s, nus=nus, gmap=gmap, nmu=nmu)
            import re as _re
            used = {int(v) for line in body for v in _re.findall(r"G\[(\d+)\]", line)}
            assert used <= set(range(len(comps))), "adjoint pass reads a component outside its range"
            kern_src[prec].append(ADJOINT_TEMPLATE.format(split=sch.get("split", 1), pidx=pidx, nus=nus, tag=tag, ncomp=len(comps), nmu=nmu,
                                                    comp_list=", ".join(map(str, comps)),
                                                    body="\n".join(" " * 4 + l for l in body)))
        pre, adj_lines = _adjoint_launches([(f"{prec}s{sidx}_p{pidx}", nus) for pidx, (nus, _) in enumerate(passes)],
                                           sch.get("split", 1))
        body = (["if (!reuse_moments) {"] + ["  " + l for l in mom_lines] + ["}"] +
                ["if (moments_only) return hipGetLastError();"] + pre +
                ["hipLaunchKernelGGL((contract_fwd_kernel<T, WANT_B>), grid, dim3(BLOCK), 0, s, args);"] +
                rev_lines + adj_lines)
        sched_launch[(prec, sidx)] = body
    # loss path: the contraction on dual numbers, split into graph passes,
    # the basis step and reverse passes (dual values need twice the registers)
    fwd_lines = con[:con.index("MTP_RELOAD_M();")]
    vpos = fwd_lines.index("T V = T(0);")
    basis_lines = fwd_lines[vpos:]
    ng = len(s.terms)
    tgraph_budget, trev_groups = 40, [(n,) for n in range(s.nu_max + 1)]
    tkern, tlaunch = [], []
    for pidx, graphs in enumerate(graph_groups(s, tgraph_budget)):
        tag = f"p{pidx}"
        body, m_used = [], set()
        for g in graphs:
            body.append(f"T g{g} = T(0);")
            for coef, idx in s.terms[g]:
                m_used.update(idx)
                expr = _prod([f"M[{k}]" for k in idx])
                if coef != 1:
                    expr = f"{_const(coef)} * {expr}"
                body.append(f"g{g} += {expr};")
        tkern.append(TGRAPH_TEMPLATE.format(
            pidx=pidx, graphs=graphs, tag=tag,
            load_m="\n".join(f"  M[{q}] = T(args.M[(size_t){q} * args.stride + i], la.dM[(size_t){q} * args.stride + i]);"
                             for q in sorted(m_used)),
            body="\n".join("  " + l for l in body),
            store_g="\n".join(f"  la.gd[(size_t){g} * args.stride + i] = g{g}.v; "
                               f"la.gd[(size_t){ng + g} * args.stride + i] = g{g}.d;" for g in graphs)))
        tlaunch.append(f"  hipLaunchKernelGGL((tgraph_{tag}_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);")
    tkern.append(TBASIS_TEMPLATE.format(
        load_g="\n".join(f"  const T g{g}(la.gd[(size_t){g} * args.stride + i], la.gd[(size_t){ng + g} * args.stride + i]);"
                         for g in range(ng)),
        body="\n".join("  " + l for l in basis_lines),
        store_dg="\n".join(f"  la.gd[(size_t){g} * args.stride + i] = dg{g}.v; "
                            f"la.gd[(size_t){ng + g} * args.stride + i] = dg{g}.d;" for g in range(ng))))
    tlaunch.append("  hipLaunchKernelGGL((tbasis_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);")
    for pidx, grp in enumerate(trev_groups):
        ks = [k for k in range(s.C) if comp_nu[k] in grp]
        if not ks:
            continue
        tag = f"p{pidx}"
        body, m_used, g_used = emit_reverse_pass(s, ks)
        tkern.append(TREV_TEMPLATE.format(
            pidx=pidx, nus=list(grp), tag=tag,
            load_m="\n".join(f"  M[{q}] = T(args.M[(size_t){q} * args.stride + i], la.dM[(size_t){q} * args.stride + i]);"
                             for q in m_used),
            load_dg="\n".join(f"  const T dg{g}(la.gd[(size_t){g} * args.stride + i], la.gd[(size_t){ng + g} * args.stride + i]);"
                              for g in g_used),
            fence=" ".join(f'asm volatile("" : "+v"(M[{q}].v), "+v"(M[{q}].d));' for q in m_used),
            body="\n".join("  " + l for l in body)))
        tlaunch.append(f"  hipLaunchKernelGGL((trev_{tag}_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);")
    old_launch = "  hipLaunchKernelGGL((tangent_contract_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);"
    assert old_launch in loss_launch
    loss_launch = loss_launch.replace(old_launch, "\n".join(tlaunch))
    loss_src = loss_src + "\n" + "\n".join(tkern)
    f64_cases = []
    for k in range(len(SCHEDULES_F64)):
        f64_cases.append(f"    case {k}: {{")
        f64_cases += ["      " + l for l in sched_launch[("f64", k)]]
        f64_cases.append("    } break;")
    launch_body64 = "\n".join(["  switch (schedule) {"] + f64_cases +
                               ["    default: return hipErrorInvalidValue;", "  }"])
    launch_body32 = "\n".join(["  if (schedule != 0) return hipErrorInvalidValue;"] +
                               ["  " + l for l in sched_launch[("f32", 0)]])
    # radial work per pair: distance 6, Chebyshev 3 per term, f_mu 2 per (mu, beta),
    # derivative pass adds dT and df
    nq = 8
    rad_f = 6 + 3 * (nq - 2) + 2 * s.n_mu * nq + 2 * s.n_mu
    rad_b = rad_f + 5 * (nq - 2) + 2 * s.n_mu * nq + 4 * s.n_mu + 2
    flops_pair_fwd = ops_f + rad_f
    flops_pair_bwd = ops_b + rad_b + 1
    graph_keys, graph_offsets = [], [0]
    for k in s.keys:
        graph_keys += list(k)
        graph_offsets.append(len(graph_keys))
    func_factors, func_offsets = [], [0]
    for f in s.funcs:
        func_factors += list(f)
        func_offsets.append(len(func_factors))
    ind = lambda lines, n: "\n".join(" " * n + l for l in lines)
    src = KERNEL_TEMPLATE.format(
        level=lev_max, m=len(s.funcs), ngraphs=len(s.keys), C=s.C, n_mu=s.n_mu, nu_max=s.nu_max,
        block=block, ns=ns,
        moments_kernels="\n".join(["#if MTP_PART == 1"] + kern_src["f64"] + ["#else"] + kern_src["f32"] + ["#endif"]),
        launch_body64=launch_body64, launch_body32=launch_body32,
        contraction=ind(con, 2),
        contraction_fwd=ind(con[:con.index("MTP_RELOAD_M();")], 2),
        contract_rev_kernels="",
        store_dg=ind([f"args.D[(size_t){g} * args.stride + i] = dg{g};" for g in range(len(s.terms))], 2),
        adjoint_kernels="", n_sched=len(SCHEDULES_F64),
        loss_kernels=loss_src, launch_loss=loss_launch, creduce=CREDUCE_TEMPLATE.format(),
        moments=", ".join(f"{mu}, {nu}" for mu, nu in s.moments),
        n_moments=len(s.moments),
        graph_offsets=", ".join(map(str, graph_offsets)),
        graph_keys=", ".join(map(str, graph_keys)),
        func_offsets=", ".join(map(str, func_offsets)),
        func_factors=", ".join(map(str, func_factors)),
        flops_pair_fwd=float(flops_pair_fwd), flops_pair_bwd=float(flops_pair_bwd),
        flops_atom=float(ops_c))
    meta = s.metadata()
    meta.update({"flops_pair_fwd": flops_pair_fwd, "flops_pair_bwd": flops_pair_bwd,
                 "flops_atom_contraction": ops_c, "flops_counted_for_nq": nq})
    return src, meta


# --------------------------------------------------------------------------
# Table-driven bases (levels whose straight-line contraction is too large to
# compile): the per-pair passes stay generated code, the contraction walks
# per-graph tries of component indices (csrc/contract_table.h).
# --------------------------------------------------------------------------

def build_tries(s):
    """Per graph, the trie of its terms' sorted factor tuples.  Returns
    (nodes [k, c0, c1] with children [c0, c1) or, at a leaf, c0 = its weight's
    index), the weights, the roots per depth {D: [(graph, r0, r1)]}."""
    nodes, coefs, roots = [], [], defaultdict(list)
    for g, terms in enumerate(s.terms):
        depth = len(terms[0][1])
        assert all(len(idx) == depth for _, idx in terms)
        tree = {}
        for coef, idx in terms:
            cur = tree
            for k in idx[:-1]:
                cur = cur.setdefault(k, {})
            assert idx[-1] not in cur
            cur[idx[-1]] = coef

        def place(d, level):
            r0 = len(nodes)
            items = sorted(d.items())
            nodes.extend([k, 0, 0] for k, _ in items)
            for t, (_, v) in enumerate(items):
                if level == depth:
                    coefs.append(v)
                    nodes[r0 + t][1] = len(coefs) - 1
                else:
                    nodes[r0 + t][1], nodes[r0 + t][2] = place(v, level + 1)
            return r0, r0 + len(items)

        r0, r1 = place(tree, 1)
        roots[depth].append((g, r0, r1))
    return nodes, coefs, dict(roots)


def contraction_flops(s):
    """Algorithmic flops of the contraction forward and reverse per atom as
    emit_contraction counts them (products of the terms, basis products,
    dV/dg, then every component's share of the reverse), without emitting
    the code."""
    ops = 0
    for terms in s.terms:
        ops += sum(len(idx) + (1 if coef != 1 else 0) for coef, idx in terms)
    for fn in s.funcs:
        ops += len(fn) - 1 + 2
        counts = defaultdict(int)
        for g in fn:
            counts[g] += 1
        for g, n in counts.items():
            ops += (len(fn) - 1) + 1 + (1 if n > 1 else 0)
    contrib = defaultdict(lambda: defaultdict(int))
    for g, terms in enumerate(s.terms):
        for coef, idx in terms:
            for k in set(idx):
                cnt = idx.count(k)
                rest = len(idx) - 1
                contrib[k][g] += (1 if coef * cnt != 1 and rest else 0) + max(rest - 1, 0) + 1
    for k in contrib:
        for g in contrib[k]:
            ops += contrib[k][g] + 1
    return ops


TABLE_TEMPLATE = r"""// Generated by paper_2007_08555_amd/codegen.py for the MTP basis of level {level}
// ({m} basis functions, {ngraphs} connected contractions, {C} moment components;
// {nnodes} trie nodes).  Table-driven contraction; do not edit.
#include "mtp_device.h"
#include "mtp_variant.h"
#if MTP_PART >= 1
#include "contract_table.h"
#endif

namespace {{
namespace {ns} {{

constexpr int C = {C};
constexpr int NMU = {n_mu};
constexpr int BLOCK = 64;

__device__ __forceinline__ int clamp_species(int z, int S) {{ return z < 0 ? 0 : (z >= S ? S - 1 : z); }}

#if MTP_PART >= 1
// trie nodes (k, c0, c1, slot), leaf weights, roots (graph, r0, r1, share) by
// depth, basis functions as lists of graphs, and per graph the components of
// its kSlots local slots (-1: unused); a node's slot is that of its k within
// its graph, or -1 when k is not among the graph's kSlots most frequent
__device__ const int kNode[] __attribute__((aligned(16))) = {{ {node_data} }};
__device__ const int kSlotK[] = {{ {slot_data} }};
__device__ const double kCoef[] = {{ {coef_data} }};
__device__ const int kRoots[] __attribute__((aligned(16))) = {{ {root_data} }};
__device__ const int kFOff[] = {{ {foff_data} }};
__device__ const int kFFac[] = {{ {ffac_data} }};

struct Tab {{
  static constexpr int kGraphs = {ngraphs};
  static constexpr int kC = C;
  static constexpr int kM = {m};
  static constexpr int kDepth = {depth};
  static constexpr int kMaxFactors = {qmax};
  static constexpr int kSlots = {slots};       // slots per graph in the table
  static constexpr int kSlots32 = {slots32};   // slots the FP32 kernels use (the first ones)
  static constexpr int kSlots64 = {slots64};   // slots the FP64 kernels use
  __device__ static const int4* node() {{ return reinterpret_cast<const int4*>(kNode); }}
  __device__ static const int* slot_k() {{ return kSlotK; }}
  __device__ static const double* coef() {{ return kCoef; }}
  __device__ static const int4* roots() {{ return reinterpret_cast<const int4*>(kRoots); }}
  __device__ static int root_begin(int d) {{
    constexpr int b[] = {{ {root_begin} }};
    return b[d];
  }}
  __device__ static const int* func_off() {{ return kFOff; }}
  __device__ static const int* func_fac() {{ return kFFac; }}
}};
#endif

#if MTP_PART == 1 || MTP_PART == 2
#if MTP_PART == 1
{kernels64}
#else
{kernels32}
#endif

template <typename T, bool COMP, bool WANT_B, int NQ, bool PR64 = false>
hipError_t launch_t(const void* a, unsigned flags, int schedule, hipStream_t s) {{
  const auto& args = *static_cast<const mtp::EvalArgs<T>*>(a);
  const bool reuse_moments = (flags & mtp::kEvalReuseMoments) != 0;   // the moments always go through memory
  const bool moments_only = (flags & mtp::kEvalMomentsOnly) != 0;
  // degrees whose adjoint the caller needs (all unless kEvalNuMask)
  const unsigned nu_need = (flags & mtp::kEvalNuMask) ? (flags >> mtp::kEvalNuShift) : ~0u;
  if (schedule != 0) return hipErrorInvalidValue;
  if (args.n_atoms <= 0) return hipSuccess;
  const dim3 grid((args.n_atoms + BLOCK - 1) / BLOCK);
  const size_t smem = (size_t)(args.n_c + args.n_c / args.nq) * sizeof(T);   // c, padded
#if MTP_PART == 1
{launch64}
#else
{launch32}
#endif
  return hipGetLastError();
}}
#endif  // parts 1, 2

#if MTP_PART == 3
{loss_kernels}
{creduce}

template <typename T>
hipError_t launch_loss_t(const void* a, const void* l, hipStream_t s) {{
  const auto& args = *static_cast<const mtp::EvalArgs<T>*>(a);
  const auto& la = *static_cast<const mtp::LossArgs<T>*>(l);
  if (args.n_atoms <= 0) return hipSuccess;
  const dim3 grid((args.n_atoms + BLOCK - 1) / BLOCK);
  const size_t smem = (size_t)(args.n_c + args.n_c / args.nq) * sizeof(T);   // c, padded
{launch_loss}
  return hipGetLastError();
}}
#endif  // part 3

}}  // namespace {ns}
}}  // namespace

namespace mtp_gen_{ns} {{
hipError_t eval64(unsigned flags, int schedule, const void* a, hipStream_t s);
hipError_t eval32(int precision, unsigned flags, int schedule, const void* a, hipStream_t s);
hipError_t loss(int precision, const void* a, const void* l, hipStream_t s);
#if MTP_PART == 1
hipError_t eval64(unsigned flags, int schedule, const void* a, hipStream_t s) {{
  using namespace {ns};
  const bool want_b = (flags & mtp::kEvalWantB) != 0;
  if (static_cast<const mtp::EvalArgs<double>*>(a)->nq == 8)
    return want_b ? launch_t<double, false, true, 8>(a, flags, schedule, s)
                  : launch_t<double, false, false, 8>(a, flags, schedule, s);
  return want_b ? launch_t<double, false, true, 0>(a, flags, schedule, s)
                : launch_t<double, false, false, 0>(a, flags, schedule, s);
}}
#elif MTP_PART == 2
hipError_t eval32(int precision, unsigned flags, int schedule, const void* a, hipStream_t s) {{
  using namespace {ns};
  const bool want_b = (flags & mtp::kEvalWantB) != 0;
  if (precision == 3)   // mixed precision: FP32 moments from the FP64 pair records
    return (flags & mtp::kEvalMomentsOnly) ? launch_t<float, false, false, 0, true>(a, flags, schedule, s)
                                           : hipErrorInvalidValue;
  if (precision == 2)
    return want_b ? launch_t<float, true, true, 0>(a, flags, schedule, s) : launch_t<float, true, false, 0>(a, flags, schedule, s);
  return want_b ? launch_t<float, false, true, 0>(a, flags, schedule, s) : launch_t<float, false, false, 0>(a, flags, schedule, s);
}}
#elif MTP_PART == 3
hipError_t loss(int precision, const void* a, const void* l, hipStream_t s) {{
  using namespace {ns};
  return precision == 0 ? launch_loss_t<double>(a, l, s) : launch_loss_t<float>(a, l, s);
}}
#endif
}}  // namespace mtp_gen_{ns}

#if MTP_PART == 0
namespace {{
namespace {ns} {{
hipError_t launch(int precision, unsigned flags, int schedule, const void* a, hipStream_t s) {{
  if (precision == 0) return mtp_gen_{ns}::eval64(flags, schedule, a, s);
  if (precision >= 1 && precision <= 3) return mtp_gen_{ns}::eval32(precision, flags, schedule, a, s);
  return hipErrorInvalidValue;
}}

{launch_loss_entry}

const int kMoments[] = {{ {moments} }};
const int kGraphKeyOffsets[] = {{ {graph_offsets} }};
const int kGraphKeys[] = {{ {graph_keys} }};
const int kFuncOffsets[] = {{ {func_offsets} }};
const int kFuncFactors[] = {{ {func_factors} }};

}}  // namespace {ns}
}}  // namespace

#if !defined(__HIP_DEVICE_COMPILE__)
extern const mtp::BasisVariant {ns}_variant = {{
  "{ns}", {level}, {n_moments}, {ns}::kMoments, {ngraphs}, {ns}::kGraphKeyOffsets, {ns}::kGraphKeys,
  {m}, {ns}::kFuncOffsets, {ns}::kFuncFactors, {C}, {n_mu}, {nu_max},
  {flops_pair_fwd}, {flops_pair_bwd}, {flops_atom}, {ns}::launch, {loss_ptr}, {ns}::BLOCK, 1, {partial_rows} }};
#endif
#endif  // part 0
"""

# pass splits of the table-driven bases: FP64 and FP32 components per pass
SCHEDULE_TABLE = {"f64": {"mom": 85, "adj": 90}, "f32": {"mom": 120, "adj": 120}}
# the loss gradient is compiled for table-driven levels up to this one
TABLE_LOSS_MAX_LEVEL = 20
# wavefronts sharing a workgroup's 64 atoms in the split table kernels
TABLE_WAVES = 4
# local LDS slots per graph for the split kernels' dV/dM shares, per level,
# (FP32, FP64): more slots catch more of the reverse walk's adds but hold
# fewer workgroups per CU (measured at level 24: FP64 best with 16 slots of
# 12, 16, 24, 32; FP32 best with 16 of 8, 16, 32; level 20 with 24)
TABLE_SLOTS = {20: (24, 24), 24: (16, 16)}


def table_slots(level, fp64=None):
    """Slots the FP32 (fp64=False) or FP64 (fp64=True) kernels use at a level;
    with fp64=None the table's slot count per graph (the larger)."""
    s32, s64 = TABLE_SLOTS.get(level, (16, 16))
    return max(s32, s64) if fp64 is None else (s64 if fp64 else s32)


def _moments_launch(tag, split):
    """Launch of one moments pass: the compensated kernel when COMP."""
    grid = _grid(split)
    return (f"if constexpr (COMP) {{ hipLaunchKernelGGL((moments_{tag}_ckernel<T, 0, PR64>), {grid}, dim3(BLOCK), smem, s, args); }} "
            f"else {{ hipLaunchKernelGGL((moments_{tag}_kernel<T, 0, PR64>), {grid}, dim3(BLOCK), smem, s, args); }}")


def _pair_pass_kernels(s, prec, sidx, sch):
    """Moments and adjoint pass kernels of one schedule and their launches."""
    src, mom_lines, adj_lines = [], [], []
    for pidx, (nus, comps) in enumerate(adjoint_passes(s, sch["mom"])):
        tag = f"{prec}s{sidx}_p{pidx}"
        kmap = {k: j for j, k in enumerate(comps)}
        body, _ = emit_pair_forward(s, comp_mode=True, nus=set(nus), kmap=kmap)
        nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
        src.append(MOMENTS_TEMPLATE.format(split=sch.get("split", 1), pidx=pidx, nus=nus, tag=tag, ncomp=len(comps), nmu=nmu,
                                           comp_list=", ".join(map(str, comps)),
                                           body="\n".join(" " * 4 + l for l in body)))
        mom_lines.append(_moments_launch(tag, sch.get('split', 1)))
    passes = adjoint_passes(s, sch["adj"])
    for pidx, (nus, comps) in enumerate(passes):
        tag = f"{prec}s{sidx}_p{pidx}"
        gmap = {k: j for j, k in enumerate(comps)}
        nmu = 1 + max(mu for (mu, nu, abc), k in s.comp.items() if nu in nus)
        body, _ = emit_pair_backward(s, nus=nus, gmap=gmap, nmu=nmu)
        src.append(ADJOINT_TEMPLATE.format(split=sch.get("split", 1), pidx=pidx, nus=nus, tag=tag, ncomp=len(comps), nmu=nmu,
                                           comp_list=", ".join(map(str, comps)),
                                           body="\n".join(" " * 4 + l for l in body)))
    pre, adj = _adjoint_launches([(f"{prec}s{sidx}_p{pidx}", nus) for pidx, (nus, _) in enumerate(passes)],
                                 sch.get("split", 1))
    return src, mom_lines, pre + adj


def generate_table(lev_max):
    """Source of a table-driven basis (same entry points and table entry as
    generate())."""
    s = Schedule(lev_max)
    ns = f"lev{lev_max}"
    nodes, coefs, roots = build_tries(s)
    depth = max(roots)
    qmax = max(len(f) for f in s.funcs)
    # each root's share (wavefront) in the split kernels: largest tries first,
    # each to the wavefront with the fewest nodes so far
    def trie_size(r0, r1, level, depth_):
        n = r1 - r0
        if level < depth_:
            for t in range(r0, r1):
                n += trie_size(nodes[t][1], nodes[t][2], level + 1, depth_)
        return n
    sizes = {g: trie_size(r0, r1, 1, d) for d, lst in roots.items() for g, r0, r1 in lst}
    # local slots: per graph its nslot most frequent components (the
    # split kernels add their dV/dM shares in LDS, flushed once per graph)
    node_slot = [-1] * len(nodes)
    nslot = table_slots(lev_max)
    slot_k = [-1] * (nslot * len(s.keys))
    for d, lst in roots.items():
        for g, r0, r1 in lst:
            members, stack = [], [(r0, r1, 1)]
            while stack:
                a, b, level = stack.pop()
                for t in range(a, b):
                    members.append(t)
                    if level < d:
                        stack.append((nodes[t][1], nodes[t][2], level + 1))
            freq = defaultdict(int)
            for t in members:
                freq[nodes[t][0]] += 1
            top = sorted(freq, key=lambda k: (-freq[k], k))[:nslot]
            slot_of = {k: j for j, k in enumerate(top)}
            for j, k in enumerate(top):
                slot_k[g * nslot + j] = k
            for t in members:
                node_slot[t] = slot_of.get(nodes[t][0], -1)
    load, share = [0] * TABLE_WAVES, {}
    for g in sorted(sizes, key=lambda g: (-sizes[g], g)):
        w = min(range(TABLE_WAVES), key=lambda t: (load[t], t))
        share[g] = w
        load[w] += sizes[g]
    root_list, root_begin = [], [0, 0]
    for d in range(1, depth + 1):
        for g, r0, r1 in roots.get(d, []):
            root_list += [g, r0, r1, share[g]]
        root_begin.append(len(root_list) // 4)
    parts = {}
    for prec in ("f64", "f32"):
        src, mom, adj = _pair_pass_kernels(s, prec, 0, SCHEDULE_TABLE[prec])
        W = TABLE_WAVES
        split_grid = "dim3((args.n_atoms + 63) / 64), dim3(64 * " + str(W) + ")"
        launch = (["if (!reuse_moments) {"] + ["  " + l for l in mom] + ["}"] +
                  ["if (moments_only) return hipGetLastError();",
                   "// the graphs of a workgroup's atoms shared out among wavefronts (with the",
                   "// partial rows at hand), except for degree-masked calls (xi = e_alpha: few",
                   "// graphs, where summing the shares would cost more than it spreads)",
                   "const bool split = args.Gpart && !(flags & mtp::kEvalNuMask);",
                   "if (args.M32) {   // mixed precision: FP32 moments",
                   "  if constexpr (std::is_same<T, double>::value) {",
                   "    if (split)",
                   f"      hipLaunchKernelGGL((mtp::contract_table_split_kernel<T, WANT_B, Tab, true, {W}>), {split_grid}, 0, s, args);",
                   "    else",
                   "      hipLaunchKernelGGL((mtp::contract_table_kernel<T, WANT_B, Tab, true>), grid, dim3(BLOCK), 0, s, args);",
                   "  } else {",
                   "    return hipErrorInvalidValue;",
                   "  }",
                   "} else if (split) {",
                   f"  hipLaunchKernelGGL((mtp::contract_table_split_kernel<T, WANT_B, Tab, false, {W}>), {split_grid}, 0, s, args);",
                   "} else {",
                   "  hipLaunchKernelGGL((mtp::contract_table_kernel<T, WANT_B, Tab>), grid, dim3(BLOCK), 0, s, args);",
                   "}"] +
                  adj)
        parts[prec] = ("\n".join(src), "\n".join("  " + l for l in launch))
    with_loss = lev_max <= TABLE_LOSS_MAX_LEVEL
    if with_loss:
        loss_src, loss_launch = emit_loss_kernels(s, budget=45)
        old = "  hipLaunchKernelGGL((tangent_contract_kernel<T>), grid, dim3(BLOCK), 0, s, args, la);"
        assert old in loss_launch
        loss_launch = loss_launch.replace(
            old, "  if (args.Gpart)\n"
                 f"    hipLaunchKernelGGL((mtp::contract_table_loss_split_kernel<T, Tab, {TABLE_WAVES}>), "
                 f"dim3((args.n_atoms + 63) / 64), dim3(64 * {TABLE_WAVES}), 0, s, args, la);\n"
                 "  else\n"
                 "    hipLaunchKernelGGL((mtp::contract_table_loss_kernel<T, Tab>), grid, dim3(BLOCK), 0, s, args, la);")
        creduce = CREDUCE_TEMPLATE.format()
        loss_entry = (f"hipError_t launch_loss(int precision, const void* a, const void* l, hipStream_t s) {{\n"
                      f"  return mtp_gen_{ns}::loss(precision, a, l, s);\n}}")
        loss_ptr = f"{ns}::launch_loss"
    else:
        loss_src, loss_launch, creduce, loss_entry, loss_ptr = "", "  return hipErrorNotSupported;", "", "", "nullptr"
    _, ops_f = emit_pair_forward(s, comp_mode=True)
    _, ops_b = emit_pair_backward(s)
    ops_c = contraction_flops(s)
    nq = 8
    rad_f = 6 + 3 * (nq - 2) + 2 * s.n_mu * nq + 2 * s.n_mu
    rad_b = rad_f + 5 * (nq - 2) + 2 * s.n_mu * nq + 4 * s.n_mu + 2
    graph_keys, graph_offsets = [], [0]
    for k in s.keys:
        graph_keys += list(k)
        graph_offsets.append(len(graph_keys))
    func_factors, func_offsets = [], [0]
    for f in s.funcs:
        func_factors += list(f)
        func_offsets.append(len(func_factors))
    join = lambda v: ", ".join(map(str, v))
    src = TABLE_TEMPLATE.format(
        level=lev_max, m=len(s.funcs), ngraphs=len(s.keys), C=s.C, n_mu=s.n_mu, nu_max=s.nu_max, ns=ns,
        nnodes=len(nodes), depth=depth, qmax=qmax,
        node_data=join(v for t, nd in enumerate(nodes) for v in (nd[0], nd[1], nd[2], node_slot[t])),
        slot_data=join(slot_k), slots=nslot, slots32=table_slots(lev_max, fp64=False),
        slots64=table_slots(lev_max, fp64=True),
        coef_data=", ".join(repr(float(c)) for c in coefs),
        root_data=join(root_list), root_begin=join(root_begin),
        foff_data=join(func_offsets), ffac_data=join(func_factors),
        kernels64=parts["f64"][0], kernels32=parts["f32"][0], launch64=parts["f64"][1], launch32=parts["f32"][1],
        loss_kernels=loss_src, creduce=creduce, launch_loss=loss_launch, launch_loss_entry=loss_entry,
        loss_ptr=loss_ptr,
        # per atom: (TABLE_WAVES - 1) shares of C + 2 n_graphs rows (the loss kernel's need; the
        # evaluation uses C + n_graphs of them)
        partial_rows=(TABLE_WAVES - 1) * (s.C + 2 * len(s.keys)),
        moments=", ".join(f"{mu}, {nu}" for mu, nu in s.moments), n_moments=len(s.moments),
        graph_offsets=join(graph_offsets), graph_keys=join(graph_keys),
        func_offsets=join(func_offsets), func_factors=join(func_factors),
        flops_pair_fwd=float(ops_f + rad_f), flops_pair_bwd=float(ops_b + rad_b + 1), flops_atom=float(ops_c))
    assert all(float(c) == c for c in coefs), "a term weight is not exact in FP64"
    meta = s.metadata()
    meta.update({"flops_pair_fwd": ops_f + rad_f, "flops_pair_bwd": ops_b + rad_b + 1,
                 "flops_atom_contraction": ops_c, "flops_counted_for_nq": nq, "table": True,
                 "trie_nodes": len(nodes), "loss": with_loss})
    return src, meta


LEVELS = (2, 4, 6, 8, 10, 12, 14, 16)
# bases compiled with the table-driven contraction
TABLE_LEVELS = (20, 24)


PARTS = (("", 0), ("_eval64", 1), ("_eval32", 2), ("_loss", 3))


def write_all(outdir, levels=LEVELS):
    """Writes, per level, the generated kernels (gen_levL.inc) and four
    translation units that compile its parts (the table entry and launchers;
    FP64 evaluation; FP32 evaluation; loss gradient), so that the parts of a
    large basis compile in parallel."""
    os.makedirs(outdir, exist_ok=True)
    metas = {}
    files = []

    def put(path, text):
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as fh:
                fh.write(text)

    for L in levels:
        src, meta = generate_table(L) if L in TABLE_LEVELS else generate(L)
        put(os.path.join(outdir, f"gen_lev{L}.inc"), src)
        for suffix, part in PARTS:
            path = os.path.join(outdir, f"gen_lev{L}{suffix}.hip")
            put(path, f"// Part {part} of the generated kernels of level {L}.\n#define MTP_PART {part}\n"
                      f'#include "gen_lev{L}.inc"\n')
            files.append(path)
        metas[f"lev{L}"] = meta
    reg = ["// Generated: the table of compiled bases.", '#include "mtp_variant.h"', ""]
    reg += [f"extern const mtp::BasisVariant lev{L}_variant;" for L in levels]
    reg += ["", "namespace mtp {", "const BasisVariant* const kVariants[] = {"]
    reg += [f"  &lev{L}_variant," for L in levels]
    reg += ["};", f"const int kNumVariants = {len(levels)};", "}  // namespace mtp", ""]
    reg_src = "\n".join(reg)
    reg_path = os.path.join(outdir, "variants.cpp")
    if not os.path.exists(reg_path) or open(reg_path).read() != reg_src:
        with open(reg_path, "w") as fh:
            fh.write(reg_src)
    files.append(reg_path)
    with open(os.path.join(outdir, "variants.json"), "w") as fh:
        json.dump(metas, fh, indent=1)
    return files, metas
