// Table-driven contraction of the moments of one atom (paper, section 2.1:
// eqs. V_MTP and MTPbasisLevel8, the connected contractions and their
// products), used for the bases whose straight-line kernels would be too
// large to compile (levels 20 and 24).
//
// A connected contraction is a sum over index assignments of products of
// symmetric moment components; the terms of one graph all have one factor
// per vertex.  Sorting each term's factors and sharing common prefixes gives
// a trie per graph: a node holds a component index k, an inner node the
// range of its children, a leaf (depth D = number of vertices) the term's
// integer weight.  With T(n) the value below node n (the weight at a leaf,
// else the sum over children c of M[k_c] T(c)), the graph value is
// T(root), and its derivative in M[k] is the sum over nodes n with k_n = k
// of P(n) T(n), P(n) the product of M over n's strict ancestors.  One walk
// in order gives the value; a second walk with P carried down and T
// returned up accumulates dV/dM = sum_g dV/dg dg/dM.
//
// One thread per atom; the tables are read by every lane at the same index,
// so the node loads are uniform across the wavefront.  M, G, the graph
// values and dV/dg are [rows][stride] columns of the atom (Mi = M + i).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mtp_device.h"

namespace mtp {

// A term weight (an integer, exact in FP64) in the arithmetic type.
template <typename T>
__device__ __forceinline__ T from_coef(double c);
template <>
__device__ __forceinline__ float from_coef<float>(double c) { return static_cast<float>(c); }
template <>
__device__ __forceinline__ double from_coef<double>(double c) { return c; }
template <>
__device__ __forceinline__ Dual<double> from_coef<Dual<double>>(double c) { return Dual<double>(c); }
template <>
__device__ __forceinline__ Dual<float> from_coef<Dual<float>>(double c) { return Dual<float>(static_cast<float>(c)); }

// Value below the nodes [a, b) at depth L of a graph with D vertices.
template <typename T, int L, int D, typename Tab, typename MLoad>
__device__ T trie_value(int a, int b, const MLoad& mload) {
  T s = T(0);
  for (int n = a; n < b; ++n) {
    const int4 nd = Tab::node()[n];
    const T m = mload(nd.x);
    if constexpr (L == D) {
      s += from_coef<T>(Tab::coef()[nd.y]) * m;
    } else {
      s += m * trie_value<T, L + 1, D, Tab>(nd.y, nd.z, mload);
    }
  }
  return s;
}

// As trie_value, and adds P(n) T(n) to the adjoint of M[k_n] for every node
// (P = dV/dg times the product of the ancestors' moments).
template <typename T, int L, int D, typename Tab, typename MLoad, typename GAdd>
__device__ T trie_reverse(int a, int b, T P, const MLoad& mload, const GAdd& gadd) {
  T s = T(0);
  for (int n = a; n < b; ++n) {
    const int4 nd = Tab::node()[n];
    const T m = mload(nd.x);
    T sub;
    if constexpr (L == D) {
      sub = from_coef<T>(Tab::coef()[nd.y]);
    } else {
      sub = trie_reverse<T, L + 1, D, Tab>(nd.y, nd.z, P * m, mload, gadd);
    }
    gadd(nd.x, P * sub);
    s += m * sub;
  }
  return s;
}

// As trie_reverse, with gadd given the node record (k in .x, local slot in .w).
template <typename T, int L, int D, typename Tab, typename MLoad, typename GAdd>
__device__ T trie_reverse_nd(int a, int b, T P, const MLoad& mload, const GAdd& gadd) {
  T s = T(0);
  for (int n = a; n < b; ++n) {
    const int4 nd = Tab::node()[n];
    const T m = mload(nd.x);
    T sub;
    if constexpr (L == D) {
      sub = from_coef<T>(Tab::coef()[nd.y]);
    } else {
      sub = trie_reverse_nd<T, L + 1, D, Tab>(nd.y, nd.z, P * m, mload, gadd);
    }
    gadd(nd, P * sub);
    s += m * sub;
  }
  return s;
}

// Graph values of every graph with D vertices (roots listed per depth) whose
// root entry e (graph e.x, trie e.y .. e.z, workgroup share e.w) take(e)
// accepts.
template <typename T, int D, typename Tab, typename MLoad, typename VStore, typename Take>
__device__ __forceinline__ void graphs_forward(const MLoad& mload, const VStore& vstore, const Take& take) {
  if constexpr (D <= Tab::kDepth) {
    for (int r = Tab::root_begin(D); r < Tab::root_begin(D + 1); ++r) {
      const int4 e = Tab::roots()[r];
      if (take(e)) vstore(e.x, trie_value<T, 1, D, Tab>(e.y, e.z, mload));
    }
    graphs_forward<T, D + 1, Tab>(mload, vstore, take);
  }
}

template <typename T, int D, typename Tab, typename MLoad, typename VStore>
__device__ __forceinline__ void graphs_forward(const MLoad& mload, const VStore& vstore) {
  graphs_forward<T, D, Tab>(mload, vstore, [](const int4&) { return true; });
}

// A graph whose dV/dg is exactly zero adds nothing and is skipped (for
// xi = e_alpha, as in the normal equations, all but alpha's graphs); only
// the roots take(e) accepts are walked.
template <typename T, int D, typename Tab, typename MLoad, typename DgLoad, typename GAdd, typename Take>
__device__ __forceinline__ void graphs_reverse(const MLoad& mload, const DgLoad& dgload, const GAdd& gadd,
                                               const Take& take) {
  if constexpr (D <= Tab::kDepth) {
    for (int r = Tab::root_begin(D); r < Tab::root_begin(D + 1); ++r) {
      const int4 e = Tab::roots()[r];
      if (!take(e)) continue;
      const T P = dgload(e.x);
      if constexpr (std::is_floating_point<T>::value) {
        if (P == T(0)) continue;
      }
      (void)trie_reverse<T, 1, D, Tab>(e.y, e.z, P, mload, gadd);
    }
    graphs_reverse<T, D + 1, Tab>(mload, dgload, gadd, take);
  }
}

template <typename T, int D, typename Tab, typename MLoad, typename DgLoad, typename GAdd>
__device__ __forceinline__ void graphs_reverse(const MLoad& mload, const DgLoad& dgload, const GAdd& gadd) {
  graphs_reverse<T, D, Tab>(mload, dgload, gadd, [](const int4&) { return true; });
}

// graphs_reverse for the split kernels: the shares of each graph's L (at
// most kSlots, the table's slot count) most frequent components are added
// into local slots (szero, sadd; an
// atom's slots in LDS) and flushed into the atom's rows once per graph
// (sflush(j, k)); the other components go to the rows directly (gadd).  The
// slot count trades the share of adds the slots catch (level 24 with 16
// slots: 72 %; level 20 with 24: 91 %) against workgroups per CU.
template <typename T, int D, typename Tab, int L, typename MLoad, typename DgLoad, typename SZero, typename SAdd,
          typename SFlush, typename GAdd, typename Take>
__device__ __forceinline__ void graphs_reverse_slots(const MLoad& mload, const DgLoad& dgload, const SZero& szero,
                                                     const SAdd& sadd, const SFlush& sflush, const GAdd& gadd,
                                                     const Take& take) {
  if constexpr (D <= Tab::kDepth) {
    for (int r = Tab::root_begin(D); r < Tab::root_begin(D + 1); ++r) {
      const int4 e = Tab::roots()[r];
      if (!take(e)) continue;
      const T P = dgload(e.x);
      if constexpr (std::is_floating_point<T>::value) {
        if (P == T(0)) continue;
      }
      for (int j = 0; j < L; ++j) szero(j);
      (void)trie_reverse_nd<T, 1, D, Tab>(e.y, e.z, P, mload, [&](const int4& nd, T v) {
        if (nd.w >= 0 && nd.w < L)
          sadd(nd.w, v);
        else
          gadd(nd.x, v);
      });
      for (int j = 0; j < L; ++j) {
        const int k = Tab::slot_k()[e.x * Tab::kSlots + j];
        if (k >= 0) sflush(j, k);
      }
    }
    graphs_reverse_slots<T, D + 1, Tab, L>(mload, dgload, szero, sadd, sflush, gadd, take);
  }
}

// Basis functions B_alpha = product of graph values (eq. MTPbasisLevel8 and
// its generalisation), V = sum_alpha xi_alpha B_alpha, and dV/dg added to
// the graphs' adjoints: for each function, prefix products times suffix
// products give the product of the other factors.  bout(alpha, B) receives
// every B when ALL_B; otherwise functions with xi_alpha exactly zero, which
// add nothing, are skipped.  Only the functions a0, a0 + a_step, ... are
// formed (a share of a workgroup's wavefronts), or, with alist, the acount
// functions it lists in ascending order.
template <typename T, typename Tab, bool ALL_B, typename XiLoad, typename VLoad, typename DgAdd, typename BOut>
__device__ __forceinline__ T basis_products(const XiLoad& xiload, const VLoad& vload, const DgAdd& dgadd,
                                            const BOut& bout, int a0 = 0, int a_step = 1,
                                            const int* alist = nullptr, int acount = 0) {
  constexpr int Q = Tab::kMaxFactors;
  T V = T(0);
  const int n_iter = alist ? acount : (Tab::kM - a0 + a_step - 1) / a_step;
  for (int t = 0; t < n_iter; ++t) {
    const int a = alist ? alist[t] : a0 + t * a_step;
    if constexpr (!ALL_B && std::is_floating_point<T>::value) {
      if (xiload(a) == T(0)) continue;
    }
    const int f0 = Tab::func_off()[a];
    const int q = Tab::func_off()[a + 1] - f0;
    int g[Q];
    T v[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      g[j] = j < q ? Tab::func_fac()[f0 + j] : 0;
      v[j] = j < q ? vload(g[j]) : T(1);
    }
    T pre[Q + 1];
    pre[0] = T(1);
#pragma unroll
    for (int j = 0; j < Q; ++j) pre[j + 1] = pre[j] * v[j];
    const T B = pre[Q];
    const T x = xiload(a);
    V += x * B;
    bout(a, B);
    T suf = T(1);
#pragma unroll
    for (int j = Q - 1; j >= 0; --j) {
      if (j < q) dgadd(g[j], x * (pre[j] * suf));
      suf = suf * v[j];
    }
  }
  return V;
}

// Forward contraction, basis products and reverse sweep of one atom per
// thread: graph values to the upper half of D, B (when wanted), V to site,
// dV/dg to the lower half of D, G = dV/dM.
// M32: the moments are read from args.M32 (FP32, the mixed-precision path)
// and widened.
template <typename T, bool WANT_B, typename Tab, bool M32 = false>
__global__ void __launch_bounds__(64) contract_table_kernel(const EvalArgs<T> args) {
  // graphs that some function with xi_alpha != 0 uses (a bit per graph),
  // whether that is all of them, and the functions with xi_alpha != 0 in
  // ascending order (the workgroup is one wavefront: ballots compact them)
  __shared__ uint32_t need[(Tab::kGraphs + 31) / 32];
  __shared__ int alist[WANT_B ? 1 : Tab::kM];
  int n_zero = 0, acount = Tab::kM;
  if constexpr (!WANT_B) {
    for (int w = threadIdx.x; w < (Tab::kGraphs + 31) / 32; w += 64) need[w] = 0u;
    const int lane = threadIdx.x;
    int base = 0;
    for (int a0 = 0; a0 < Tab::kM; a0 += 64) {
      const int a = a0 + lane;
      const bool nz = a < Tab::kM && args.xi[a] != T(0);
      const unsigned long long bal = __ballot(nz);
      if (nz) alist[base + __popcll(bal & ((1ull << lane) - 1ull))] = a;
      base += __popcll(bal);
    }
    acount = base;
    n_zero = Tab::kM - base;
    __syncthreads();
    if (n_zero > 0) {   // uniform over the workgroup
      for (int t0 = threadIdx.x; t0 < acount; t0 += 64)
        for (int t = Tab::func_off()[alist[t0]]; t < Tab::func_off()[alist[t0] + 1]; ++t) {
          const int g = Tab::func_fac()[t];
          atomicOr(&need[g >> 5], 1u << (g & 31));
        }
      __syncthreads();
    }
  }
  const bool need_all = WANT_B || n_zero == 0;
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= args.n_atoms) return;
  const size_t st = args.stride;
  const T* Mi = args.M + i;
  const float* M32i = args.M32 + i;
  T* Gi = args.G + i;
  T* Dg = args.D + i;
  T* Dv = args.D + (size_t)Tab::kGraphs * st + i;
  const auto mload = [&](int k) {
    if constexpr (M32)
      return static_cast<T>(M32i[(size_t)k * st]);
    else
      return Mi[(size_t)k * st];
  };
  if constexpr (WANT_B) {
    graphs_forward<T, 1, Tab>(mload, [&](int g, T v) { Dv[(size_t)g * st] = v; });
  } else {
    // only the graphs of functions with xi_alpha != 0 (the others' values
    // are never read): for xi = e_alpha, as in the normal equations, alpha's
    const bool all = need_all;
    graphs_forward<T, 1, Tab>(mload, [&](int g, T v) { Dv[(size_t)g * st] = v; },
                              [&](const int4& e) { return all || ((need[e.x >> 5] >> (e.x & 31)) & 1u); });
  }
  for (int g = 0; g < Tab::kGraphs; ++g) Dg[(size_t)g * st] = T(0);
  // with some xi_alpha zero (xi = e_alpha in the normal equations) only the
  // listed functions are formed: the others would add nothing
  const T V = basis_products<T, Tab, WANT_B>(
      [&](int a) { return args.xi[a]; }, [&](int g) { return Dv[(size_t)g * st]; },
      [&](int g, T v) { Dg[(size_t)g * st] += v; },
      [&](int a, T B) {
        if (WANT_B) args.B[(size_t)a * args.b_stride + i] = B;
      },
      0, 1, need_all ? nullptr : alist, acount);
  args.site[i] = V;
  for (int k = 0; k < Tab::kC; ++k) Gi[(size_t)k * st] = T(0);
  // graphs outside the need mask have dV/dg = 0 exactly: skipped without
  // loading their dV/dg (the loads of every root, each waited on before its
  // branch, dominated the degree-masked calls of the normal equations)
  graphs_reverse<T, 1, Tab>(mload, [&](int g) { return Dg[(size_t)g * st]; },
                            [&](int k, T v) { Gi[(size_t)k * st] += v; },
                            [&](const int4& e) { return need_all || ((need[e.x >> 5] >> (e.x & 31)) & 1u); });
}

// The same with the work of a workgroup's 64 atoms shared out among W
// wavefronts that take the same atoms (lane l of every wavefront is atom
// l): a batch of some ten thousand atoms gives one thread-per-atom wavefront
// per SIMD or fewer, too few to cover the latencies of the walks' dependent
// loads.  Root e goes to wavefront e.w % W (shares balanced by trie size
// when the tables are generated), function a to wavefront a % W.  Each
// wavefront writes the values of its graphs, adds the dV/dg of its
// functions and the dV/dM of its graphs' reverse walks into rows of its own
// (wavefront 0 into D and G, wavefront w > 0 into rows w - 1 of
// args.Gpart: C rows for dV/dM, then n_graphs rows for dV/dg), and the
// shares are added in wavefront order where they are read (bitwise
// repeatable; a different order of the sums than the one-wavefront kernel).
// The reverse walks add into per-graph LDS slots (graphs_reverse_slots).
template <typename T, bool WANT_B, typename Tab, bool M32, int W>
__global__ void __launch_bounds__(64 * W) contract_table_split_kernel(const EvalArgs<T> args) {
  __shared__ uint32_t need[(Tab::kGraphs + 31) / 32];
  __shared__ int n_zero;
  __shared__ T vpart[W][64];
  // local dV/dM slots of each wavefront's graph (the first kSlots32 or
  // kSlots64 of the table's slots, by precision)
  constexpr int L = sizeof(T) == 8 ? Tab::kSlots64 : Tab::kSlots32;
  __shared__ T gslot[W][L][64];
  if constexpr (!WANT_B) {
    for (int w = threadIdx.x; w < (Tab::kGraphs + 31) / 32; w += 64 * W) need[w] = 0u;
    if (threadIdx.x == 0) n_zero = 0;
    __syncthreads();
    for (int a = threadIdx.x; a < Tab::kM; a += 64 * W)
      if (args.xi[a] == T(0)) atomicAdd(&n_zero, 1);
    __syncthreads();
    if (n_zero > 0) {   // uniform over the workgroup
      for (int a = threadIdx.x; a < Tab::kM; a += 64 * W)
        if (args.xi[a] != T(0))
          for (int t = Tab::func_off()[a]; t < Tab::func_off()[a + 1]; ++t) {
            const int g = Tab::func_fac()[t];
            atomicOr(&need[g >> 5], 1u << (g & 31));
          }
      __syncthreads();
    }
  }
  const bool need_all = WANT_B || n_zero == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const bool active = i < args.n_atoms;
  const size_t st = args.stride;
  const size_t rows = (size_t)Tab::kC + Tab::kGraphs;   // partial rows per wavefront
  const T* Mi = args.M + i;
  const float* M32i = args.M32 + i;
  T* Gi = args.G + i;
  T* Dg = args.D + i;
  T* Dv = args.D + (size_t)Tab::kGraphs * st + i;
  T* Gw = wave == 0 ? Gi : args.Gpart + (size_t)(wave - 1) * rows * st + i;
  T* Dw = wave == 0 ? Dg : args.Gpart + ((size_t)(wave - 1) * rows + Tab::kC) * st + i;
  const auto mload = [&](int k) {
    if constexpr (M32)
      return static_cast<T>(M32i[(size_t)k * st]);
    else
      return Mi[(size_t)k * st];
  };
  const auto mine = [&](const int4& e) { return (e.w % W) == wave; };
  if (active) {
    for (int k = 0; k < Tab::kC; ++k) Gw[(size_t)k * st] = T(0);
    for (int g = 0; g < Tab::kGraphs; ++g) Dw[(size_t)g * st] = T(0);
    const bool all = need_all;
    graphs_forward<T, 1, Tab>(mload, [&](int g, T v) { Dv[(size_t)g * st] = v; }, [&](const int4& e) {
      return mine(e) && (all || ((need[e.x >> 5] >> (e.x & 31)) & 1u));
    });
  }
  __syncthreads();   // every graph value written
  T V = T(0);
  if (active)
    V = basis_products<T, Tab, WANT_B>(
        [&](int a) { return args.xi[a]; }, [&](int g) { return Dv[(size_t)g * st]; },
        [&](int g, T v) { Dw[(size_t)g * st] += v; },
        [&](int a, T B) {
          if (WANT_B) args.B[(size_t)a * args.b_stride + i] = B;
        },
        wave, W);
  vpart[wave][lane] = V;
  __syncthreads();   // every share of dV/dg and V written
  if (active) {
    if (wave == 0) {
      T s = vpart[0][lane];
      for (int w = 1; w < W; ++w) s += vpart[w][lane];
      args.site[i] = s;
    }
    const auto dgload = [&](int g) {
      T d = Dg[(size_t)g * st];
      for (int w = 1; w < W; ++w) d += args.Gpart[((size_t)(w - 1) * rows + Tab::kC + g) * st + i];
      return d;
    };
    graphs_reverse_slots<T, 1, Tab, L>(
        mload, dgload, [&](int j) { gslot[wave][j][lane] = T(0); },
        [&](int j, T v) { gslot[wave][j][lane] += v; },
        [&](int j, int k) { Gw[(size_t)k * st] += gslot[wave][j][lane]; },
        [&](int k, T v) { Gw[(size_t)k * st] += v; }, mine);
  }
  __syncthreads();   // every share of dV/dM written
  if (active)
    for (int k = wave; k < Tab::kC; k += W) {
      T g = Gi[(size_t)k * st];
      for (int w = 1; w < W; ++w) g += args.Gpart[((size_t)(w - 1) * rows + k) * st + i];
      Gi[(size_t)k * st] = g;
    }
}

// The same on dual numbers for the loss gradient: moments carry their
// tangent along the displacement field (la.dM), so the forward walk gives
// graph values and tangents, the products give a B_alpha + tangent of
// B_alpha per atom (the xi part of the gradient) and dV/dg with its tangent,
// and the reverse walk the tangent of G (la.dG).  la.gd holds four blocks of
// n_graphs rows: values, their tangents, dV/dg, its tangent.
template <typename R, typename Tab>
__global__ void __launch_bounds__(64) contract_table_loss_kernel(const EvalArgs<R> args, const LossArgs<R> la) {
  using T = Dual<R>;
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= args.n_atoms) return;
  const size_t st = args.stride;
  const size_t ng = Tab::kGraphs;
  const R* Mi = args.M + i;
  const R* dMi = la.dM + i;
  R* gd = la.gd + i;
  R* dGi = la.dG + i;
  const R aw = la.a_atom[i];
  const auto mload = [&](int k) { return T(Mi[(size_t)k * st], dMi[(size_t)k * st]); };
  graphs_forward<T, 1, Tab>(mload, [&](int g, T v) {
    gd[(size_t)g * st] = v.v;
    gd[(ng + g) * st] = v.d;
  });
  for (size_t g = 0; g < ng; ++g) {
    gd[(2 * ng + g) * st] = R(0);
    gd[(3 * ng + g) * st] = R(0);
  }
  (void)basis_products<T, Tab, true>(
      [&](int a) { return T(args.xi[a]); },
      [&](int g) { return T(gd[(size_t)g * st], gd[(ng + g) * st]); },
      [&](int g, T v) {
        gd[(2 * ng + g) * st] += v.v;
        gd[(3 * ng + g) * st] += v.d;
      },
      [&](int a, T B) { la.xi_terms[(size_t)a * st + i] = aw * B.v + B.d; });
  for (int k = 0; k < Tab::kC; ++k) dGi[(size_t)k * st] = R(0);
  graphs_reverse<T, 1, Tab>(mload, [&](int g) { return T(gd[(2 * ng + g) * st], gd[(3 * ng + g) * st]); },
                            [&](int k, T v) { dGi[(size_t)k * st] += v.d; });
}

// contract_table_loss_kernel with the work shared out among W wavefronts as
// in contract_table_split_kernel: each wavefront's share of dV/dg and its
// tangent, and of the tangent of G, in rows of its own (wavefront w > 0:
// rows w - 1 of args.Gpart, C rows for dG, then 2 n_graphs rows for dV/dg
// and its tangent), added in wavefront order where they are read.
template <typename R, typename Tab, int W>
__global__ void __launch_bounds__(64 * W) contract_table_loss_split_kernel(const EvalArgs<R> args,
                                                                          const LossArgs<R> la) {
  using T = Dual<R>;
  constexpr int L = sizeof(R) == 8 ? Tab::kSlots64 : Tab::kSlots32;
  __shared__ R gslot[W][L][64];   // local slots of the tangent of dV/dM
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const bool active = i < args.n_atoms;
  const size_t st = args.stride;
  const size_t ng = Tab::kGraphs;
  const size_t rows = (size_t)Tab::kC + 2 * ng;
  const R* Mi = args.M + i;
  const R* dMi = la.dM + i;
  R* gd = la.gd + i;
  R* dGi = la.dG + i;
  R* dGw = wave == 0 ? dGi : args.Gpart + (size_t)(wave - 1) * rows * st + i;
  // dV/dg and its tangent of this wavefront's functions
  R* Dw = wave == 0 ? gd + 2 * ng * st : args.Gpart + ((size_t)(wave - 1) * rows + Tab::kC) * st + i;
  const auto mload = [&](int k) { return T(Mi[(size_t)k * st], dMi[(size_t)k * st]); };
  const auto mine = [&](const int4& e) { return (e.w % W) == wave; };
  if (active) {
    for (int k = 0; k < Tab::kC; ++k) dGw[(size_t)k * st] = R(0);
    for (size_t g = 0; g < 2 * ng; ++g) Dw[g * st] = R(0);
    graphs_forward<T, 1, Tab>(mload, [&](int g, T v) {
      gd[(size_t)g * st] = v.v;
      gd[(ng + g) * st] = v.d;
    }, mine);
  }
  __syncthreads();   // every graph value and tangent written
  if (active) {
    const R aw = la.a_atom[i];
    (void)basis_products<T, Tab, true>(
        [&](int a) { return T(args.xi[a]); },
        [&](int g) { return T(gd[(size_t)g * st], gd[(ng + g) * st]); },
        [&](int g, T v) {
          Dw[(size_t)g * st] += v.v;
          Dw[(ng + g) * st] += v.d;
        },
        [&](int a, T B) { la.xi_terms[(size_t)a * st + i] = aw * B.v + B.d; }, wave, W);
  }
  __syncthreads();   // every share of dV/dg written
  if (active) {
    const auto dgload = [&](int g) {
      R v = gd[(2 * ng + g) * st], d = gd[(3 * ng + g) * st];
      for (int w = 1; w < W; ++w) {
        const R* p = args.Gpart + ((size_t)(w - 1) * rows + Tab::kC) * st + i;
        v += p[(size_t)g * st];
        d += p[(ng + g) * st];
      }
      return T(v, d);
    };
    graphs_reverse_slots<T, 1, Tab, L>(
        mload, dgload, [&](int j) { gslot[wave][j][lane] = R(0); },
        [&](int j, T v) { gslot[wave][j][lane] += v.d; },
        [&](int j, int k) { dGw[(size_t)k * st] += gslot[wave][j][lane]; },
        [&](int k, T v) { dGw[(size_t)k * st] += v.d; }, mine);
  }
  __syncthreads();   // every share of dG written
  if (active)
    for (int k = wave; k < Tab::kC; k += W) {
      R g = dGi[(size_t)k * st];
      for (int w = 1; w < W; ++w) g += args.Gpart[((size_t)(w - 1) * rows + k) * st + i];
      dGi[(size_t)k * st] = g;
    }
}

}  // namespace mtp
