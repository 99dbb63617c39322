// Device-side pieces shared by the generated MTP evaluation kernels.
//
// Radial part, paper section 2.1, eqs. f_mu and radial-basis:
//   Q^(beta)(r) = T_{beta-1}(x) (R_cut - r)^2 for r < R_cut,
//   x = (2 r - R_min - R_cut) / (R_cut - R_min),
//   f_mu(r, z_i, z_j) = sum_beta c[mu][z_i][z_j][beta] Q^(beta)(r).
// Pairs handed to a kernel are always inside the cutoff (strict r < R_cut).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtp {

// One neighbour pair as stored in the ELL lists: r_ij = x_j + n.L - x_i and
// the neighbour's species, written and read as one 16-byte-aligned record.
template <typename T>
struct PairRec;
template <>
struct alignas(16) PairRec<double> {
  double x, y, z;
  int zj;
  int pad;
};
template <>
struct alignas(16) PairRec<float> {
  float x, y, z;
  int zj;
};

// Arguments of one evaluation launch.  Pair data uses an ELL layout: slot p of
// atom i lives at p * stride + i, so a wavefront of consecutive atoms reads and
// writes consecutive addresses for the same slot.
template <typename T>
struct EvalArgs {
  int n_atoms;
  int stride;          // >= n_atoms, row pitch of the ELL arrays
  int nq;              // radial basis size N_Q
  int n_species;       // S
  int n_c;             // n_mu * S * S * N_Q
  T rmin, rcut;
  double rmin64, rcut64; // the same in FP64 (radial arguments of the mixed-precision path)
  const int* nbr_count;  // [n_atoms]
  const PairRec<T>* pr;  // [K * stride] pair vectors and neighbour species
  const PairRec<double>* pr64;  // the same in FP64, read instead of pr by the moments
                                // passes of the mixed-precision path (else unused)
  const int* species;    // [n_atoms]
  const T* c;            // [n_mu][S][S][N_Q]
  const T* xi;           // [m] in the kernel's basis order
  T* site;               // [n_atoms]   site energies V_i
  T* M;                  // [C][stride] moment components of every atom
  const float* M32;      // the same in FP32, read instead of M by the contraction
                         // kernels of the mixed-precision path (else null)
  T* G;                  // [C][stride] dV_i / dM (moment components)
  T* g;                  // [K * stride][3] dV_i / dr_ij, packed per pair
  T* atom_virial;        // [9][stride]  sum_j g_a r_b
  double* own;          // [3][stride]  sum_j g_ij in FP64 (the atom's own share of its force)
  T* D;                  // [n_graphs][stride] dV_i / dg for every connected graph g
  T* Gpart;              // [partial_rows][stride] shares of the table-driven contraction's
                         // wavefronts (BasisVariant::partial_rows; null: one wavefront per atom)
  T* B;                  // [m][b_stride] optional basis values
  int b_stride;
};

// One pair's vector and neighbour species in the arithmetic type T: from
// the records of the evaluation's own precision, or (PR64, the moments of
// the mixed-precision path) from the FP64 records, rounded to T after the
// radial arguments were formed from them in FP64: the Chebyshev argument u
// of |r| and s = R_cut - |r| (a distance rounded to FP32 moves an atom by
// about 1e-7 A, and the steep radial functions turn that into force errors
// of tens of micro-eV/A; rounding u and s instead keeps them near 1e-6).
template <typename T>
struct PairVec {
  T x, y, z;
  T u, s;   // (PR64 only) Chebyshev argument and R_cut - |r|
  int zj;
};
template <typename T, bool PR64>
__device__ __forceinline__ PairVec<T> load_pair(const EvalArgs<T>& a, size_t e) {
  if constexpr (PR64) {
    const PairRec<double> q = a.pr64[e];
    const double r = sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
    const double span_inv = 1.0 / (a.rcut64 - a.rmin64);
    const double u = (2.0 * r - a.rmin64 - a.rcut64) * span_inv;
    return {(T)q.x, (T)q.y, (T)q.z, (T)u, (T)(a.rcut64 - r), q.zj};
  } else {
    const PairRec<T> q = a.pr[e];
    return {q.x, q.y, q.z, T(0), T(0), q.zj};
  }
}

// f_mu and, when DERIV, df_mu/dr for the NMU radial functions of one pair.
// cs points at c staged in LDS; base = ((0 * S + zi) * S + zj) * nq and the
// stride between consecutive mu is S * S * nq.
// NQ > 0 fixes the radial basis size at compile time (nq is then ignored
// and the recurrence is unrolled); NQ = 0 takes nq at run time.
// Fused multiply-add of the radial recurrences (overloaded for dual numbers
// further down).
__device__ __forceinline__ double fmadd(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return fmaf(a, b, c); }
template <typename R>
struct Dual;
template <typename R>
__device__ __forceinline__ Dual<R> fmadd(R a, Dual<R> b, Dual<R> c);

// radial_us takes the Chebyshev argument x of r, dx/dr and s = R_cut - r.
// CT: type of the coefficients (the arithmetic type, or its real part when T
// is a dual number).
template <typename T, int NMU, bool DERIV, int NQ = 0, typename CT = T>
__device__ __forceinline__ void radial_us(const CT* __restrict__ cs, int base, int mu_stride, int nq,
                                          T x, T s, T dxdr, T (&f)[NMU], T (&df)[NMU]) {
  if constexpr (NQ > 0) nq = NQ;
  T acc[NMU], dacc[NMU];
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) {
    acc[mu] = cs[base + mu * mu_stride];          // T_0 = 1
    dacc[mu] = T(0);
  }
  T t_prev = T(1), t_cur = x;                     // T_0, T_1
  T d_prev = T(0), d_cur = T(1);                  // dT_0/dx, dT_1/dx
#pragma unroll
  for (int b = 1; b < (NQ > 0 ? NQ : nq); ++b) {
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu) {
      const CT cb = cs[base + mu * mu_stride + b];
      acc[mu] = fmadd(cb, t_cur, acc[mu]);
      if (DERIV) dacc[mu] = fmadd(cb, d_cur, dacc[mu]);
    }
    const T t_next = T(2) * x * t_cur - t_prev;
    if (DERIV) {
      const T d_next = T(2) * t_cur + T(2) * x * d_cur - d_prev;
      d_prev = d_cur;
      d_cur = d_next;
    }
    t_prev = t_cur;
    t_cur = t_next;
  }
  const T s2 = s * s;
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) {
    f[mu] = acc[mu] * s2;
    if (DERIV) df[mu] = dacc[mu] * dxdr * s2 - T(2) * s * acc[mu];
  }
}

template <typename T, int NMU, bool DERIV, int NQ = 0, typename CT = T>
__device__ __forceinline__ void radial(const CT* __restrict__ cs, int base, int mu_stride, int nq,
                                       T r, T rmin, T rcut, T (&f)[NMU], T (&df)[NMU]) {
  const T span_inv = T(1) / (rcut - rmin);
  const T x = (T(2) * r - rmin - rcut) * span_inv;
  const T dxdr = T(2) * span_inv;
  radial_us<T, NMU, DERIV, NQ, CT>(cs, base, mu_stride, nq, x, rcut - r, dxdr, f, df);
}

// Sum over aligned groups of SPLIT consecutive lanes (SPLIT = 1, 2 or 4):
// DPP quad permutations [1,0,3,2] then [2,3,0,1], each a lane-to-lane move
// of the 32-bit halves inside a quad of lanes (every lane of a group ends
// with the group's sum, formed in the same order).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int SPLIT, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(SPLIT == 1 || SPLIT == 2 || SPLIT == 4, "groups of 1, 2 or 4 lanes");
  if constexpr (SPLIT >= 2) v = v + dpp_move<0xB1>(v);
  if constexpr (SPLIT >= 4) v = v + dpp_move<0x4E>(v);
  return v;
}

// Makes the values of a register array opaque to the optimiser (an empty asm
// that may rewrite them), so that products formed before it are not kept
// alive to be reused after it.
template <typename T, int N>
__device__ __forceinline__ void opaque(T (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("" : "+v"(v[k]));
}

// First-order dual number v + d e (e^2 = 0): running the contraction code on
// duals gives the directional derivative of every value along the tangent
// carried in d (forward mode over the reverse sweep for the loss gradient).
template <typename R>
struct Dual {
  R v, d;
  __device__ __forceinline__ Dual() = default;
  __device__ __forceinline__ constexpr Dual(R x) : v(x), d(R(0)) {}
  __device__ __forceinline__ constexpr Dual(R x, R y) : v(x), d(y) {}
};
template <typename R>
__device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) { return Dual<R>(a.v + b.v, a.d + b.d); }
template <typename R>
__device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b) { return Dual<R>(a.v * b.v, fma(a.d, b.v, a.v * b.d)); }
template <typename R>
__device__ __forceinline__ Dual<R> operator*(R a, Dual<R> b) { return Dual<R>(a * b.v, a * b.d); }
template <typename R>
__device__ __forceinline__ Dual<R>& operator+=(Dual<R>& a, Dual<R> b) { a.v += b.v; a.d += b.d; return a; }
template <typename R>
__device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) { return Dual<R>(a.v - b.v, a.d - b.d); }
template <typename R>
__device__ __forceinline__ Dual<R> operator/(Dual<R> a, Dual<R> b) {
  const R q = a.v / b.v;
  return Dual<R>(q, (a.d - q * b.d) / b.v);
}
template <typename R>
__device__ __forceinline__ Dual<R> dsqrt(Dual<R> a) {
  const R r = sqrt(a.v);
  return Dual<R>(r, a.d / (R(2) * r));
}
// a b + c with a real coefficient a (radial coefficients times a dual)
template <typename R>
__device__ __forceinline__ Dual<R> fmadd(R a, Dual<R> b, Dual<R> c) { return Dual<R>(fma(a, b.v, c.v), fma(a, b.d, c.d)); }

template <typename R, int N>
__device__ __forceinline__ void opaque(Dual<R> (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("" : "+v"(v[k].v), "+v"(v[k].d));
}

// Per-launch arguments of the loss-gradient kernels (all [.][stride] arrays
// are indexed like EvalArgs).
template <typename T>
struct LossArgs {
  const T* a_atom;     // [n_atoms] a_k = 2 w_e (E_k - E_k^t) of the atom's configuration
  const T* u;          // [n_atoms][3] u_i = -2 w_f (F_i - F_i^t)
  const T* eps_atom;   // [9][stride] eps_k = 2 w_s (W_k - W_k^t) of the atom's configuration
  const int* nbr;      // [K * stride] neighbour home index of slot p of atom i at p * stride + i
  int K;
  T* dM;               // [C][stride] tangent of the moments along delta r
  T* dG;               // [C][stride] tangent of G = dV/dM
  T* xi_terms;         // [m][stride] a B_alpha + tangent of B_alpha
  T* gd;               // [2 n_graphs][stride] graph values and tangents, then dV/dg and its tangent
  T* pa;               // [NMU][K * stride] per pair: coefficient of Q_beta
  T* pb;               // [NMU][K * stride] per pair: coefficient of dQ_beta/dr
  double* cpart;       // [blocks][n_c] partial sums of dL/dc per workgroup
  T* hvp;              // [K * stride][3] per pair: tangent of g = dV_i/dr_ij along delta r plus
                       // eps^T g (for dL/dx); null when the position gradient is not wanted
};

// Error-free sum (Knuth's TwoSum): hi + lo carries the accumulated sum.
template <typename T>
__device__ __forceinline__ void two_sum_acc(T& hi, T& lo, T v) {
  const T s = hi + v;
  const T bp = s - hi;
  const T err = (hi - (s - bp)) + (v - bp);
  hi = s;
  lo += err;
}

namespace {

// The per-atom sums of the final adjoint pass — the per-atom virial
// sum_p g_p (x) r_p and the atom's own force share sum_p g_p in FP64 — as a
// kernel of their own, one thread per atom over its pairs in slot order, for
// launches whose last pass is an earlier pass of a split (the later passes
// skipped by a degree mask): folding the twelve sums into that pass would
// make it spill.
template <typename T>
__global__ void __launch_bounds__(256) adjoint_sums_kernel(const EvalArgs<T> args) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= args.n_atoms) return;
  const int cnt = args.nbr_count[i];
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  T w0 = T(0), w1 = T(0), w2 = T(0), w3 = T(0), w4 = T(0), w5 = T(0), w6 = T(0), w7 = T(0), w8 = T(0);
#pragma unroll 4
  for (int p = 0; p < cnt; ++p) {
    const size_t e = (size_t)p * args.stride + i;
    const PairRec<T> q = args.pr[e];
    const T tx = args.g[3 * e], ty = args.g[3 * e + 1], tz = args.g[3 * e + 2];
    w0 += tx * q.x; w1 += tx * q.y; w2 += tx * q.z;
    w3 += ty * q.x; w4 += ty * q.y; w5 += ty * q.z;
    w6 += tz * q.x; w7 += tz * q.y; w8 += tz * q.z;
    o0 += (double)tx; o1 += (double)ty; o2 += (double)tz;
  }
  T* wv = args.atom_virial + i;
  const size_t st = args.stride;
  wv[0] = w0; wv[st] = w1; wv[2 * st] = w2; wv[3 * st] = w3; wv[4 * st] = w4;
  wv[5 * st] = w5; wv[6 * st] = w6; wv[7 * st] = w7; wv[8 * st] = w8;
  double* ow = args.own + i;
  ow[0] = o0; ow[st] = o1; ow[2 * st] = o2;
}

}  // namespace

}  // namespace mtp
