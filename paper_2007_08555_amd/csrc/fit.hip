// Normal equations of the training problem in xi at fixed radial
// coefficients c (paper, section 2.2, eq. Fitting).  E, f and the virial are
// linear in xi (eq. for V_i is a linear combination of the B_alpha), so with
// J the Jacobian of every predicted quantity with respect to xi, y the
// targets and W the diagonal of per-row weights, the loss is
//   L(xi) = (J xi - y)^T W (J xi - y) = xi^T H xi - 2 g^T xi + yy
// with H = J^T W J, g = J^T W y, yy = y^T W y, and its minimiser solves
// H xi = g.
//
// Row order of J and y, per batch of K configurations and N atoms:
// K energies, then 3 N force components (atom-major), then 9 K virial
// components (configuration-major).  Column alpha of J (file basis order)
// holds the energies, forces and virials of the potential with xi = e_alpha;
// column m holds y, so one Gram product of [J | y] gives H, g and yy.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 16;  // output tile of the Gram product (16 x 16 entries)
constexpr int kRows = 64;  // rows of [J | y] staged in LDS per step

// Per-row weight w_r and target y_r (column m of Ja).
__global__ void fit_rows_kernel(int n_cfg, int64_t N, int64_t R, const CfgInfo* cfg, const int32_t* atom_cfg,
                                double we, double wf, double ws, int scaling, const double* Et, const double* Ft,
                                const double* Wt, double* w, double* y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int k, kind;  // kind: 0 energy, 1 force, 2 virial
  double t;
  if (r < n_cfg) {
    k = (int)r; t = Et[k]; kind = 0;
  } else if (r < n_cfg + 3 * N) {
    const int64_t q = r - n_cfg;
    k = atom_cfg[q / 3]; t = Ft[q]; kind = 1;
  } else {
    const int64_t q = r - n_cfg - 3 * N;
    k = (int)(q / 9); t = Wt[q]; kind = 2;
  }
  const CfgInfo& c = cfg[k];
  double a = 0, b = 0, d = 0;
  if (c.n > 0) weights(scaling, (double)c.n, we, wf, ws, a, b, d);
  const double wr = kind == 0 ? a : (kind == 1 ? b : (c.pbc ? d : 0.0));
  w[r] = wr;
  // a cluster's virial row carries no weight; its target is not read
  y[r] = wr != 0.0 ? t : 0.0;
}

// Partial Gram products P[s] = Ja^T diag(w) Ja over the rows of split s, for
// the output tiles (ta, tb) with ta <= tb, on the FP64 matrix cores: one
// wavefront per tile pair and split.  Rows are staged kRows at a time in LDS
// (coalesced along the rows of the column-major Ja [n][R]); each
// v_mfma_f64_16x16x4 takes four of them, lane l supplying
// w[r] Ja[ta*16 + l%16][r] and Ja[tb*16 + l%16][r] for r = r0 + l/16, and
// lane l holds entry (4j + l/16, l%16) of the tile in slot j.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(64) gram_kernel(int n, int64_t R, int64_t rows_per_split,
                                                  const double* __restrict__ Ja, const double* __restrict__ w,
                                                  double* __restrict__ P) {
  __shared__ double sa[kTile][kRows + 1];
  __shared__ double sb[kTile][kRows + 1];
  // tile pair of this workgroup: blockIdx.x enumerates ta <= tb row by row
  const int nt = (n + kTile - 1) / kTile;
  int ta = 0, rem = blockIdx.x;
  while (rem >= nt - ta) {
    rem -= nt - ta;
    ++ta;
  }
  const int tb = ta + rem;
  const int l = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = min(R, r0 + rows_per_split);
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r0; rb < r1; rb += kRows) {
    for (int e = l; e < kTile * kRows; e += 64) {
      const int col = e / kRows, rr = e % kRows;
      const int64_t row = rb + rr;
      const bool in = row < r1;
      const int ca = ta * kTile + col, cb = tb * kTile + col;
      sa[col][rr] = (in && ca < n) ? Ja[(size_t)ca * R + row] * w[row] : 0.0;
      sb[col][rr] = (in && cb < n) ? Ja[(size_t)cb * R + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k0 = 0; k0 < kRows; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[l & 15][k0 + (l >> 4)], sb[l & 15][k0 + (l >> 4)], acc, 0, 0, 0);
    __syncthreads();
  }
  const int cb = tb * kTile + (l & 15);
  for (int j = 0; j < 4; ++j) {
    const int ca = ta * kTile + 4 * j + (l >> 4);
    if (ca < n && cb < n) P[(size_t)blockIdx.y * n * n + (size_t)ca * n + cb] = acc[j];
  }
}

// Sum of the partials in split order (deterministic); H [m][m], g [m], yy.
__global__ void gram_reduce_kernel(int n, int splits, const double* __restrict__ P, int accumulate, double* H,
                                   double* g, double* yy) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int a = idx / n, b = idx % n;
  // (min, max) lies in a tile pair with ta <= tb; reading the same entry for
  // (a, b) and (b, a) keeps H exactly symmetric
  const int lo = min(a, b), hi = max(a, b);
  double s = 0.0;
  for (int q = 0; q < splits; ++q) s += P[(size_t)q * n * n + (size_t)lo * n + hi];
  const int m = n - 1;
  double* dst = nullptr;
  if (a < m && b < m) dst = H + (size_t)a * m + b;
  else if (a < m && b == m) dst = g ? g + a : nullptr;
  else if (a == m && b == m) dst = yy;
  if (dst) *dst = accumulate ? *dst + s : s;
}

// Column k of the identity in rows: eye[k][j] = (j == k).
template <typename T>
__global__ void eye_kernel(int m, T* eye) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < m * m) eye[idx] = (idx / m == idx % m) ? T(1) : T(0);
}

// D_a = 1 / sqrt(H_aa) (1 where H_aa <= 0); [D H D | I] for Gauss-Jordan.
__global__ void solve_fill_kernel(int m, const double* H, double* D, double* W2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int r = idx / m, c = idx % m;
  const double hr = H[(size_t)r * m + r], hc = H[(size_t)c * m + c];
  const double dr = hr > 0 ? 1.0 / sqrt(hr) : 1.0, dc = hc > 0 ? 1.0 / sqrt(hc) : 1.0;
  W2[(size_t)r * 2 * m + c] = dr * H[(size_t)r * m + c] * dc;
  W2[(size_t)r * 2 * m + m + c] = r == c ? 1.0 : 0.0;
  if (c == 0) D[r] = dr;
}

// xi = D (D H D)^{-1} D g, one thread per entry, fixed summation order.
__global__ void solve_apply_kernel(int m, const double* inv, const double* D, const double* g, double* xi) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  double s = 0.0;
  for (int b = 0; b < m; ++b) s = fma(inv[(size_t)a * m + b], D[b] * g[b], s);
  xi[a] = D[a] * s;
}

}  // namespace

hipError_t fit_rows(int n_cfg, int64_t N, int64_t R, const CfgInfo* cfg, const int32_t* atom_cfg, double we,
                    double wf, double ws, int scaling, const double* Et, const double* Ft, const double* Wt,
                    double* w, double* y, hipStream_t s) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(fit_rows_kernel, dim3((unsigned)((R + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n_cfg, N,
                     R, cfg, atom_cfg, we, wf, ws, scaling, Et, Ft, Wt, w, y);
  return hipGetLastError();
}

int gram_splits(int n, int64_t R) {
  const int nt = (n + kTile - 1) / kTile;
  const int pairs = nt * (nt + 1) / 2;
  // about 4096 workgroups, each over at least 256 rows
  int64_t sp = (4096 + pairs - 1) / pairs;
  sp = std::min<int64_t>(sp, (R + 255) / 256);
  return (int)std::max<int64_t>(1, sp);
}

hipError_t gram(int n, int64_t R, const double* Ja, const double* w, double* P, int splits, int accumulate,
                double* H, double* g, double* yy, hipStream_t s) {
  const int nt = (n + kTile - 1) / kTile;
  const int pairs = nt * (nt + 1) / 2;
  const int64_t per = (R + splits - 1) / splits;
  hipLaunchKernelGGL(gram_kernel, dim3(pairs, splits), dim3(64), 0, s, n, R, per, Ja, w, P);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((n * n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, splits, P,
                     accumulate, H, g, yy);
  return hipGetLastError();
}

hipError_t fill_eye(int fp64, int m, void* eye, hipStream_t s) {
  const dim3 grid((m * m + kBlock - 1) / kBlock);
  if (fp64)
    hipLaunchKernelGGL(eye_kernel<double>, grid, dim3(kBlock), 0, s, m, (double*)eye);
  else
    hipLaunchKernelGGL(eye_kernel<float>, grid, dim3(kBlock), 0, s, m, (float*)eye);
  return hipGetLastError();
}

hipError_t solve_prepare(int m, const double* H, double* D, double* W2, hipStream_t s) {
  hipLaunchKernelGGL(solve_fill_kernel, dim3((m * m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m, H, D, W2);
  return hipGetLastError();
}

hipError_t solve_apply(int m, const double* inv, const double* D, const double* g, double* xi, hipStream_t s) {
  hipLaunchKernelGGL(solve_apply_kernel, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m, inv, D, g, xi);
  return hipGetLastError();
}

}  // namespace mtp
