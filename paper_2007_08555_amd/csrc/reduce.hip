// Force gather and per-configuration reductions.
//
// With g_p = dV_i/dr_ij for pair p = (i -> j, image n) and rev(p) the pair
// (j -> i, image -n), the force F_i = -dE/dx_i = sum_{p of i} (g_p - g_rev(p)):
// V_i depends on x_i through every r_ij (dr_ij/dx_i = -I) and V_j depends on
// x_i through r_ji (dr_ji/dx_i = +I).  The gather is deterministic.
#include <hip/hip_runtime.h>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kBlock = 256;

// Atom block of workgroup b when workgroups go to XCD b % 8 in turn: XCD x
// takes the contiguous run of q + (x < r) blocks starting at x q + min(x, r)
// (q = n / 8, r = n % 8): a bijection of [0, n).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t x = b % kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

// Forces F_i = sum over slots p of (g_p - g_rev(p)): the first sum was taken
// in FP64 by the last adjoint pass (own, [3][stride]), so only the reverse
// pairs' g is fetched here, subtracted in FP64 in slot order.  Pairs are
// taken eight at a time so that the eight dependent loads g[rev[e]] are in
// flight together.  (The per-atom virials are summed by the last adjoint
// pass as well.)  The reverse pairs of a configuration's atoms lie in the
// records of that configuration, so consecutive blocks of atoms share cache
// lines: workgroups are dispatched to the eight XCDs in turn, each with its
// own L2, and block b takes the atom block xcd_block(b), which keeps runs of
// consecutive atom blocks on one XCD.
template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(int64_t n_atoms, int stride,
                                                        const int32_t* __restrict__ count,
                                                        const int32_t* __restrict__ rev,
                                                        const T* __restrict__ g, const double* __restrict__ own,
                                                        double* __restrict__ F) {
  constexpr int U = 8;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  double fx = own[i], fy = own[stride + i], fz = own[2 * (size_t)stride + i];
  const int c = count[i];
  for (int p0 = 0; p0 < c; p0 += U) {
    double hx[U], hy[U], hz[U];
    size_t q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = (size_t)rev[(size_t)(p0 + u < c ? p0 + u : p0) * stride + i];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      hx[u] = (double)g[3 * q[u]]; hy[u] = (double)g[3 * q[u] + 1]; hz[u] = (double)g[3 * q[u] + 2];
    }
    // a select, not a branch: the loads above stay unconditional and issue
    // together (slots past the count were loaded at a clamped index)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = p0 + u < c;
      fx = ok ? fx - hx[u] : fx;
      fy = ok ? fy - hy[u] : fy;
      fz = ok ? fz - hz[u] : fz;
    }
  }
  F[3 * i] = fx;
  F[3 * i + 1] = fy;
  F[3 * i + 2] = fz;
}

// Per-configuration sums (site energies -> E_k, per-atom virials -> W_k,
// basis values -> b_k) as segmented row sums.  Every configuration is cut
// into chunks of kChunk atoms from its first atom; each chunk is one work
// item (one workgroup).  A workgroup's wavefronts take kRowU rows at a time, the
// lanes every 64th atom of the chunk, and the 64 partial sums are combined by
// a butterfly; a configuration of one chunk writes its sums directly, a
// larger one writes a partial per chunk that rows_finish_kernel adds in chunk
// order.  The order of every sum is fixed by the configuration's size alone
// (bitwise repeatable, and the same for a configuration evaluated alone), and
// a configuration of any size is spread over ceil(n / kChunk) workgroups.
constexpr int kChunk = 1024;
constexpr int kRowWaves = kBlock / 64;
constexpr int kRowU = 4;

// item_start[k] = first work item of configuration k (n_cfg + 1 entries),
// item_cfg[item] = its configuration; items past max_items are not recorded
// (only reachable with invalid atom offsets, which the search reports).
__global__ void __launch_bounds__(1024) chunk_items_kernel(int n_cfg, const CfgInfo* __restrict__ cfg,
                                                           int max_items, int32_t* item_start, int32_t* item_cfg) {
  __shared__ int32_t sc[1024];
  const int t = threadIdx.x;
  int base = 0;
  for (int k0 = 0; k0 < n_cfg; k0 += 1024) {
    const int k = k0 + t;
    const int n = k < n_cfg ? cfg[k].n : 0;
    const int cnt = k < n_cfg ? (n > kChunk ? (n + kChunk - 1) / kChunk : 1) : 0;
    sc[t] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan (Hillis-Steele)
      const int v = t >= off ? sc[t - off] : 0;
      __syncthreads();
      sc[t] += v;
      __syncthreads();
    }
    const int first = base + sc[t] - cnt;
    if (k < n_cfg) {
      item_start[k] = first;
      for (int c = 0; c < cnt && first + c < max_items; ++c) item_cfg[first + c] = k;
    }
    base += sc[1023];
    __syncthreads();
  }
  if (t == 0) item_start[n_cfg] = base;
}

// Rows: 0 the site energies, then (has_v) the nine per-atom virial
// components, then (B) the m basis values in file order (perm).
struct RowSums {
  int n_cfg, stride, n_rows, has_v, m, b_stride, max_items;
  const CfgInfo* cfg;
  const void* site;
  const void* wv;
  const void* B;
  const int32_t* perm;
  const int32_t* item_start;
  const int32_t* item_cfg;
  double* partial;   // [max_items][n_rows]
  double *energy, *virial, *b, *site_out;
};

template <typename T>
__device__ inline const T* row_ptr(const RowSums& a, int r) {
  if (r == 0) return (const T*)a.site;
  if (a.has_v && r <= 9) return (const T*)a.wv + (size_t)(r - 1) * a.stride;
  return (const T*)a.B + (size_t)a.perm[r - 1 - 9 * a.has_v] * a.b_stride;
}

__device__ inline void row_out(const RowSums& a, int k, int r, double v) {
  if (r == 0) {
    if (a.energy) a.energy[k] = v;
  } else if (a.has_v && r <= 9) {
    if (a.virial) a.virial[9 * k + r - 1] = v;
  } else {
    a.b[(size_t)k * a.m + r - 1 - 9 * a.has_v] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) rows_kernel(RowSums a) {
  const int item = blockIdx.x;
  const int total = a.item_start[a.n_cfg];
  if (item >= total || item >= a.max_items) return;
  const int k = a.item_cfg[item];
  const int first = a.item_start[k], items = a.item_start[k + 1] - first;
  const int64_t end = a.cfg[k].start + a.cfg[k].n;
  const int64_t c0 = a.cfg[k].start + (int64_t)(item - first) * kChunk;
  const int64_t c1 = c0 + kChunk < end ? c0 + kChunk : end;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r0 = wave * kRowU; r0 < a.n_rows; r0 += kRowWaves * kRowU) {
    const T* row[kRowU];
    double s[kRowU];
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      row[u] = row_ptr<T>(a, r0 + u < a.n_rows ? r0 + u : r0);
      s[u] = 0.0;
    }
    for (int64_t i = c0 + lane; i < c1; i += 64) {
      double v[kRowU];
#pragma unroll
      for (int u = 0; u < kRowU; ++u) v[u] = (double)row[u][i];
#pragma unroll
      for (int u = 0; u < kRowU; ++u) s[u] += v[u];
      if (r0 == 0 && a.site_out) a.site_out[i] = v[0];
    }
#pragma unroll
    for (int u = 0; u < kRowU; ++u)
      for (int o = 32; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, 64);
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < kRowU; ++u) {
        if (r0 + u >= a.n_rows) break;
        if (items == 1)
          row_out(a, k, r0 + u, s[u]);
        else
          a.partial[(size_t)item * a.n_rows + r0 + u] = s[u];
      }
  }
}

// Configurations of several chunks: one thread per (configuration, row)
// adds the chunk partials in chunk order.
__global__ void __launch_bounds__(kBlock) rows_finish_kernel(RowSums a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.n_cfg * a.n_rows) return;
  const int k = (int)(t / a.n_rows), r = (int)(t - (int64_t)k * a.n_rows);
  const int i0 = a.item_start[k], i1 = a.item_start[k + 1];
  if (i1 - i0 <= 1) return;
  double v = 0.0;
  for (int it = i0; it < i1 && it < a.max_items; ++it) v += a.partial[(size_t)it * a.n_rows + r];
  row_out(a, k, r, v);
}

}  // namespace

hipError_t gather_forces(int fp64, int64_t n_atoms, int stride, const int32_t* count,
                         const int32_t* rev, const void* gp, const double* own, double* forces, hipStream_t s) {
  if (n_atoms == 0 || !forces) return hipSuccess;
  const dim3 g((unsigned)((n_atoms + kBlock - 1) / kBlock));
  if (fp64)
    hipLaunchKernelGGL(gather_kernel<double>, g, dim3(kBlock), 0, s, n_atoms, stride, count, rev,
                       (const double*)gp, own, forces);
  else
    hipLaunchKernelGGL(gather_kernel<float>, g, dim3(kBlock), 0, s, n_atoms, stride, count, rev,
                       (const float*)gp, own, forces);
  return hipGetLastError();
}

int reduce_max_items(int n_cfg, int64_t n_atoms) {
  return (int)((n_atoms + kChunk - 1) / kChunk) + n_cfg;
}

int reduce_rows(int has_virial, int m, bool b) { return 1 + (has_virial ? 9 : 0) + (b ? m : 0); }

hipError_t reduce_items(int n_cfg, const CfgInfo* cfg, int max_items, int32_t* item_start, int32_t* item_cfg,
                        hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_items_kernel, dim3(1), dim3(1024), 0, s, n_cfg, cfg, max_items, item_start, item_cfg);
  return hipGetLastError();
}

hipError_t reduce_configs(int fp64, int n_cfg, const CfgInfo* offs, int stride, const void* site,
                          const void* atom_virial, const void* B, int m, int b_stride,
                          const int32_t* perm, double* energy, double* virial, double* b,
                          double* site_out, const ReduceItems& it, hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  const bool want_b = b && B;
  const bool has_v = virial && atom_virial;
  if (!energy && !has_v && !site_out && !want_b) return hipSuccess;
  RowSums a;
  a.n_cfg = n_cfg;
  a.stride = stride;
  a.has_v = has_v ? 1 : 0;
  a.m = m;
  a.n_rows = reduce_rows(a.has_v, m, want_b);
  a.b_stride = b_stride;
  a.max_items = it.max_items;
  a.cfg = offs;
  a.site = site;
  a.wv = atom_virial;
  a.B = B;
  a.perm = perm;
  a.item_start = it.item_start;
  a.item_cfg = it.item_cfg;
  a.partial = it.partial;
  a.energy = energy;
  a.virial = has_v ? virial : nullptr;
  a.b = want_b ? b : nullptr;
  a.site_out = site_out;
  if (fp64)
    hipLaunchKernelGGL(rows_kernel<double>, dim3(it.max_items), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(rows_kernel<float>, dim3(it.max_items), dim3(kBlock), 0, s, a);
  const int64_t fin = (int64_t)n_cfg * a.n_rows;
  hipLaunchKernelGGL(rows_finish_kernel, dim3((unsigned)((fin + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace mtp
