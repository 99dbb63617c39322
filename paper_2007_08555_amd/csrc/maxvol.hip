// MaxVol selection of an active set from a pool of descriptor rows (paper,
// section 2.3: the step of Goreinov et al. that the paper cites for its
// query strategy).  For a pool B [K][m] and m selected rows A = B[rows],
// C = B A^{-1}; while the largest |C_ij| exceeds 1 + delta, row j of A is
// replaced by pool row i, which multiplies |det A| by |C_ij|.  After the
// swap C' = C - C[:, j] (C[i, :] - e_j) / C_ij, a rank-one update; C is
// recomputed from A^{-1} every few swaps and before the search may stop.
#include <hip/hip_runtime.h>

#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kMVBlock = 256;

// Starting rows: Gaussian elimination with partial pivoting of the pool with
// every column scaled to max |entry| = 1.  W [K][m] is overwritten; perm [K]
// holds the current row order.  Step t takes the first row, in the current
// order, of largest |W| in column t among positions t..K-1, swaps it into
// position t and eliminates column t below it.  The m pivot rows are
// returned in ascending order.  A zero pivot sets *singular, after which
// every later kernel of the elimination returns at once.  One launch per
// column for the scaling, then two per step (pivot search in one workgroup,
// elimination over the whole grid).

// perm = identity and column t scaled by 1 / max |W[:, t]| (one block per column).
__global__ void __launch_bounds__(kMVBlock) pr_scale_kernel(int K, int m, double* W, int32_t* perm, int* singular) {
  __shared__ double red[kMVBlock];
  const int col = blockIdx.x, tid = threadIdx.x;
  if (col == 0) {
    for (int r = tid; r < K; r += blockDim.x) perm[r] = r;
    if (tid == 0) *singular = 0;
  }
  double mx = 0.0;
  for (int r = tid; r < K; r += blockDim.x) mx = fmax(mx, fabs(W[(size_t)r * m + col]));
  red[tid] = mx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  mx = red[0];
  if (mx > 0.0)
    for (int r = tid; r < K; r += blockDim.x) W[(size_t)r * m + col] /= mx;
}

// Step t, pivot: largest |W[perm[p]][t]| over positions p >= t, the first one
// on ties, swapped into position t.
__global__ void __launch_bounds__(kMVBlock) pr_pivot_kernel(int K, int m, int t, const double* W, int32_t* perm,
                                                            int* singular) {
  __shared__ double bv[kMVBlock];
  __shared__ int bi[kMVBlock];
  if (*singular) return;
  const int tid = threadIdx.x;
  double best = -1.0;
  int bp = K;
  for (int p = t + tid; p < K; p += blockDim.x) {
    const double v = fabs(W[(size_t)perm[p] * m + t]);
    if (v > best) { best = v; bp = p; }
  }
  bv[tid] = best;
  bi[tid] = bp;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double ov = bv[tid + w];
      const int op = bi[tid + w];
      if (ov > bv[tid] || (ov == bv[tid] && op < bi[tid])) { bv[tid] = ov; bi[tid] = op; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (!(bv[0] > 0.0)) {
      *singular = 1;
    } else {
      const int p = bi[0];
      const int tmp = perm[t];
      perm[t] = perm[p];
      perm[p] = tmp;
    }
  }
}

// Step t, elimination of column t from the rows at positions t+1..K-1: one
// wavefront per row, lanes over the columns right of t.
__global__ void __launch_bounds__(kMVBlock) pr_eliminate_kernel(int K, int m, int t, double* W,
                                                                const int32_t* __restrict__ perm,
                                                                const int* singular) {
  if (*singular) return;
  const int lane = threadIdx.x & 63;
  const int r = t + 1 + blockIdx.x * (kMVBlock / 64) + (threadIdx.x >> 6);
  if (r >= K) return;
  const double* prow = W + (size_t)perm[t] * m;
  double* row = W + (size_t)perm[r] * m;
  const double l = row[t] / prow[t];
  for (int k = t + 1 + lane; k < m; k += 64) row[k] -= l * prow[k];
}

// The pivot rows in ascending order (they are distinct): rank by counting.
__global__ void __launch_bounds__(kMVBlock) pr_rank_kernel(int m, const int32_t* __restrict__ perm, int32_t* rows,
                                                           const int* singular) {
  if (*singular) return;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    const int v = perm[t];
    int rank = 0;
    for (int u = 0; u < m; ++u) rank += perm[u] < v ? 1 : 0;
    rows[rank] = v;
  }
}

// [A | I] with A = pool[rows], the input of the Gauss-Jordan inverse.
__global__ void gather_rows_kernel(int m, const double* __restrict__ pool, const int32_t* __restrict__ rows,
                                   double* W) {
  const int r = blockIdx.x;
  for (int k = threadIdx.x; k < 2 * m; k += blockDim.x)
    W[(size_t)r * 2 * m + k] = k < m ? pool[(size_t)rows[r] * m + k] : (k - m == r ? 1.0 : 0.0);
}

// Largest |C_ij| over the pool from the per-row maxima: (value, i, j), the
// lowest i on ties (row maxima already take the lowest j).
__global__ void __launch_bounds__(kMVBlock) argmax_rows_kernel(int K, const double* __restrict__ rowmax,
                                                               const int32_t* __restrict__ rowarg, MaxvolPick* out) {
  const int tid = threadIdx.x;
  __shared__ double bv[kMVBlock];
  __shared__ int bi[kMVBlock];
  double best = -1.0;
  int b = K;
  for (int i = tid; i < K; i += blockDim.x)
    if (rowmax[i] > best) { best = rowmax[i]; b = i; }
  bv[tid] = best;
  bi[tid] = b;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double ov = bv[tid + w];
      const int oi = bi[tid + w];
      if (ov > bv[tid] || (ov == bv[tid] && oi < bi[tid])) { bv[tid] = ov; bi[tid] = oi; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    out->value = bv[0];
    out->i = bi[0];
    out->j = bi[0] < K ? rowarg[bi[0]] : 0;
  }
}

// Swap of pool row i into position j: copies of column j and row i of C,
// then C -= C[:, j] (C[i, :] - e_j) / C_ij and rows[j] = i.
__global__ void swap_copy_kernel(int K, int m, const double* __restrict__ C, const MaxvolPick* pick, double* colj,
                                 double* rowi) {
  const int i = pick->i, j = pick->j;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < K) colj[q] = C[(size_t)q * m + j];
  if (q < m) rowi[q] = C[(size_t)i * m + q];
}

__global__ void swap_update_kernel(int K, int m, double* C, const MaxvolPick* pick, const double* __restrict__ colj,
                                   const double* __restrict__ rowi, int32_t* rows) {
  const int j = pick->j;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) rows[j] = pick->i;
  if (q >= (int64_t)K * m) return;
  const int r = (int)(q / m), k = (int)(q % m);
  const double cij = rowi[j];
  C[q] -= colj[r] * ((rowi[k] - (k == j ? 1.0 : 0.0)) / cij);
}

}  // namespace

hipError_t maxvol_pivot_rows(int K, int m, double* W, int32_t* perm, int32_t* rows, int* singular, hipStream_t s) {
  hipLaunchKernelGGL(pr_scale_kernel, dim3(m), dim3(kMVBlock), 0, s, K, m, W, perm, singular);
  for (int t = 0; t < m; ++t) {
    hipLaunchKernelGGL(pr_pivot_kernel, dim3(1), dim3(kMVBlock), 0, s, K, m, t, W, perm, singular);
    const int rows_below = K - t - 1;
    if (rows_below > 0)
      hipLaunchKernelGGL(pr_eliminate_kernel, dim3((rows_below + kMVBlock / 64 - 1) / (kMVBlock / 64)),
                         dim3(kMVBlock), 0, s, K, m, t, W, perm, singular);
  }
  hipLaunchKernelGGL(pr_rank_kernel, dim3(1), dim3(kMVBlock), 0, s, m, perm, rows, singular);
  return hipGetLastError();
}

hipError_t maxvol_gather(int m, const double* pool, const int32_t* rows, double* W, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(m), dim3(kMVBlock), 0, s, m, pool, rows, W);
  return hipGetLastError();
}

hipError_t maxvol_pick(int K, const double* rowmax, const int32_t* rowarg, MaxvolPick* out, hipStream_t s) {
  hipLaunchKernelGGL(argmax_rows_kernel, dim3(1), dim3(kMVBlock), 0, s, K, rowmax, rowarg, out);
  return hipGetLastError();
}

hipError_t maxvol_swap(int K, int m, double* C, const MaxvolPick* pick, double* colj, double* rowi, int32_t* rows,
                       hipStream_t s) {
  const int n1 = K > m ? K : m;
  hipLaunchKernelGGL(swap_copy_kernel, dim3((n1 + kMVBlock - 1) / kMVBlock), dim3(kMVBlock), 0, s, K, m, C, pick,
                     colj, rowi);
  const int64_t n2 = (int64_t)K * m;
  hipLaunchKernelGGL(swap_update_kernel, dim3((unsigned)((n2 + kMVBlock - 1) / kMVBlock)), dim3(kMVBlock), 0, s, K,
                     m, C, pick, colj, rowi, rows);
  return hipGetLastError();
}

}  // namespace mtp
