// FP64 dense kernels of the extrapolation grade (paper, section 2.3):
// the active-set inverse A^{-1} and c = b A^{-1}, gamma = max_j |c_j|,
// argmax_j |c_j| (lowest index on ties).
#include <hip/hip_runtime.h>

#include <mutex>
#include <math.h>

#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kGJBlock = 256;

// Gauss-Jordan elimination with partial pivoting on [A | I] (row-major,
// m x 2m); the right half ends as A^{-1}.  Columns of A are equilibrated
// first (A D, then D (AD)^{-1} = A^{-1}; D is kept in inv's first row until
// the end).  One launch per column for the scaling, two per step (pivot
// search, row swap and normalisation in one workgroup; elimination from
// every other row over the whole grid), two at the end.  A pivot at
// rounding level sets *singular, after which the later kernels return at
// once.

__global__ void __launch_bounds__(kGJBlock) gj_scale_kernel(int m, double* W, double* inv, int* singular) {
  __shared__ double red[kGJBlock];
  const int col = blockIdx.x, t = threadIdx.x;
  const int n2 = 2 * m;
  if (col == 0 && t == 0) *singular = 0;
  double mx = 0.0;
  for (int r = t; r < m; r += blockDim.x) mx = fmax(mx, fabs(W[(size_t)r * n2 + col]));
  red[t] = mx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double d = red[0] > 0 ? 1.0 / red[0] : 1.0;
  if (t == 0) inv[col] = d;
  for (int r = t; r < m; r += blockDim.x) W[(size_t)r * n2 + col] *= d;
}

// Step k: pivot = largest |W[r][k]| for r >= k (lowest row on ties), rows
// k and pivot swapped, row k divided by the pivot.
__global__ void __launch_bounds__(kGJBlock) gj_pivot_kernel(int m, int k, double* W, int* singular) {
  __shared__ double s_val[kGJBlock];
  __shared__ int s_idx[kGJBlock];
  __shared__ int s_stop;
  const int t = threadIdx.x;
  const int n2 = 2 * m;
  if (t == 0) s_stop = *singular;
  __syncthreads();
  if (s_stop) return;
  double best = -1;
  int bi = k;
  for (int r = k + t; r < m; r += blockDim.x) {
    const double v = fabs(W[(size_t)r * n2 + k]);
    if (v > best) { best = v; bi = r; }
  }
  s_val[t] = best;
  s_idx[t] = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) {
      const double v = s_val[t + w];
      const int ix = s_idx[t + w];
      if (v > s_val[t] || (v == s_val[t] && ix < s_idx[t])) { s_val[t] = v; s_idx[t] = ix; }
    }
    __syncthreads();
  }
  // columns are scaled to max |entry| = 1: a pivot at rounding level means
  // A is numerically singular
  if (!(s_val[0] > 1e-13)) {
    if (t == 0) *singular = 1;
    return;
  }
  const int pr = s_idx[0];
  if (pr != k)
    for (int col = t; col < n2; col += blockDim.x) {
      const double a = W[(size_t)k * n2 + col];
      W[(size_t)k * n2 + col] = W[(size_t)pr * n2 + col];
      W[(size_t)pr * n2 + col] = a;
    }
  __syncthreads();
  const double ip = 1.0 / W[(size_t)k * n2 + k];
  __syncthreads();
  for (int col = t; col < n2; col += blockDim.x) W[(size_t)k * n2 + col] *= ip;
}

// Step k: column k eliminated from every other row (one wavefront per row,
// lanes over the columns; the row's factor is read before any lane writes).
__global__ void __launch_bounds__(kGJBlock) gj_eliminate_kernel(int m, int k, double* W, const int* singular) {
  if (*singular) return;
  const int n2 = 2 * m;
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (kGJBlock / 64) + (threadIdx.x >> 6);
  if (r >= m || r == k) return;
  double* row = W + (size_t)r * n2;
  const double* prow = W + (size_t)k * n2;
  const double f = row[k];
  if (f != 0.0)
    for (int col = lane; col < n2; col += 64)
      if (col != k) row[col] -= f * prow[col];
  if (lane == 0) row[k] = 0.0;
}

// A^{-1} = D (AD)^{-1}: row r of the right half scaled by D[r], then copied.
__global__ void gj_unscale_kernel(int m, double* W, const double* inv, const int* singular) {
  if (*singular) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int r = (int)(idx / m), col = (int)(idx % m);
  W[(size_t)r * 2 * m + m + col] *= inv[r];
}

__global__ void gj_copy_kernel(int m, const double* W, double* inv, const int* singular) {
  if (*singular) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int r = (int)(idx / m), col = (int)(idx % m);
  inv[idx] = W[(size_t)r * 2 * m + m + col];
}

// c = b A^{-1} on the FP64 matrix cores: one wavefront per 16 x 16 tile of c;
// each v_mfma_f64_16x16x4 takes four k, lane l supplying b[row0 + l%16][k]
// and A^{-1}[k][col0 + l%16] for k = k0 + l/16 (zero past m), and lane l
// holds c[row0 + 4j + l/16][col0 + l%16] in slot j.  Then, per row, the max |c|
// and its first index.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) gemm_kernel(int n, int m, const double* __restrict__ b,
                                                   const double* __restrict__ A, double* __restrict__ c) {
  const int l = threadIdx.x & 63;
  const int tiles_m = (m + 15) / 16;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int row0 = (tile / tiles_m) * 16, col0 = (tile % tiles_m) * 16;
  if (row0 >= n) return;   // the whole wavefront
  const int ar = row0 + (l & 15), bc = col0 + (l & 15), kk = l >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += 4) {
    const int k = k0 + kk;
    const double x = (ar < n && k < m) ? b[(size_t)ar * m + k] : 0.0;
    const double y = (k < m && bc < m) ? A[(size_t)k * m + bc] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
  }
  for (int j = 0; j < 4; ++j) {
    const int r = row0 + 4 * j + kk;
    if (r < n && bc < m) c[(size_t)r * m + bc] = acc[j];
  }
}

__global__ void maxabs_kernel(int n, int m, const double* __restrict__ c, double* gamma, int32_t* arg) {
  const int row = blockIdx.x * blockDim.y + threadIdx.y;
  if (row >= n) return;
  const int lane = threadIdx.x;  // 64 lanes per row
  double best = -1;
  int bi = 0;
  for (int j = lane; j < m; j += 64) {
    const double v = fabs(c[(size_t)row * m + j]);
    if (v > best) { best = v; bi = j; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(best, off, 64);
    const int oi = __shfl_down(bi, off, 64);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (lane == 0) {
    gamma[row] = best;
    arg[row] = bi;
  }
}

}  // namespace

// Scratch of mtp_grade_from_b_noalloc: the product c = b A^{-1} of one call,
// in a fixed device array (one copy per GPU, kept until the process ends).
static __device__ __align__(256) double grade_scratch[kGradeScratchDoubles];

hipError_t grade_scratch_address(int device, double** out) {
  // The array's name is a host-side stand-in: its device address on the
  // current device comes from the runtime, once per device.
  static std::mutex mu;
  static double* addr[kMaxGradeDevices] = {};
  if (device < 0 || device >= kMaxGradeDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(grade_scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t gauss_jordan_inverse(int m, double* work, double* inv, int* singular, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_scale_kernel, dim3(m), dim3(kGJBlock), 0, s, m, work, inv, singular);
  const unsigned row_blocks = (unsigned)((m + kGJBlock / 64 - 1) / (kGJBlock / 64));
  for (int k = 0; k < m; ++k) {
    hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(kGJBlock), 0, s, m, k, work, singular);
    hipLaunchKernelGGL(gj_eliminate_kernel, dim3(row_blocks), dim3(kGJBlock), 0, s, m, k, work, singular);
  }
  const unsigned blocks = (unsigned)(((int64_t)m * m + 255) / 256);
  hipLaunchKernelGGL(gj_unscale_kernel, dim3(blocks), dim3(256), 0, s, m, work, inv, singular);
  hipLaunchKernelGGL(gj_copy_kernel, dim3(blocks), dim3(256), 0, s, m, work, inv, singular);
  return hipGetLastError();
}

hipError_t grade_rows(int n, int m, const double* b, const double* Ainv, double* gamma, int32_t* argmax,
                      double* c, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int tiles = ((n + 15) / 16) * ((m + 15) / 16);
  hipLaunchKernelGGL(gemm_kernel, dim3((tiles + 3) / 4), dim3(256), 0, s, n, m, b, Ainv, c);
  hipLaunchKernelGGL(maxabs_kernel, dim3((n + 3) / 4), dim3(64, 4), 0, s, n, m, c, gamma, argmax);
  return hipGetLastError();
}

hipError_t row_maxima(int n, int m, const double* c, double* gamma, int32_t* argmax, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(maxabs_kernel, dim3((n + 3) / 4), dim3(64, 4), 0, s, n, m, c, gamma, argmax);
  return hipGetLastError();
}

}  // namespace mtp
