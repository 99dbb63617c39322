// Residuals and final reductions of the training loss (paper, section 2.2,
// eq. Fitting with the weightings of eqs. train-structures and
// train-vibrations).  The stress term uses the extensive virial W = dE/d eps
// (eV); configurations without periodicity have no stress term.
//
// With a_k = 2 w_e (E_k - E_k^t), u_i = -2 w_f (F_i - F_i^t) and
// eps_k = 2 w_s (W_k - W_k^t) held fixed, dL/dtheta equals the theta-derivative
// of S = sum_k a_k E_k + sum_pairs g_ij . (u_j - u_i + eps_k r_ij): the force
// term through the directional derivative of E along the displacement field u,
// the stress term through the one along the strain eps.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kBlock = 256;

__global__ void residual_config_kernel(LossResidualArgs r) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.n_cfg) return;
  const CfgInfo& c = r.cfg[k];
  double we = 0, wf = 0, ws = 0;
  if (c.n > 0) weights(r.scaling, (double)c.n, r.we, r.wf, r.ws, we, wf, ws);
  const double dE = r.E[k] - r.Et[k];
  double loss = we * dE * dE;
  r.a_cfg[k] = 2.0 * we * dE;
  r.wf_cfg[k] = wf;
  for (int t = 0; t < 9; ++t) {
    double e = 0.0;
    if (c.pbc) {
      const double dW = r.W[9 * k + t] - r.Wt[9 * k + t];
      loss += ws * dW * dW;
      e = 2.0 * ws * dW;
    }
    r.eps_cfg[9 * k + t] = e;
  }
  r.loss_cfg[k] = loss;
}

template <typename T>
__global__ void residual_atom_kernel(LossResidualArgs r, T* a_atom, T* u, T* eps_atom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r.N) return;
  const int k = r.atom_cfg[i];
  const double wf = r.wf_cfg[k];
  double loss = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double dF = r.F[3 * i + d] - r.Ft[3 * i + d];
    loss += wf * dF * dF;
    u[3 * i + d] = (T)(-2.0 * wf * dF);
  }
  r.loss_atom[i] = loss;
  a_atom[i] = (T)r.a_cfg[k];
  for (int t = 0; t < 9; ++t) eps_atom[(size_t)t * r.stride + i] = (T)r.eps_cfg[9 * k + t];
}

// Sum of n values in a fixed order: strided per-thread partial sums, then a
// tree over the workgroup.
__device__ double block_sum(double v) {
  __shared__ double red[kBlock];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// Two-level sums in a fixed order, spread over the GPU (one workgroup
// summing a long array waits on its loads one round after another): first
// kSplit partial sums per output over contiguous chunks, then the partials in
// chunk order.  kSplit workgroups per output.
constexpr int kSplit = 32;

// Partial sums of the loss terms: the configuration terms followed by the
// atom terms, as one array of n_cfg + N values cut into kSplit chunks.
__global__ void __launch_bounds__(kBlock) loss_part_kernel(int n_cfg, int64_t N, const double* loss_cfg,
                                                           const double* loss_atom, double* part) {
  const int64_t total = n_cfg + N;
  const int64_t chunk = (total + kSplit - 1) / kSplit;
  const int64_t a0 = blockIdx.x * chunk, a1 = std::min(total, a0 + chunk);
  double v = 0.0;
  for (int64_t t = a0 + threadIdx.x; t < a1; t += blockDim.x) v += t < n_cfg ? loss_cfg[t] : loss_atom[t - n_cfg];
  const double s = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// grad_xi[f] = sum over atoms of xi_terms[perm[f]][atom]: workgroup (f, c)
// sums chunk c of row f.
template <typename T>
__global__ void __launch_bounds__(kBlock) grad_xi_part_kernel(int64_t N, int stride, const T* xi_terms,
                                                              const int32_t* perm, double* part) {
  const int f = blockIdx.x, c = blockIdx.y;
  const T* row = xi_terms + (size_t)perm[f] * stride;
  const int64_t chunk = (N + kSplit - 1) / kSplit;
  const int64_t a0 = c * chunk, a1 = std::min(N, a0 + chunk);
  double v = 0.0;
  for (int64_t i = a0 + threadIdx.x; i < a1; i += blockDim.x) v += (double)row[i];
  const double s = block_sum(v);
  if (threadIdx.x == 0) part[(size_t)f * kSplit + c] = s;
}

// out[r] = sum over c of part[r][c] in order, for n rows.
__global__ void part_sum_kernel(int n, const double* part, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double v = 0.0;
  for (int c = 0; c < kSplit; ++c) v += part[(size_t)r * kSplit + c];
  out[r] = v;
}

// grad_c[t] = sum over workgroups b of cpart[b][t], b in order per thread
// (strided), then a tree over the workgroup: one workgroup per entry t.
__global__ void __launch_bounds__(kBlock) grad_c_kernel(int n_blocks, int n_c, const double* cpart, double* grad) {
  const int t = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) v += cpart[(size_t)b * n_c + t];
  const double s = block_sum(v);
  if (threadIdx.x == 0) grad[t] = s;
}

// Rows of the nonlinear grade (section 2.3): dE_k/dtheta of every
// configuration.  With a_i = 1, u = 0 and eps = 0 the loss kernels differentiate
// S = sum_k E_k and leave, per pair, the coefficients pa_mu and pb_mu of
// Q_beta and dQ_beta/dr in dV_i/dc; summed per configuration (not per
// workgroup) they give dE_k/dc.  The xi part of the row is b_k.
template <typename T>
__global__ void unit_weights_kernel(int64_t N, int64_t n_eps, T* a_atom, T* u, T* eps_atom) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) a_atom[t] = T(1);
  if (t < 3 * N) u[t] = T(0);
  if (t < n_eps) eps_atom[t] = T(0);
}

// One workgroup per configuration; threads over its atoms.  One pass per
// c block (z_i, z_j, mu): each thread sums, in order, the contributions of
// its atoms of species z_i and their pairs with neighbours of species z_j to
// the N_Q entries of the block, then the thread sums are added in thread
// order (no atomics: the rows are bitwise repeatable).  LDS: [nq][kBlock].
template <typename T>
__global__ void __launch_bounds__(kBlock) c_rows_kernel(const ThetaRowArgs a, const PairRec<T>* __restrict__ pr,
                                                        const T* __restrict__ pa, const T* __restrict__ pb) {
  extern __shared__ double tile[];   // [nq][kBlock]
  const int k = blockIdx.x;
  const int64_t a0 = a.cfg[k].start, a1 = a0 + a.cfg[k].n;
  const size_t n_slots = (size_t)a.K * a.stride;
  const double span_inv = 1.0 / (a.rcut - a.rmin), dxdr = 2.0 * span_inv;
  const int S = a.n_species, nq = a.nq;
  double* row = a.rows + (size_t)k * (a.m + a.n_c) + a.m;
  for (int zi = 0; zi < S; ++zi)
    for (int zj = 0; zj < S; ++zj)
      for (int mu = 0; mu < a.n_mu; ++mu) {
        double acc[16];
        for (int b = 0; b < 16; ++b) acc[b] = 0.0;
        for (int64_t i = a0 + threadIdx.x; i < a1; i += blockDim.x) {
          int z = a.species[i];
          z = z < 0 ? 0 : (z >= S ? S - 1 : z);
          if (z != zi) continue;
          const int cnt = a.count[i];
          for (int p = 0; p < cnt; ++p) {
            const size_t e = (size_t)p * a.stride + i;
            const PairRec<T> q = pr[e];
            if (q.zj != zj) continue;
            const double x = q.x, y = q.y, zz = q.z;
            const double r = sqrt(x * x + y * y + zz * zz);
            const double sc = a.rcut - r;
            const double xq = (2.0 * r - a.rmin - a.rcut) * span_inv;
            const double va = (double)pa[(size_t)mu * n_slots + e], vb = (double)pb[(size_t)mu * n_slots + e];
            // Chebyshev T_b(xq) and dT_b/dxq by their three-term recurrences
            double t0 = 1.0, t1 = xq, d0 = 0.0, d1 = 1.0;
#pragma unroll
            for (int b = 0; b < 16; ++b) {
              if (b < nq) {
                const double tb = b == 0 ? t0 : t1, db = b == 0 ? d0 : d1;
                acc[b] += va * (tb * sc * sc) + vb * (db * dxdr * sc * sc - 2.0 * tb * sc);
                if (b >= 1) {
                  const double t2 = 2.0 * xq * t1 - t0, d2 = 2.0 * t1 + 2.0 * xq * d1 - d0;
                  t0 = t1; t1 = t2; d0 = d1; d1 = d2;
                }
              }
            }
          }
        }
#pragma unroll
        for (int b = 0; b < 16; ++b)
          if (b < nq) tile[(size_t)b * kBlock + threadIdx.x] = acc[b];
        __syncthreads();
        for (int b = threadIdx.x; b < nq; b += blockDim.x) {
          double v = 0.0;
          for (int l = 0; l < kBlock; ++l) v += tile[(size_t)b * kBlock + l];
          row[((mu * S + zi) * S + zj) * nq + b] = v;
        }
        __syncthreads();
      }
}

__global__ void copy_b_kernel(int n_cfg, int m, int n_c, const double* __restrict__ b, double* rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_cfg * m) return;
  rows[(t / m) * (m + n_c) + t % m] = b[t];
}

// dL/dx_i = -a_i F_i - (sum over the slots p of atom i of hvp_p - sum of
// hvp at the reverse slots), in FP64: the energy term (dE_k/dx_i = -F_i)
// and the derivative of S_u = sum over pairs of g . delta r through the pair
// vectors (r_ij = x_j - x_i), whose per-pair values the position passes left
// in hvp.
template <typename T>
__global__ void __launch_bounds__(kBlock) grad_pos_kernel(int64_t N, int stride, const int32_t* __restrict__ count,
                                                          const int32_t* __restrict__ rev, const T* __restrict__ hvp,
                                                          const T* __restrict__ a_atom, const double* __restrict__ F,
                                                          double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double a = (double)a_atom[i];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const int c = count[i];
  for (int p = 0; p < c; ++p) {
    const size_t e = (size_t)p * stride + i;
    const size_t q = (size_t)rev[e];
    s0 += (double)hvp[3 * e] - (double)hvp[3 * q];
    s1 += (double)hvp[3 * e + 1] - (double)hvp[3 * q + 1];
    s2 += (double)hvp[3 * e + 2] - (double)hvp[3 * q + 2];
  }
  out[3 * i] = -a * F[3 * i] - s0;
  out[3 * i + 1] = -a * F[3 * i + 1] - s1;
  out[3 * i + 2] = -a * F[3 * i + 2] - s2;
}

}  // namespace

hipError_t loss_grad_pos(int fp64, int64_t N, int stride, const int32_t* count, const int32_t* rev, const void* hvp,
                         const void* a_atom, const double* F, double* out, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const dim3 g((unsigned)((N + kBlock - 1) / kBlock));
  if (fp64)
    hipLaunchKernelGGL(grad_pos_kernel<double>, g, dim3(kBlock), 0, s, N, stride, count, rev, (const double*)hvp,
                       (const double*)a_atom, F, out);
  else
    hipLaunchKernelGGL(grad_pos_kernel<float>, g, dim3(kBlock), 0, s, N, stride, count, rev, (const float*)hvp,
                       (const float*)a_atom, F, out);
  return hipGetLastError();
}

hipError_t loss_residuals(LossResidualArgs& r, int fp64, void* a_atom, void* u, void* eps_atom, hipStream_t s) {
  if (r.n_cfg > 0)
    hipLaunchKernelGGL(residual_config_kernel, dim3((r.n_cfg + kBlock - 1) / kBlock), dim3(kBlock), 0, s, r);
  if (r.N > 0) {
    const dim3 g((unsigned)((r.N + kBlock - 1) / kBlock));
    if (fp64)
      hipLaunchKernelGGL(residual_atom_kernel<double>, g, dim3(kBlock), 0, s, r, (double*)a_atom, (double*)u,
                         (double*)eps_atom);
    else
      hipLaunchKernelGGL(residual_atom_kernel<float>, g, dim3(kBlock), 0, s, r, (float*)a_atom, (float*)u,
                         (float*)eps_atom);
  }
  return hipGetLastError();
}

hipError_t loss_finish(int fp64, int n_cfg, int64_t N, int stride, int m, int n_c, int n_blocks,
                       const double* loss_cfg, const double* loss_atom, const void* xi_terms, const int32_t* perm,
                       const double* cpart, double* part, double* loss, double* grad, hipStream_t s) {
  double* part_xi = part + kSplit;
  hipLaunchKernelGGL(loss_part_kernel, dim3(kSplit), dim3(kBlock), 0, s, n_cfg, N, loss_cfg, loss_atom, part);
  hipLaunchKernelGGL(part_sum_kernel, dim3(1), dim3(64), 0, s, 1, part, loss);
  if (N > 0) {
    if (fp64)
      hipLaunchKernelGGL(grad_xi_part_kernel<double>, dim3(m, kSplit), dim3(kBlock), 0, s, N, stride,
                         (const double*)xi_terms, perm, part_xi);
    else
      hipLaunchKernelGGL(grad_xi_part_kernel<float>, dim3(m, kSplit), dim3(kBlock), 0, s, N, stride,
                         (const float*)xi_terms, perm, part_xi);
    hipLaunchKernelGGL(part_sum_kernel, dim3((m + 63) / 64), dim3(64), 0, s, m, part_xi, grad);
    hipLaunchKernelGGL(grad_c_kernel, dim3(n_c), dim3(kBlock), 0, s, n_blocks, n_c, cpart, grad + m);
  } else {
    hipError_t e = hipMemsetAsync(grad, 0, sizeof(double) * (m + n_c), s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

int loss_finish_scratch_doubles(int m) { return kSplit * (1 + m); }

hipError_t theta_rows_prepare(int fp64, int64_t N, int stride, void* a_atom, void* u, void* eps_atom, hipStream_t s) {
  const int64_t n_eps = 9 * (int64_t)stride;
  const int64_t n = std::max(3 * N, n_eps);
  if (n == 0) return hipSuccess;
  const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
  if (fp64)
    hipLaunchKernelGGL(unit_weights_kernel<double>, g, dim3(kBlock), 0, s, N, n_eps, (double*)a_atom, (double*)u,
                       (double*)eps_atom);
  else
    hipLaunchKernelGGL(unit_weights_kernel<float>, g, dim3(kBlock), 0, s, N, n_eps, (float*)a_atom, (float*)u,
                       (float*)eps_atom);
  return hipGetLastError();
}

hipError_t theta_rows_finish(int fp64, const ThetaRowArgs& a, const void* pr, const void* pa, const void* pb,
                             const double* b, hipStream_t s) {
  if (a.n_cfg == 0) return hipSuccess;
  if (a.nq > 16) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (size_t)a.nq * kBlock;
  if (fp64)
    hipLaunchKernelGGL(c_rows_kernel<double>, dim3(a.n_cfg), dim3(kBlock), lds, s, a, (const PairRec<double>*)pr,
                       (const double*)pa, (const double*)pb);
  else
    hipLaunchKernelGGL(c_rows_kernel<float>, dim3(a.n_cfg), dim3(kBlock), lds, s, a, (const PairRec<float>*)pr,
                       (const float*)pa, (const float*)pb);
  const int64_t nb = (int64_t)a.n_cfg * a.m;
  if (nb > 0)
    hipLaunchKernelGGL(copy_b_kernel, dim3((unsigned)((nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a.n_cfg, a.m,
                       a.n_c, b, a.rows);
  return hipGetLastError();
}

}  // namespace mtp
