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

__global__ void __launch_bounds__(kBlock) loss_total_kernel(int n_cfg, int64_t N, const double* loss_cfg,
                                                            const double* loss_atom, double* loss) {
  double v = 0.0;
  for (int64_t k = threadIdx.x; k < n_cfg; k += blockDim.x) v += loss_cfg[k];
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) v += loss_atom[i];
  const double s = block_sum(v);
  if (threadIdx.x == 0) *loss = s;
}

// grad_xi[f] = sum over atoms of xi_terms[perm[f]][atom]; one workgroup per f.
template <typename T>
__global__ void __launch_bounds__(kBlock) grad_xi_kernel(int64_t N, int stride, const T* xi_terms,
                                                         const int32_t* perm, double* grad) {
  const int f = blockIdx.x;
  const T* row = xi_terms + (size_t)perm[f] * stride;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) v += (double)row[i];
  const double s = block_sum(v);
  if (threadIdx.x == 0) grad[f] = s;
}

// grad_c[t] = sum over workgroups of cpart[b][t].
__global__ void grad_c_kernel(int n_blocks, int n_c, const double* cpart, double* grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_c) return;
  double v = 0.0;
  for (int b = 0; b < n_blocks; ++b) v += cpart[(size_t)b * n_c + t];
  grad[t] = v;
}

}  // namespace

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
                       const double* cpart, double* loss, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(kBlock), 0, s, n_cfg, N, loss_cfg, loss_atom, loss);
  if (N > 0) {
    if (fp64)
      hipLaunchKernelGGL(grad_xi_kernel<double>, dim3(m), dim3(kBlock), 0, s, N, stride, (const double*)xi_terms,
                         perm, grad);
    else
      hipLaunchKernelGGL(grad_xi_kernel<float>, dim3(m), dim3(kBlock), 0, s, N, stride, (const float*)xi_terms,
                         perm, grad);
    hipLaunchKernelGGL(grad_c_kernel, dim3((n_c + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n_blocks, n_c, cpart,
                       grad + m);
  } else {
    hipError_t e = hipMemsetAsync(grad, 0, sizeof(double) * (m + n_c), s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace mtp
