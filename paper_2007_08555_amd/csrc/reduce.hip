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

// Forces (when F is not null) and the per-atom virial sum_p g_p (x) r_p
// (when wv is not null), W_ab = dE/d eps_ab for r -> (I + eps) r.
template <typename T>
__global__ void gather_kernel(int64_t n_atoms, int stride, const int32_t* __restrict__ count,
                              const int32_t* __restrict__ rev, const T* __restrict__ g,
                              const PairRec<T>* __restrict__ pr, double* __restrict__ F, T* __restrict__ wv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  double fx = 0, fy = 0, fz = 0;
  double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int c = count[i];
  for (int p = 0; p < c; ++p) {
    const size_t e = (size_t)p * stride + i;
    const double gx = (double)g[3 * e], gy = (double)g[3 * e + 1], gz = (double)g[3 * e + 2];
    if (F) {
      const size_t q = (size_t)rev[e];
      fx += gx - (double)g[3 * q];
      fy += gy - (double)g[3 * q + 1];
      fz += gz - (double)g[3 * q + 2];
    }
    if (wv) {
      const PairRec<T> q = pr[e];
      const double x = (double)q.x, y = (double)q.y, z = (double)q.z;
      w[0] += gx * x; w[1] += gx * y; w[2] += gx * z;
      w[3] += gy * x; w[4] += gy * y; w[5] += gy * z;
      w[6] += gz * x; w[7] += gz * y; w[8] += gz * z;
    }
  }
  if (F) {
    F[3 * i] = fx;
    F[3 * i + 1] = fy;
    F[3 * i + 2] = fz;
  }
  if (wv)
    for (int t = 0; t < 9; ++t) wv[(size_t)t * stride + i] = (T)w[t];
}

// One block per configuration.  Sums are formed in FP64 in a fixed order
// (per-thread strided partial sums, then a tree over the block).
template <typename T>
__global__ void __launch_bounds__(kBlock) config_kernel(int n_cfg, const CfgInfo* __restrict__ cfg,
                                                        int stride, const T* __restrict__ site,
                                                        const T* __restrict__ wv, double* energy,
                                                        double* virial, double* site_out) {
  const int k = blockIdx.x;
  if (k >= n_cfg) return;
  const int64_t a0 = cfg[k].start, a1 = cfg[k].start + cfg[k].n;
  double acc[10];
  for (int t = 0; t < 10; ++t) acc[t] = 0.0;
  for (int64_t i = a0 + threadIdx.x; i < a1; i += blockDim.x) {
    const double v = (double)site[i];
    acc[0] += v;
    if (site_out) site_out[i] = v;
    if (wv)
      for (int t = 0; t < 9; ++t) acc[1 + t] += (double)wv[(size_t)t * stride + i];
  }
  __shared__ double red[10][kBlock];
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (energy) energy[k] = red[0][0];
    if (virial && wv)
      for (int t = 0; t < 9; ++t) virial[9 * k + t] = red[1 + t][0];
  }
}

// b[k][f] = sum over atoms of configuration k of B[perm[f]][atom]; one block
// per configuration, threads over basis functions.
template <typename T>
__global__ void __launch_bounds__(kBlock) b_kernel(int n_cfg, const CfgInfo* __restrict__ cfg,
                                                   const T* __restrict__ B, int m, int b_stride,
                                                   const int32_t* __restrict__ perm, double* b) {
  const int k = blockIdx.x;
  if (k >= n_cfg) return;
  const int64_t a0 = cfg[k].start, a1 = cfg[k].start + cfg[k].n;
  for (int f = threadIdx.x; f < m; f += blockDim.x) {
    const T* row = B + (size_t)perm[f] * b_stride;
    double s = 0.0;
    for (int64_t i = a0; i < a1; ++i) s += (double)row[i];
    b[(size_t)k * m + f] = s;
  }
}

}  // namespace

hipError_t gather_forces(int fp64, int64_t n_atoms, int stride, const int32_t* count,
                         const int32_t* rev, const void* gp, const void* pr, double* forces,
                         void* atom_virial, hipStream_t s) {
  if (n_atoms == 0 || (!forces && !atom_virial)) return hipSuccess;
  const dim3 g((unsigned)((n_atoms + kBlock - 1) / kBlock));
  if (fp64)
    hipLaunchKernelGGL(gather_kernel<double>, g, dim3(kBlock), 0, s, n_atoms, stride, count, rev,
                       (const double*)gp, (const PairRec<double>*)pr, forces, (double*)atom_virial);
  else
    hipLaunchKernelGGL(gather_kernel<float>, g, dim3(kBlock), 0, s, n_atoms, stride, count, rev,
                       (const float*)gp, (const PairRec<float>*)pr, forces, (float*)atom_virial);
  return hipGetLastError();
}

hipError_t reduce_configs(int fp64, int n_cfg, const CfgInfo* offs, int stride, const void* site,
                          const void* atom_virial, const void* B, int m, int b_stride,
                          const int32_t* perm, double* energy, double* virial, double* b,
                          double* site_out, hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  if (energy || virial || site_out) {
    if (fp64)
      hipLaunchKernelGGL(config_kernel<double>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const double*)site, (const double*)atom_virial, energy, virial, site_out);
    else
      hipLaunchKernelGGL(config_kernel<float>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const float*)site, (const float*)atom_virial, energy, virial, site_out);
  }
  if (b && B) {
    if (fp64)
      hipLaunchKernelGGL(b_kernel<double>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs,
                         (const double*)B, m, b_stride, perm, b);
    else
      hipLaunchKernelGGL(b_kernel<float>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs,
                         (const float*)B, m, b_stride, perm, b);
  }
  return hipGetLastError();
}

}  // namespace mtp
