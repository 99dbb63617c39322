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

// Forces F_i = sum over slots p of (g_p - g_rev(p)): the first sum was taken
// in FP64 by the last adjoint pass (own, [3][stride]), so only the reverse
// pairs' g is fetched here, subtracted in FP64 in slot order.  Pairs are
// taken eight at a time so that the eight dependent loads g[rev[e]] are in
// flight together.  (The per-atom virials are summed by the last adjoint
// pass as well.)
template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(int64_t n_atoms, int stride,
                                                        const int32_t* __restrict__ count,
                                                        const int32_t* __restrict__ rev,
                                                        const T* __restrict__ g, const double* __restrict__ own,
                                                        double* __restrict__ F) {
  constexpr int U = 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// FP64 sums of a configuration's site energies and per-atom virials in a
// fixed order: per thread the atoms i, i + blockDim, i + 2 blockDim, ...,
// then a tree over the block;
// U atoms per thread are loaded together (U > 1 for large configurations:
// the loads of one block then overlap).
template <typename T, int U>
__device__ __forceinline__ void config_sums(int k, const CfgInfo* __restrict__ cfg, int stride,
                                            const T* __restrict__ site, const T* __restrict__ wv, double* energy,
                                            double* virial, double* site_out) {
  const int64_t a0 = cfg[k].start, a1 = cfg[k].start + cfg[k].n;
  double acc[10];
  for (int t = 0; t < 10; ++t) acc[t] = 0.0;
  for (int64_t i0 = a0 + threadIdx.x; i0 < a1; i0 += (int64_t)U * blockDim.x) {
    double v[U], w[U][9];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      const int64_t ic = i < a1 ? i : i0;
      v[u] = (double)site[ic];
      if (wv)
        for (int t = 0; t < 9; ++t) w[u][t] = (double)wv[(size_t)t * stride + ic];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      if (i >= a1) break;
      acc[0] += v[u];
      if (site_out) site_out[i] = v[u];
      if (wv)
        for (int t = 0; t < 9; ++t) acc[1 + t] += w[u][t];
    }
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

// One block per configuration; configurations above kLargeCfg atoms are left
// to config_large_kernel (one atom per thread keeps this kernel's registers,
// and so its occupancy over many small configurations, low).
constexpr int kLargeCfg = 4 * kBlock;

template <typename T>
__global__ void __launch_bounds__(kBlock) config_kernel(int n_cfg, const CfgInfo* __restrict__ cfg, int stride,
                                                        const T* __restrict__ site, const T* __restrict__ wv,
                                                        double* energy, double* virial, double* site_out) {
  const int k = blockIdx.x;
  if (k >= n_cfg || cfg[k].n > kLargeCfg) return;
  config_sums<T, 1>(k, cfg, stride, site, wv, energy, virial, site_out);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) config_large_kernel(int n_cfg, const CfgInfo* __restrict__ cfg, int stride,
                                                              const T* __restrict__ site, const T* __restrict__ wv,
                                                              double* energy, double* virial, double* site_out) {
  const int k = blockIdx.x;
  if (k >= n_cfg || cfg[k].n <= kLargeCfg) return;
  config_sums<T, 4>(k, cfg, stride, site, wv, energy, virial, site_out);
}

// b[k][f] = sum over atoms of configuration k of B[perm[f]][atom]; one block
// per configuration, each wavefront four basis functions at a time: lanes
// read consecutive atoms (coalesced) and the 64 partial sums are combined by
// a butterfly in a fixed order.
template <typename T>
__global__ void __launch_bounds__(kBlock) b_kernel(int n_cfg, const CfgInfo* __restrict__ cfg,
                                                   const T* __restrict__ B, int m, int b_stride,
                                                   const int32_t* __restrict__ perm, double* b) {
  constexpr int U = 4;
  constexpr int kWaves = kBlock / 64;
  const int k = blockIdx.x;
  if (k >= n_cfg) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t a0 = cfg[k].start, a1 = cfg[k].start + cfg[k].n;
  for (int f0 = wave * U; f0 < m; f0 += kWaves * U) {
    const T* row[U];
    double s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      row[u] = B + (size_t)perm[f0 + u < m ? f0 + u : f0] * b_stride;
      s[u] = 0.0;
    }
    for (int64_t i = a0 + lane; i < a1; i += 64)
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] += (double)row[u][i];
#pragma unroll
    for (int u = 0; u < U; ++u)
      for (int o = 32; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, 64);
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (f0 + u < m) b[(size_t)k * m + f0 + u] = s[u];
  }
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

hipError_t reduce_configs(int fp64, int n_cfg, const CfgInfo* offs, int stride, const void* site,
                          const void* atom_virial, const void* B, int m, int b_stride,
                          const int32_t* perm, double* energy, double* virial, double* b,
                          double* site_out, hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  if (energy || virial || site_out) {
    if (fp64) {
      hipLaunchKernelGGL(config_kernel<double>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const double*)site, (const double*)atom_virial, energy, virial, site_out);
      hipLaunchKernelGGL(config_large_kernel<double>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const double*)site, (const double*)atom_virial, energy, virial, site_out);
    } else {
      hipLaunchKernelGGL(config_kernel<float>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const float*)site, (const float*)atom_virial, energy, virial, site_out);
      hipLaunchKernelGGL(config_large_kernel<float>, dim3(n_cfg), dim3(kBlock), 0, s, n_cfg, offs, stride,
                         (const float*)site, (const float*)atom_virial, energy, virial, site_out);
    }
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
