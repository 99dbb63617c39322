// Velocity-Verlet updates for molecular dynamics with the potential's forces
// (the MD loops in which the paper's active learning runs, section 2.3).
// Units: positions in Angstrom, velocities in Angstrom/fs, forces in eV/A,
// masses in atomic mass units; a = F / m with 1 eV/(A amu) = 1/103.6427 A/fs^2.
#include <hip/hip_runtime.h>

#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kMDBlock = 256;
constexpr double kAccel = 1.0 / 103.642696562;   // (eV / A / amu) in A / fs^2

// v += (dt / 2) F / m; then, when drift, x += dt v.
__global__ void __launch_bounds__(kMDBlock) kick_kernel(int64_t n, const int32_t* __restrict__ species, int S,
                                                        const double* __restrict__ inv_mass, double* pos, double* vel,
                                                        const double* __restrict__ F, double dt, int drift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int z = species[i];
  z = z < 0 ? 0 : (z >= S ? S - 1 : z);
  const double h = 0.5 * dt * kAccel * inv_mass[z];
  for (int d = 0; d < 3; ++d) {
    const double v = vel[3 * i + d] + h * F[3 * i + d];
    vel[3 * i + d] = v;
    if (drift) pos[3 * i + d] += dt * v;
  }
}

// One FIRE step (Bitzek, Koskinen, Gaehler, Moseler and Gumbsch, Phys. Rev.
// Lett. 97, 170201 (2006)) for relaxing each configuration to a minimum of
// the potential, one workgroup per configuration.  With P = F . v summed over
// the configuration: if P >= 0 the velocities are mixed towards the force,
// v <- (1 - alpha) v + alpha |v| F / |F|, and after more than n_min such steps
// in a row the step grows (dt <- min(f_inc dt, dt_max)) and alpha shrinks
// (alpha <- f_alpha alpha); if P < 0 the velocities are zeroed, dt <- f_dec dt
// and alpha is reset.  Then a semi-implicit Euler step: v += dt F / m,
// x += dt v.  state[k] = (dt, alpha, steps with P >= 0, unused) per
// configuration.  Sums in a fixed order (per thread strided, then a tree).
__global__ void __launch_bounds__(kMDBlock) fire_kernel(int n_cfg, int64_t n_atoms, const int64_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ species, int S,
                                                        const double* __restrict__ inv_mass, double* pos,
                                                        double* vel, const double* __restrict__ F, double* state,
                                                        FireParams fp) {
  __shared__ double red[3][kMDBlock];
  __shared__ double mix[4];
  const int k = blockIdx.x;
  const int t = threadIdx.x;
  // the range clamped to [0, n_atoms): a malformed offsets array stays in bounds
  int64_t a0 = offsets[k], a1 = offsets[k + 1];
  a0 = a0 < 0 ? 0 : (a0 > n_atoms ? n_atoms : a0);
  a1 = a1 < a0 ? a0 : (a1 > n_atoms ? n_atoms : a1);
  double p = 0.0, vv = 0.0, ff = 0.0;
  for (int64_t i = a0 + t; i < a1; i += blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double f = F[3 * i + d], v = vel[3 * i + d];
      p += f * v;
      vv += v * v;
      ff += f * f;
    }
  red[0][t] = p;
  red[1][t] = vv;
  red[2][t] = ff;
  __syncthreads();
  for (int h = kMDBlock / 2; h > 0; h >>= 1) {
    if (t < h)
      for (int q = 0; q < 3; ++q) red[q][t] += red[q][t + h];
    __syncthreads();
  }
  if (t == 0) {
    double* st = state + 4 * (size_t)k;
    double dt = st[0], alpha = st[1], npos = st[2];
    double cv = 1.0, cf = 0.0, zero = 0.0;
    if (red[0][0] >= 0.0) {
      const double vn = sqrt(red[1][0]), fn = sqrt(red[2][0]);
      cv = 1.0 - alpha;
      cf = fn > 0.0 ? alpha * vn / fn : 0.0;
      if (npos > fp.n_min) {
        dt = fmin(dt * fp.f_inc, fp.dt_max);
        alpha *= fp.f_alpha;
      }
      npos += 1.0;
    } else {
      zero = 1.0;
      dt *= fp.f_dec;
      alpha = fp.alpha_start;
      npos = 0.0;
    }
    st[0] = dt;
    st[1] = alpha;
    st[2] = npos;
    mix[0] = dt;
    mix[1] = cv;
    mix[2] = cf;
    mix[3] = zero;
  }
  __syncthreads();
  const double dt = mix[0], cv = mix[1], cf = mix[2];
  const bool zero = mix[3] != 0.0;
  for (int64_t i = a0 + t; i < a1; i += blockDim.x) {
    int z = species[i];
    z = z < 0 ? 0 : (z >= S ? S - 1 : z);
    const double h = dt * kAccel * inv_mass[z];
    for (int d = 0; d < 3; ++d) {
      const double f = F[3 * i + d];
      double v = zero ? 0.0 : cv * vel[3 * i + d] + cf * f;
      v += h * f;
      vel[3 * i + d] = v;
      pos[3 * i + d] += dt * v;
    }
  }
}

// Kinetic energy sum_i m_i |v_i|^2 / 2 (eV) of every configuration, one
// workgroup each, summed in a fixed order (per thread strided, then a tree).
__global__ void __launch_bounds__(kMDBlock) kinetic_kernel(int n_cfg, int64_t n_atoms,
                                                           const int64_t* __restrict__ offsets,
                                                           const int32_t* __restrict__ species, int S,
                                                           const double* __restrict__ inv_mass,
                                                           const double* __restrict__ vel, double* ekin) {
  __shared__ double red[kMDBlock];
  const int k = blockIdx.x;
  const int t = threadIdx.x;
  int64_t a0 = offsets[k], a1 = offsets[k + 1];
  a0 = a0 < 0 ? 0 : (a0 > n_atoms ? n_atoms : a0);
  a1 = a1 < a0 ? a0 : (a1 > n_atoms ? n_atoms : a1);
  double e = 0.0;
  for (int64_t i = a0 + t; i < a1; i += blockDim.x) {
    int z = species[i];
    z = z < 0 ? 0 : (z >= S ? S - 1 : z);
    const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    e += 0.5 / (kAccel * inv_mass[z]) * (vx * vx + vy * vy + vz * vz);
  }
  red[t] = e;
  __syncthreads();
  for (int h = kMDBlock / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) ekin[k] = red[0];
}

}  // namespace

hipError_t md_kick(int64_t n, const int32_t* species, int S, const double* inv_mass, double* pos, double* vel,
                   const double* F, double dt, int drift, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kick_kernel, dim3((unsigned)((n + kMDBlock - 1) / kMDBlock)), dim3(kMDBlock), 0, s, n, species,
                     S, inv_mass, pos, vel, F, dt, drift);
  return hipGetLastError();
}

hipError_t md_kinetic(int n_cfg, int64_t n_atoms, const int64_t* offsets, const int32_t* species, int S,
                      const double* inv_mass, const double* vel, double* ekin, hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  hipLaunchKernelGGL(kinetic_kernel, dim3(n_cfg), dim3(kMDBlock), 0, s, n_cfg, n_atoms, offsets, species, S, inv_mass,
                     vel, ekin);
  return hipGetLastError();
}

hipError_t md_fire(int n_cfg, int64_t n_atoms, const int64_t* offsets, const int32_t* species, int S,
                   const double* inv_mass, double* pos, double* vel, const double* F, double* state,
                   const FireParams& fp, hipStream_t s) {
  if (n_cfg == 0) return hipSuccess;
  hipLaunchKernelGGL(fire_kernel, dim3(n_cfg), dim3(kMDBlock), 0, s, n_cfg, n_atoms, offsets, species, S, inv_mass,
                     pos, vel, F, state, fp);
  return hipGetLastError();
}

}  // namespace mtp
