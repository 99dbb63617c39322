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

}  // namespace

hipError_t md_kick(int64_t n, const int32_t* species, int S, const double* inv_mass, double* pos, double* vel,
                   const double* F, double dt, int drift, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kick_kernel, dim3((unsigned)((n + kMDBlock - 1) / kMDBlock)), dim3(kMDBlock), 0, s, n, species,
                     S, inv_mass, pos, vel, F, dt, drift);
  return hipGetLastError();
}

}  // namespace mtp
