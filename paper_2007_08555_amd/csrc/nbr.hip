// Neighbour lists on the device: every atom j and periodic image n with
// 0 < |x_j + n.L - x_i| < R_cut (the neighbourhood of section 2.1, images of
// atom i itself included).
//
// Pair vectors are formed so that the reverse pair is the exact negation:
// d = x_j - x_i is negated exactly when i and j swap, the fractional offset
// s = d . L^{-1} and every image shift n . L change sign exactly, and
// round-to-nearest is symmetric.  Hence |r_ij| == |r_ji| bit for bit, the
// lists are symmetric, and the reverse of a pair is found by matching the
// negated vector.
//
// Small or free configurations are searched by brute force over atoms and
// over the image box that can reach R_cut; large periodic boxes (at least
// three bins of width >= R_cut along each lattice direction) use a cell list.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kBlock = 256;
constexpr int kBinnedMinAtoms = 2048;

__global__ void cfg_prepare_kernel(NbrArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_cfg) return;
  CfgInfo c;
  c.start = a.atom_offsets[k];
  c.n = (int32_t)(a.atom_offsets[k + 1] - a.atom_offsets[k]);
  const bool bad = a.atom_offsets[k + 1] < a.atom_offsets[k] || (k == 0 && a.atom_offsets[0] != 0) ||
                   (k == a.n_cfg - 1 && a.atom_offsets[k + 1] != a.n_atoms) ||
                   a.atom_offsets[k + 1] - a.atom_offsets[k] > 0x7fffffffLL;
  if (bad) {
    atomicAdd(&a.status->bad_offsets, 1ull);
    c.n = 0;
  }
  c.pbc = a.pbc[k] ? 1 : 0;
  c.binned = 0;
  c.nb[0] = c.nb[1] = c.nb[2] = 1;
  c.bin0 = 0;
  for (int t = 0; t < 9; ++t) {
    c.L[t] = a.cell[9 * k + t];
    c.inv[t] = 0.0;
  }
  c.w[0] = c.w[1] = c.w[2] = 0.0;
  if (c.pbc) {
    const double* L = c.L;
    // cofactors of L; inv = adj / det
    const double c00 = L[4] * L[8] - L[5] * L[7], c01 = L[5] * L[6] - L[3] * L[8],
                 c02 = L[3] * L[7] - L[4] * L[6];
    const double c10 = L[2] * L[7] - L[1] * L[8], c11 = L[0] * L[8] - L[2] * L[6],
                 c12 = L[1] * L[6] - L[0] * L[7];
    const double c20 = L[1] * L[5] - L[2] * L[4], c21 = L[2] * L[3] - L[0] * L[5],
                 c22 = L[0] * L[4] - L[1] * L[3];
    const double det = L[0] * c00 + L[1] * c01 + L[2] * c02;
    const double id = 1.0 / det;
    // inv[a][b] = cofactor[b][a] / det
    c.inv[0] = c00 * id; c.inv[1] = c10 * id; c.inv[2] = c20 * id;
    c.inv[3] = c01 * id; c.inv[4] = c11 * id; c.inv[5] = c21 * id;
    c.inv[6] = c02 * id; c.inv[7] = c12 * id; c.inv[8] = c22 * id;
    // |L_l x L_m| = |cofactor row k|, spacing_k = |det| / |L_l x L_m|
    const double cr[3] = {sqrt(c00 * c00 + c01 * c01 + c02 * c02),
                          sqrt(c10 * c10 + c11 * c11 + c12 * c12),
                          sqrt(c20 * c20 + c21 * c21 + c22 * c22)};
    bool ok = c.n >= kBinnedMinAtoms;
    for (int d = 0; d < 3; ++d) {
      const double spacing = fabs(det) / cr[d];
      c.w[d] = a.rcut / spacing;
      const int nb = (int)floor(spacing / a.rcut);
      c.nb[d] = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
      if (nb < 3) ok = false;
    }
    c.binned = ok ? 1 : 0;
    if (!ok) c.nb[0] = c.nb[1] = c.nb[2] = 1;
  }
  a.cfg[k] = c;
}

// Prefix sum of bins over binned configs (one thread; configs are few
// thousand at most) and the total in *n_bins.
__global__ void bin_offsets_kernel(NbrArgs a, int64_t* n_bins) {
  int64_t acc = 0;
  for (int k = 0; k < a.n_cfg; ++k) {
    CfgInfo& c = a.cfg[k];
    c.bin0 = acc;
    if (c.binned) acc += (int64_t)c.nb[0] * c.nb[1] * c.nb[2];
  }
  *n_bins = acc;
}

__global__ void atom_cfg_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_atoms) return;
  int lo = 0, hi = a.n_cfg;  // find k with offsets[k] <= i < offsets[k+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.atom_offsets[mid] <= i) lo = mid; else hi = mid;
  }
  a.atom_cfg[i] = lo;
}

__device__ inline int3 bin_of(const CfgInfo& c, double x, double y, double z) {
  int b[3];
  for (int d = 0; d < 3; ++d) {
    double f = x * c.inv[0 * 3 + d] + y * c.inv[1 * 3 + d] + z * c.inv[2 * 3 + d];
    f -= floor(f);
    int v = (int)(f * c.nb[d]);
    b[d] = v < 0 ? 0 : (v >= c.nb[d] ? c.nb[d] - 1 : v);
  }
  return make_int3(b[0], b[1], b[2]);
}

__global__ void bin_count_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_atoms) return;
  const CfgInfo& c = a.cfg[a.atom_cfg[i]];
  if (!c.binned) {
    a.atom_bin[i] = -1;
    return;
  }
  const int3 b = bin_of(c, a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]);
  const int64_t flat = c.bin0 + ((int64_t)b.x * c.nb[1] + b.y) * c.nb[2] + b.z;
  a.atom_bin[i] = (int32_t)flat;
  atomicAdd(&a.bin_count[flat], 1);
}

// Exclusive scan of bin counts, one block.
__global__ void bin_scan_kernel(NbrArgs a) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int64_t n = a.n_bins;
  const int64_t per = (n + blockDim.x - 1) / blockDim.x;
  const int64_t lo = t * per, hi = lo + per < n ? lo + per : n;
  int32_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += a.bin_count[b];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0;
    for (int u = 0; u < (int)blockDim.x; ++u) {
      const int32_t v = part[u];
      part[u] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int32_t acc = part[t];
  for (int64_t b = lo; b < hi; ++b) {
    a.bin_start[b] = acc;
    acc += a.bin_count[b];
    a.bin_fill[b] = 0;
  }
  if (hi == n && lo < hi) a.bin_start[n] = acc;
  if (n == 0 && t == 0) a.bin_start[0] = 0;
}

__global__ void bin_fill_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_atoms) return;
  const int32_t b = a.atom_bin[i];
  if (b < 0) return;
  const int32_t slot = atomicAdd(&a.bin_fill[b], 1);
  a.bin_atoms[a.bin_start[b] + slot] = (int32_t)i;
}

// Sort every bin by atom index so that pair order does not depend on the
// order in which atomics landed.
__global__ void bin_sort_kernel(NbrArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_bins) return;
  int32_t* v = a.bin_atoms + a.bin_start[b];
  const int n = a.bin_start[b + 1] - a.bin_start[b];
  for (int x = 1; x < n; ++x) {
    const int32_t key = v[x];
    int y = x - 1;
    while (y >= 0 && v[y] > key) {
      v[y + 1] = v[y];
      --y;
    }
    v[y + 1] = key;
  }
}

template <bool FILL>
struct Emitter {
  NbrArgs& a;
  int64_t i;
  int count;
  double rmin2;
  __device__ void operator()(int32_t j, double rx, double ry, double rz, double r2) {
    if (FILL && count < a.K) {
      const size_t e = (size_t)count * a.stride + i;
      a.nbr[e] = j;
      a.nbr_z[e] = a.species[j];
      if (a.fp64) {
        ((double*)a.px)[e] = rx;
        ((double*)a.py)[e] = ry;
        ((double*)a.pz)[e] = rz;
      } else {
        ((float*)a.px)[e] = (float)rx;
        ((float*)a.py)[e] = (float)ry;
        ((float*)a.pz)[e] = (float)rz;
      }
      if (r2 < rmin2) atomicAdd(&a.status->below_rmin, 1ull);
    }
    ++count;
  }
};

template <bool FILL>
__global__ void __launch_bounds__(kBlock) search_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_atoms) return;
  if (!FILL && (a.species[i] < 0 || a.species[i] >= a.n_species)) atomicAdd(&a.status->bad_species, 1ull);
  const CfgInfo& c = a.cfg[a.atom_cfg[i]];
  const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
  const double rc2 = a.rcut * a.rcut;
  Emitter<FILL> emit{a, i, 0, a.rmin * a.rmin};
  const double* L = c.L;
  const double* inv = c.inv;
  if (!c.binned) {
    const int64_t j0 = c.start, j1 = c.start + c.n;
    for (int64_t j = j0; j < j1; ++j) {
      const double dx = a.pos[3 * j] - xi, dy = a.pos[3 * j + 1] - yi, dz = a.pos[3 * j + 2] - zi;
      if (!c.pbc) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (j != i && r2 < rc2) emit((int32_t)j, dx, dy, dz, r2);
        continue;
      }
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        const double s = dx * inv[0 * 3 + d] + dy * inv[1 * 3 + d] + dz * inv[2 * 3 + d];
        lo[d] = -(int)floor(c.w[d] + s + 1e-9);
        hi[d] = (int)floor(c.w[d] - s + 1e-9);
      }
      for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
        for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
          for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
            if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
            const double sx = (double)n0 * L[0] + (double)n1 * L[3] + (double)n2 * L[6];
            const double sy = (double)n0 * L[1] + (double)n1 * L[4] + (double)n2 * L[7];
            const double sz = (double)n0 * L[2] + (double)n1 * L[5] + (double)n2 * L[8];
            const double rx = dx + sx, ry = dy + sy, rz = dz + sz;
            const double r2 = rx * rx + ry * ry + rz * rz;
            if (r2 < rc2) emit((int32_t)j, rx, ry, rz, r2);
          }
    }
  } else {
    const int3 b = bin_of(c, xi, yi, zi);
    for (int ox = -1; ox <= 1; ++ox)
      for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -1; oz <= 1; ++oz) {
          const int bx = (b.x + ox + c.nb[0]) % c.nb[0];
          const int by = (b.y + oy + c.nb[1]) % c.nb[1];
          const int bz = (b.z + oz + c.nb[2]) % c.nb[2];
          const int64_t flat = c.bin0 + ((int64_t)bx * c.nb[1] + by) * c.nb[2] + bz;
          const int32_t s0 = a.bin_start[flat], s1 = a.bin_start[flat + 1];
          for (int32_t t = s0; t < s1; ++t) {
            const int32_t j = a.bin_atoms[t];
            if (j == i) continue;
            const double dx = a.pos[3 * j] - xi, dy = a.pos[3 * j + 1] - yi, dz = a.pos[3 * j + 2] - zi;
            double n[3];
            for (int d = 0; d < 3; ++d)
              n[d] = -rint(dx * inv[0 * 3 + d] + dy * inv[1 * 3 + d] + dz * inv[2 * 3 + d]);
            const double rx = dx + (n[0] * L[0] + n[1] * L[3] + n[2] * L[6]);
            const double ry = dy + (n[0] * L[1] + n[1] * L[4] + n[2] * L[7]);
            const double rz = dz + (n[0] * L[2] + n[1] * L[5] + n[2] * L[8]);
            const double r2 = rx * rx + ry * ry + rz * rz;
            if (r2 < rc2) emit(j, rx, ry, rz, r2);
          }
        }
  }
  a.count[i] = FILL ? (emit.count < a.K ? emit.count : a.K) : emit.count;
  if (!FILL) {
    atomicMax(&a.status->max_count, (unsigned long long)emit.count);
    atomicAdd(&a.status->n_pairs, (unsigned long long)emit.count);
  }
}

template <typename T>
__global__ void reverse_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= a.n_atoms || p >= a.count[i]) return;
  const size_t e = (size_t)p * a.stride + i;
  const int32_t j = a.nbr[e];
  const T* px = (const T*)a.px;
  const T* py = (const T*)a.py;
  const T* pz = (const T*)a.pz;
  const T rx = -px[e], ry = -py[e], rz = -pz[e];
  const int cj = a.count[j];
  for (int q = 0; q < cj; ++q) {
    const size_t f = (size_t)q * a.stride + j;
    if (a.nbr[f] == (int32_t)i && px[f] == rx && py[f] == ry && pz[f] == rz) {
      a.rev[e] = (int32_t)f;
      return;
    }
  }
  a.rev[e] = (int32_t)e;
  atomicAdd(&a.status->list_errors, 1ull);
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

hipError_t nbr_prepare(NbrArgs& a, hipStream_t s) {
  if (a.n_cfg > 0)
    hipLaunchKernelGGL(cfg_prepare_kernel, grid_for(a.n_cfg), dim3(kBlock), 0, s, a);
  if (a.n_atoms > 0)
    hipLaunchKernelGGL(atom_cfg_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t nbr_bin(NbrArgs& a, hipStream_t s) {
  // caller has set n_bins and sized the bin arrays; bin_count must be zeroed
  if (a.n_atoms == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(a.bin_count, 0, sizeof(int32_t) * (a.n_bins + 1), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bin_count_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(bin_fill_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  if (a.n_bins > 0)
    hipLaunchKernelGGL(bin_sort_kernel, grid_for(a.n_bins), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t nbr_bin_offsets(NbrArgs& a, int64_t* n_bins_dev, hipStream_t s) {
  hipLaunchKernelGGL(bin_offsets_kernel, dim3(1), dim3(1), 0, s, a, n_bins_dev);
  return hipGetLastError();
}

hipError_t nbr_count(NbrArgs& a, hipStream_t s) {
  if (a.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(search_kernel<false>, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t nbr_fill(NbrArgs& a, hipStream_t s) {
  if (a.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(search_kernel<true>, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  if (a.K > 0) {
    const dim3 g((unsigned)((a.n_atoms + kBlock - 1) / kBlock), (unsigned)a.K);
    if (a.fp64)
      hipLaunchKernelGGL(reverse_kernel<double>, g, dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL(reverse_kernel<float>, g, dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace mtp
