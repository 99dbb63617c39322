// Neighbour lists on the device: every atom j and periodic image n with
// 0 < |x_j + n.L - x_i| < R_cut (the neighbourhood of section 2.1, images of
// atom i itself included).
//
// Pair vectors are formed so that the reverse pair is the exact negation:
// d = x_j - x_i is negated exactly when i and j swap, the fractional offset
// s = d . L^{-1} and every image shift n . L change sign exactly, and
// round-to-nearest is symmetric.  Hence |r_ij| == |r_ji| bit for bit and the
// lists are symmetric.
//
// Small or free configurations are searched by brute force over atoms and
// over the box of images that can reach R_cut; the entries of one neighbour
// j are then contiguous and ordered by image n.  Large periodic boxes (at
// least three bins of width >= R_cut along each lattice direction, so at most
// one image of any atom is in range) use a cell list.  Either way the
// reverse of the r-th entry of the run of j in i's list is the
// (k - 1 - r)-th entry of the run of i in j's list (negation reverses the
// image order), which gives the reverse index without comparing vectors.
//
// No host synchronisation: the lists have a fixed capacity of K slots per
// atom and the number of atoms that exceed it is counted in the status.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kBlock = 256;
constexpr int kBinnedMinAtoms = 2048;
constexpr int kSmallMax = 256;    // configurations searched by one workgroup from LDS
constexpr int kSmallBlock = 256;
constexpr int kWriteGroup = 4;   // list entries written together by the small search

__device__ inline bool is_small(const CfgInfo& c) { return !c.binned && c.n <= kSmallMax; }

__global__ void cfg_prepare_kernel(NbrArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_cfg) return;
  CfgInfo c;
  c.start = a.atom_offsets[k];
  c.n = (int32_t)(a.atom_offsets[k + 1] - a.atom_offsets[k]);
  const bool bad = a.atom_offsets[k + 1] < a.atom_offsets[k] || a.atom_offsets[k] < 0 ||
                   a.atom_offsets[k + 1] > a.n_atoms || (k == 0 && a.atom_offsets[0] != 0) ||
                   (k == a.n_cfg - 1 && a.atom_offsets[k + 1] != a.n_atoms);
  if (bad) {
    // an invalid range is searched as empty; the call then fails
    atomicAdd(&a.status->bad_offsets, 1ull);
    c.start = 0;
    c.n = 0;
  }
  c.pbc = a.pbc[k] ? 1 : 0;
  c.binned = 0;
  c.nb[0] = c.nb[1] = c.nb[2] = 1;
  c.bin0 = c.start;
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
    int nb[3];
    bool ok = c.n >= kBinnedMinAtoms && det != 0.0;
    for (int d = 0; d < 3; ++d) {
      const double spacing = fabs(det) / cr[d];
      c.w[d] = a.rcut / spacing;
      const double q = floor(spacing / a.rcut);
      nb[d] = q > 1024.0 ? 1024 : (int)q;
      if (nb[d] < 3) ok = false;
    }
    // the bins of a config live in its own atom range: at most n bins
    while (ok && (int64_t)nb[0] * nb[1] * nb[2] > c.n) {
      int d = nb[0] >= nb[1] ? (nb[0] >= nb[2] ? 0 : 2) : (nb[1] >= nb[2] ? 1 : 2);
      if (nb[d] <= 3) ok = false;
      else --nb[d];
    }
    if (ok) {
      c.binned = 1;
      c.nb[0] = nb[0];
      c.nb[1] = nb[1];
      c.nb[2] = nb[2];
    }
  }
  a.cfg[k] = c;
}

// Launch order of the small-configuration search: largest configurations
// first (a counting sort by atom count; the order among equal counts does
// not matter), so that the longest workgroups do not start last.  After the
// n_cfg positions, the numbers of small configurations that take 1, 2, 3
// and 4 wavefronts (1-64, 65-128, 129-192 and 193-256 atoms), from which
// every workgroup finds its bundle (bundle_slot).
__global__ void __launch_bounds__(1024) cfg_order_kernel(NbrArgs a) {
  constexpr int kBins = kSmallMax + 2;   // counts 0..kSmallMax, then larger ones
  __shared__ int hist[kBins], base[kBins];
  const int t = threadIdx.x;   // blockDim.x >= kBins
  if (t < kBins) hist[t] = 0;
  __syncthreads();
  auto bin_of_cfg = [&](int k) {
    const int n = a.cfg[k].n;
    return n > kSmallMax ? kBins - 1 : kSmallMax - n;   // descending counts, large boxes last
  };
  for (int k = threadIdx.x; k < a.n_cfg; k += blockDim.x) atomicAdd(&hist[bin_of_cfg(k)], 1);
  __syncthreads();
  // inclusive scan of the bins (in base), then exclusive starts
  if (t < kBins) base[t] = hist[t];
  __syncthreads();
  for (int off = 1; off < kBins; off <<= 1) {
    const int v = t < kBins && t >= off ? base[t - off] : 0;
    __syncthreads();
    if (t < kBins) base[t] += v;
    __syncthreads();
  }
  // configurations of w + 1 wavefronts: n in [64 w + 1, 64 w + 64], bins
  // kSmallMax - n in [192 - 64 w, 255 - 64 w]
  if (t < 4) {
    const int hi = 255 - 64 * t, lo = 191 - 64 * t;
    a.cfg_order[a.n_cfg + t] = base[hi] - (lo >= 0 ? base[lo] : 0);
  }
  __syncthreads();
  if (t < kBins) base[t] -= hist[t];
  __syncthreads();
  for (int k = threadIdx.x; k < a.n_cfg; k += blockDim.x) a.cfg_order[atomicAdd(&base[bin_of_cfg(k)], 1)] = k;
}

__global__ void atom_cfg_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_atoms) return;
  int lo = 0, hi = a.n_cfg;  // k with offsets[k] <= i < offsets[k+1] when the offsets are valid
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.atom_offsets[mid] <= i) lo = mid; else hi = mid;
  }
  a.atom_cfg[i] = lo;
}

__global__ void zero_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
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

__device__ inline bool in_cfg(const CfgInfo& c, int64_t i) { return i >= c.start && i < c.start + c.n; }

// One record per pair (the FP32 path rounds the FP64 pair vector).
__device__ inline void store_pair(const NbrArgs& a, size_t e, double rx, double ry, double rz, int zj) {
  if (a.fp64) {
    PairRec<double> q;
    q.x = rx; q.y = ry; q.z = rz; q.zj = zj; q.pad = 0;
    ((PairRec<double>*)a.pr)[e] = q;
  } else {
    PairRec<float> q;
    q.x = (float)rx; q.y = (float)ry; q.z = (float)rz; q.zj = zj;
    ((PairRec<float>*)a.pr)[e] = q;
  }
}

// Conservative image box of one pair: every integer n_d with
// |s_d + n_d| <= w_d, widened by a small margin (bounds in FP32; membership
// is decided by the exact FP64 distance test).
__device__ inline void image_box(const CfgInfo& c, double dx, double dy, double dz, int (&lo)[3], int (&hi)[3]) {
  const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
  for (int d = 0; d < 3; ++d) {
    const float s = fx * (float)c.inv[0 * 3 + d] + fy * (float)c.inv[1 * 3 + d] + fz * (float)c.inv[2 * 3 + d];
    const float w = (float)c.w[d] + 1e-3f;
    lo[d] = -(int)floorf(w + s);
    hi[d] = (int)floorf(w - s);
  }
}

// Bins of the binned configurations; also lists the atoms of every
// configuration that is not small (the reverse pass needs only those when the
// small search kept its lists in LDS), one atomic per wavefront.
__global__ void bin_count_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const CfgInfo* cp = i < a.n_atoms ? &a.cfg[a.atom_cfg[i]] : nullptr;
  const bool big = cp && in_cfg(*cp, i) && !is_small(*cp);
  const unsigned long long m = __ballot(big);
  if (m) {
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long first = 0;
    if (lane == leader) first = atomicAdd(&a.status->n_large, (unsigned long long)__popcll(m));
    first = __shfl(first, leader, 64);
    if (big) a.large[first + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
  }
  if (i >= a.n_atoms) return;
  const CfgInfo& c = *cp;
  if (!c.binned || !in_cfg(c, i)) {
    a.atom_bin[i] = -1;
    return;
  }
  const int3 b = bin_of(c, a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]);
  const int64_t flat = c.bin0 + ((int64_t)b.x * c.nb[1] + b.y) * c.nb[2] + b.z;
  a.atom_bin[i] = (int32_t)flat;
  atomicAdd(&a.bin_count[flat], 1);
  a.binned[atomicAdd(&a.status->n_binned, 1ull)] = (int32_t)i;
}

// Exclusive scan of the bin counts of one binned configuration (one block
// per configuration; the others return at once).  Bin b of a configuration
// starting at atom `start` lists its atoms at bin_atoms[bin_start[b] ..
// bin_start[b + 1]), inside [start, start + n).
__global__ void __launch_bounds__(256) bin_scan_kernel(NbrArgs a) {
  __shared__ int32_t part[256];
  __shared__ int32_t carry;
  const CfgInfo& c = a.cfg[blockIdx.x];
  if (!c.binned) return;
  const int t = threadIdx.x;
  const int64_t nbins = (int64_t)c.nb[0] * c.nb[1] * c.nb[2];
  if (t == 0) carry = (int32_t)c.start;
  __syncthreads();
  for (int64_t base = 0; base < nbins; base += blockDim.x) {
    const int64_t b = c.bin0 + base + t;
    const int32_t v = base + t < nbins ? a.bin_count[b] : 0;
    part[t] = v;
    __syncthreads();
    for (int w = 1; w < (int)blockDim.x; w <<= 1) {  // inclusive Hillis-Steele scan
      const int32_t u = t >= w ? part[t - w] : 0;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    if (base + t < nbins) {
      a.bin_start[b] = carry + part[t] - v;
      a.bin_fill[b] = 0;
    }
    __syncthreads();
    if (t == (int)blockDim.x - 1) carry += part[t];
    __syncthreads();
  }
  if (t == 0) a.bin_start[c.bin0 + nbins] = carry;
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
  if (b >= a.n_atoms) return;
  // bins of a binned configuration occupy the first nb0 nb1 nb2 indices of its atom range
  const CfgInfo& c = a.cfg[a.atom_cfg[b]];
  if (!c.binned || b < c.bin0 || b >= c.bin0 + (int64_t)c.nb[0] * c.nb[1] * c.nb[2]) return;
  const int n = a.bin_start[b + 1] - a.bin_start[b];
  if (n < 2) return;
  int32_t* v = a.bin_atoms + a.bin_start[b];
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

// Pair vector to the nearest image of atom j in a binned configuration (at
// most one image lies within R_cut): n = -rint(d . L^-1), r = d + n . L.
__device__ inline void binned_vector(const CfgInfo& c, double dx, double dy, double dz, double& rx, double& ry,
                                     double& rz) {
  const double* L = c.L;
  const double* inv = c.inv;
  double n[3];
  for (int d = 0; d < 3; ++d) n[d] = -rint(dx * inv[0 * 3 + d] + dy * inv[1 * 3 + d] + dz * inv[2 * 3 + d]);
  rx = dx + (n[0] * L[0] + n[1] * L[3] + n[2] * L[6]);
  ry = dy + (n[0] * L[1] + n[1] * L[4] + n[2] * L[7]);
  rz = dz + (n[0] * L[2] + n[1] * L[5] + n[2] * L[8]);
}

struct Emitter {
  NbrArgs& a;
  int64_t i;
  int count;
  double rmin2;
  int below;
  __device__ void operator()(int32_t j, double rx, double ry, double rz, double r2) {
    if (count < a.K) {
      const size_t e = (size_t)count * a.stride + i;
      int zj = a.species[j];
      zj = zj < 0 ? 0 : (zj >= a.n_species ? a.n_species - 1 : zj);
      a.nbr[e] = j;
      store_pair(a, e, rx, ry, rz, zj);
    }
    if (r2 < rmin2) ++below;
    ++count;
  }
};

// Sum and max over the 64 lanes of a wavefront (every lane must call it).
__device__ inline int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One thread per atom of the configurations that are neither small nor
// binned (large clusters, large cells too thin for three bins): brute force
// over the configuration's atoms and, in a periodic cell, over the box of
// images that can reach R_cut.
__global__ void __launch_bounds__(kBlock) search_kernel(NbrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // atoms of small configurations are searched by search_small_kernel, those
  // of binned ones by search_binned_kernel; every lane stays to the end for
  // the wavefront reductions
  const bool active = i < a.n_atoms && !((is_small(a.cfg[a.atom_cfg[i]]) || a.cfg[a.atom_cfg[i]].binned) &&
                                         in_cfg(a.cfg[a.atom_cfg[i]], i));
  Emitter emit{a, i, 0, a.rmin * a.rmin, 0};
  int bad = 0;
  if (active) {
  if (a.species[i] < 0 || a.species[i] >= a.n_species) bad = 1;
  const CfgInfo& c = a.cfg[a.atom_cfg[i]];
  if (in_cfg(c, i)) {
    const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
    const double rc2 = a.rcut * a.rcut;
    const double* L = c.L;
    {
      const int64_t j0 = c.start, j1 = c.start + c.n;
      for (int64_t j = j0; j < j1; ++j) {
        const double dx = a.pos[3 * j] - xi, dy = a.pos[3 * j + 1] - yi, dz = a.pos[3 * j + 2] - zi;
        if (!c.pbc) {
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (j != i && r2 < rc2) emit((int32_t)j, dx, dy, dz, r2);
          continue;
        }
        // images with |s_d + n_d| <= w_d can lie within R_cut
        int lo[3], hi[3];
        image_box(c, dx, dy, dz, lo, hi);
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
    }
  }
  a.count[i] = emit.count < a.K ? emit.count : a.K;
  }
  // one atomic per wavefront and counter
  const int cmax = wave_max(emit.count);
  const int csum = wave_sum(emit.count);
  const int over = wave_sum(emit.count > a.K ? 1 : 0);
  const int below = wave_sum(emit.below);
  const int nbad = wave_sum(bad);
  if ((threadIdx.x & 63) == 0 && (csum || nbad)) {
    atomicMax(&a.status->max_count, (unsigned long long)cmax);
    atomicAdd(&a.status->n_pairs, (unsigned long long)csum);
    if (over) atomicAdd(&a.status->overflow, (unsigned long long)over);
    if (below) atomicAdd(&a.status->below_rmin, (unsigned long long)below);
    if (nbad) atomicAdd(&a.status->bad_species, (unsigned long long)nbad);
  }
}

// Binned configurations, one wavefront per atom.  The candidates are the
// atoms of the 27 bins around the atom's bin, bins in the order
// (ox, oy, oz) = -1..1 and atoms of a bin in ascending index.  Lane s < 27
// loads the range of bin s, a scan over the lanes numbers the candidates, and
// each round tests 64 consecutive candidates, one per lane; a ballot ranks
// the neighbours found, so the list keeps the candidate order.  A fixed grid
// walks the atoms listed in a.binned (their number is in the status), and
// each workgroup adds its counts to the status once.  All cross-lane
// operations run with every lane active.
constexpr int kBinnedBlocks = 256;
constexpr int kBinnedBlock = 1024;

__global__ void __launch_bounds__(kBinnedBlock) search_binned_kernel(NbrArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t n_binned = (int64_t)a.status->n_binned;
  const double rc2 = a.rcut * a.rcut, rmin2 = a.rmin * a.rmin;
  int pairs = 0, cmax = 0, over = 0, nbad = 0, below = 0;
  for (int64_t k = wave; k < n_binned; k += n_waves) {
    const int64_t i = a.binned[k];
    const CfgInfo& c = a.cfg[a.atom_cfg[i]];
    const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
    const int3 b = bin_of(c, xi, yi, zi);
    int start = 0, size = 0;
    if (lane < 27) {
      const int ox = lane / 9 - 1, oy = (lane / 3) % 3 - 1, oz = lane % 3 - 1;
      const int bx = (b.x + ox + c.nb[0]) % c.nb[0];
      const int by = (b.y + oy + c.nb[1]) % c.nb[1];
      const int bz = (b.z + oz + c.nb[2]) % c.nb[2];
      const int64_t flat = c.bin0 + ((int64_t)bx * c.nb[1] + by) * c.nb[2] + bz;
      start = a.bin_start[flat];
      size = a.bin_start[flat + 1] - start;
    }
    int incl = size;   // inclusive scan over lanes 0..26 (lanes above hold 0)
    for (int o = 1; o < 32; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 26, 64);
    const int excl = incl - size;
    int count = 0;
    for (int base = 0; base < total; base += 64) {
      const int cand = base + lane;
      // first bin s with incl_s > cand: it holds candidate cand
      int lo = 0, hi = 27;
      for (int it = 0; it < 5; ++it) {
        const int mid = (lo + hi) >> 1;
        const int v = __shfl(incl, mid < 26 ? mid : 26, 64);
        if (lo < hi) {
          if (v > cand) hi = mid; else lo = mid + 1;
        }
      }
      const int sb = lo < 26 ? lo : 26;
      const int st = __shfl(start, sb, 64), ex = __shfl(excl, sb, 64);
      bool hit = false;
      int32_t j = -1;
      double rx = 0.0, ry = 0.0, rz = 0.0, r2 = 0.0;
      if (cand < total) {
        j = a.bin_atoms[st + (cand - ex)];
        if (j != (int32_t)i) {
          const double dx = a.pos[3 * j] - xi, dy = a.pos[3 * j + 1] - yi, dz = a.pos[3 * j + 2] - zi;
          binned_vector(c, dx, dy, dz, rx, ry, rz);
          r2 = rx * rx + ry * ry + rz * rz;
          hit = r2 < rc2;
        }
      }
      const unsigned long long mask = __ballot(hit);
      const int slot = count + __popcll(mask & ((1ull << lane) - 1ull));
      if (hit && slot < a.K) {
        const size_t e = (size_t)slot * a.stride + i;
        int zj = a.species[j];
        zj = zj < 0 ? 0 : (zj >= a.n_species ? a.n_species - 1 : zj);
        a.nbr[e] = j;
        store_pair(a, e, rx, ry, rz, zj);
      }
      if (hit && r2 < rmin2) ++below;
      count += __popcll(mask);
    }
    if (lane == 0) {
      a.count[i] = count < a.K ? count : a.K;
      if (a.species[i] < 0 || a.species[i] >= a.n_species) ++nbad;
    }
    pairs += count;
    cmax = count > cmax ? count : cmax;
    if (count > a.K) ++over;
  }
  below = wave_sum(below);
  nbad = wave_sum(nbad);
  // per-wavefront counts (uniform across the lanes) summed over the workgroup
  constexpr int kWaves = kBinnedBlock / 64;
  __shared__ int part[5][kWaves];
  const int w = threadIdx.x >> 6;
  if (lane == 0) {
    part[0][w] = pairs;
    part[1][w] = cmax;
    part[2][w] = over;
    part[3][w] = below;
    part[4][w] = nbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tp = 0, to = 0, tb = 0, tn = 0;
    int tm = 0;
    for (int q = 0; q < kWaves; ++q) {
      tp += part[0][q];
      tm = part[1][q] > tm ? part[1][q] : tm;
      to += part[2][q];
      tb += part[3][q];
      tn += part[4][q];
    }
    if (tp || tn) {
      atomicMax(&a.status->max_count, (unsigned long long)tm);
      atomicAdd(&a.status->n_pairs, tp);
      if (to) atomicAdd(&a.status->overflow, to);
      if (tb) atomicAdd(&a.status->below_rmin, tb);
      if (tn) atomicAdd(&a.status->bad_species, tn);
    }
  }
}

// rev[p, i] for every stored pair, one thread per slot; see the file comment
// for the rule.  The run of j around slot p gives r (entries of j before p)
// and k; the start of i's run in j's list comes from the run-start table of
// the small search, else from a search of j's list.
__device__ inline void reverse_entry(const NbrArgs& a, int64_t i, int p, int small_done) {
  if (p >= a.count[i]) return;
  const CfgInfo& c = a.cfg[a.atom_cfg[i]];
  if (!in_cfg(c, i) || (small_done && is_small(c))) return;
  const size_t st = (size_t)a.stride;
  const size_t e = (size_t)p * st + i;
  const int ci = a.count[i];
  const int32_t j = a.nbr[e];
  int rank = 0;
  while (p - rank - 1 >= 0 && a.nbr[(size_t)(p - rank - 1) * st + i] == j) ++rank;
  int after = 0;
  while (p + after + 1 < ci && a.nbr[(size_t)(p + after + 1) * st + i] == j) ++after;
  const int k = rank + 1 + after;
  const int cj = a.count[j];
  int q0 = -1;
  if (is_small(c)) {
    const int n = c.n;
    const int li = (int)(i - c.start), lj = (int)(j - c.start);
    if (lj >= 0 && lj < n) q0 = a.run_start[(size_t)c.start * kSmallMax + (size_t)lj * n + li];
  } else {
    int lo = 0;
    if (c.binned) {
      while (lo < cj && a.nbr[(size_t)lo * st + j] != (int32_t)i) ++lo;   // one image per atom
    } else {
      int hi = cj;                                                      // lists ascend in neighbour index
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.nbr[(size_t)mid * st + j] < (int32_t)i) lo = mid + 1; else hi = mid;
      }
    }
    q0 = lo;
  }
  const int q = q0 + k - 1 - rank;
  if (q0 >= 0 && q < cj && a.nbr[(size_t)q * st + j] == (int32_t)i) {
    a.rev[e] = (int32_t)((size_t)q * st + j);
  } else {
    a.rev[e] = (int32_t)e;
    atomicAdd(&a.status->list_errors, 1ull);
  }
}

// Every atom, slot p = blockIdx.y (direct lists: small configurations too).
__global__ void reverse_kernel(NbrArgs a, int small_done) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n_atoms) reverse_entry(a, i, blockIdx.y, small_done);
}

// Only the atoms listed in a.large (the small search wrote its own reverse
// indices): entries k = blockIdx.x * blockDim.x + threadIdx.x + multiples of
// the grid's width of the list, slot p = blockIdx.y.  The grid is as wide as
// the atoms up to kReverseBlocks workgroups; workgroups past the list's length
// (all of them when every configuration is small) leave after one scalar load.
constexpr int kReverseBlocks = 256;

__global__ void reverse_large_kernel(NbrArgs a) {
  const int64_t n = (int64_t)a.status->n_large;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    reverse_entry(a, a.large[k], blockIdx.y, 1);
}

// Whole search of one small configuration in one workgroup.  Positions,
// clamped species and (periodic cells) FP32 fractional coordinates are
// staged in LDS; one atom per thread walks the atoms j of its configuration.
// For a periodic cell the images n of j that can lie within R_cut satisfy
// |s_j - s_i + n_d| <= w_d per lattice direction (s fractional coordinates,
// w_d = R_cut / interplanar spacing).  With s = u + m, u = s - floor(s) in
// [0, 1) held in FP32 and m integer, the box is taken over n' = n + m_j - m_i
// with |u_j - u_i + n'_d| <= w_d (plus a margin for the rounding of u): j is
// rejected at once when the nearest integer to u_j - u_i is farther than w_d
// along some direction, otherwise the images of the box are tested with the
// exact FP64 pair vector.  When every w_d < 1/2 the box holds at most that
// nearest integer ("nearest" cells).  u_j - u_i changes sign exactly when i
// and j swap, so the box of (j, i) is the negated box of (i, j).
//
// With neighbour capacity K <= kLdsSlots the lists are built in LDS first
// (one byte per slot: the neighbour's index in the configuration); after a
// barrier a write-out pass forms each slot's pair vector again and stores the
// pair record, the neighbour index and the reverse index at p * stride + i,
// so that the threads of a wavefront store consecutive records of one slot.
// Reverse indices: the r-th of the k images in i's run of j is reversed by
// entry q0 + k - 1 - r of j's list, q0 the start of j's run of i, found by a
// binary search of j's LDS list.  With a larger K the search writes the
// records directly and records run starts in a global table
// (run_start[i][j]) that reverse_kernel reads.
constexpr int kLdsSlots = kLdsListSlots;

// Per-atom LDS records of the small search: FP64 position, FP32 wrapped
// fractional coordinates u, their integer parts m and the clamped species.
struct SmallAtoms {
  double4* x;  // (x, y, z, -)
  float4* u;   // (u0, u1, u2, -)
  int4* mz;    // (m0, m1, m2, species)
};

__device__ inline bool nearest_cell(const CfgInfo& c) {
  return c.pbc && c.w[0] + 1e-3 < 0.5 && c.w[1] + 1e-3 < 0.5 && c.w[2] + 1e-3 < 0.5;
}

// Image box of atom lj for atom li in a periodic cell: the n with
// |s_d + n'_d| <= w_d (n = n' - m_j + m_i), bounds in FP32 with a margin
// (membership is decided by the exact FP64 distance test).  Returns false
// when no image can lie within R_cut.
struct ImageBox {
  int lo0, lo1, lo2, hi0, hi1, hi2;
  double dx, dy, dz;   // x_j - x_i
};

__device__ inline bool box_may_hit(const CfgInfo& c, float4 ui, float4 uj) {
  const float w0 = (float)c.w[0] + 1e-3f, w1 = (float)c.w[1] + 1e-3f, w2 = (float)c.w[2] + 1e-3f;
  const float s0 = uj.x - ui.x, s1 = uj.y - ui.y, s2 = uj.z - ui.z;
  // bitwise, not short-circuit: all three components are tested without branches
  return !((fabsf(s0 - rintf(s0)) > w0) | (fabsf(s1 - rintf(s1)) > w1) | (fabsf(s2 - rintf(s2)) > w2));
}

// f(j, rec[j]) for j = 0..n-1 in order, the LDS records loaded kSweep at a
// time before any is used, so that their latencies overlap (one load in
// flight per candidate leaves the loop waiting on LDS).  Indices past n are
// clamped for the loads and skipped for f.
constexpr int kSweep = 8;

template <typename T, typename F>
__device__ inline void lds_sweep(const T* rec, int n, F&& f) {
  for (int j0 = 0; j0 < n; j0 += kSweep) {
    T v[kSweep];
#pragma unroll
    for (int u = 0; u < kSweep; ++u) v[u] = rec[j0 + u < n ? j0 + u : n - 1];
#pragma unroll
    for (int u = 0; u < kSweep; ++u)
      if (j0 + u < n) f(j0 + u, v[u]);
  }
}

__device__ inline ImageBox image_box_of(const CfgInfo& c, const SmallAtoms& sa, int li, int lj) {
  const float w0 = (float)c.w[0] + 1e-3f, w1 = (float)c.w[1] + 1e-3f, w2 = (float)c.w[2] + 1e-3f;
  const float4 ui = sa.u[li], uj = sa.u[lj];
  const float s0 = uj.x - ui.x, s1 = uj.y - ui.y, s2 = uj.z - ui.z;
  const int4 mi = sa.mz[li], mj = sa.mz[lj];
  const int o0 = mi.x - mj.x, o1 = mi.y - mj.y, o2 = mi.z - mj.z;
  const double4 pi = sa.x[li], pj = sa.x[lj];
  ImageBox q;
  q.lo0 = -(int)floorf(w0 + s0) + o0; q.hi0 = (int)floorf(w0 - s0) + o0;
  q.lo1 = -(int)floorf(w1 + s1) + o1; q.hi1 = (int)floorf(w1 - s1) + o1;
  q.lo2 = -(int)floorf(w2 + s2) + o2; q.hi2 = (int)floorf(w2 - s2) + o2;
  q.dx = pj.x - pi.x; q.dy = pj.y - pi.y; q.dz = pj.z - pi.z;
  return q;
}

// The pair vector of atom lj's nearest image for atom li in a nearest cell.
__device__ inline void nearest_vector(const CfgInfo& c, const SmallAtoms& sa, int li, int lj, double& rx, double& ry,
                                      double& rz) {
  const float4 ui = sa.u[li], uj = sa.u[lj];
  const int4 mi = sa.mz[li], mj = sa.mz[lj];
  const double4 pi = sa.x[li], pj = sa.x[lj];
  // n = n' - m_j + m_i with n' = -rint(u_j - u_i)
  const int n0 = -(int)rintf(uj.x - ui.x) + mi.x - mj.x;
  const int n1 = -(int)rintf(uj.y - ui.y) + mi.y - mj.y;
  const int n2 = -(int)rintf(uj.z - ui.z) + mi.z - mj.z;
  const double* L = c.L;
  rx = (pj.x - pi.x) + ((double)n0 * L[0] + (double)n1 * L[3] + (double)n2 * L[6]);
  ry = (pj.y - pi.y) + ((double)n0 * L[1] + (double)n1 * L[4] + (double)n2 * L[7]);
  rz = (pj.z - pi.z) + ((double)n0 * L[2] + (double)n1 * L[5] + (double)n2 * L[8]);
}

// All neighbours of atom li in list order: visit.pair(lj, r, r2) per entry,
// visit.run_end(lj, k) after the k images of each neighbour.
template <typename Visit>
__device__ inline void small_candidates(const CfgInfo& c, const SmallAtoms& sa, int n, int li, double rc2,
                                        Visit&& visit) {
  const double4 pi = sa.x[li];
  if (!c.pbc) {
    for (int lj = 0; lj < n; ++lj) {
      const double4 pj = sa.x[lj];
      const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (lj != li && r2 < rc2) {
        visit.pair(lj, dx, dy, dz, r2);
        visit.run_end(lj, 1);
      }
    }
    return;
  }
  // Periodic cell.  Most atoms have no image within reach (an empty box) and
  // the others a few, differently many per lane; looping over each atom's
  // box in step would keep the wavefront for the largest box of every atom.
  // Instead phase A marks, in a bit mask over the configuration's atoms, the
  // atoms whose box may hold an image (all lanes test the same atom, LDS
  // broadcasts), and phase B walks the marked atoms' images as one flat
  // sequence per lane: one image per iteration, the next marked atom taken
  // when a box is exhausted, so lanes stay busy until their own last image.
  const float4 ui = sa.u[li];
  uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;   // n <= 256 atoms
#pragma unroll
  for (int wi = 0; wi < 4; ++wi) {
    uint64_t bits = 0;
    const int top = n - 64 * wi < 64 ? n - 64 * wi : 64;
    lds_sweep(sa.u + 64 * wi, top, [&](int bi, float4 uj) {
      if (box_may_hit(c, ui, uj)) bits |= 1ull << bi;
    });
    if (wi == 0) m0 = bits; else if (wi == 1) m1 = bits; else if (wi == 2) m2 = bits; else m3 = bits;
  }
  const double* L = c.L;
  ImageBox q{0, 0, 0, -1, 0, 0, 0.0, 0.0, 0.0};
  int lj = -1, k = 0, wbase = 0, n0 = 0, n1 = 0, n2 = 0;
  while (true) {
    if (n0 > q.hi0) {   // box exhausted: the next marked atom with a non-empty box
      if (k > 0) visit.run_end(lj, k);
      k = 0;
      bool found = false;
      while (true) {
        while (m0 == 0 && wbase < 192) {
          m0 = m1; m1 = m2; m2 = m3; m3 = 0;
          wbase += 64;
        }
        if (m0 == 0) break;
        lj = wbase + __builtin_ctzll(m0);
        m0 &= m0 - 1;
        q = image_box_of(c, sa, li, lj);
        if (q.lo0 <= q.hi0 && q.lo1 <= q.hi1 && q.lo2 <= q.hi2) {
          found = true;
          break;
        }
      }
      if (!found) break;
      n0 = q.lo0; n1 = q.lo1; n2 = q.lo2;
    }
    if (!(lj == li && n0 == 0 && n1 == 0 && n2 == 0)) {
      const double sx = (double)n0 * L[0] + (double)n1 * L[3] + (double)n2 * L[6];
      const double sy = (double)n0 * L[1] + (double)n1 * L[4] + (double)n2 * L[7];
      const double sz = (double)n0 * L[2] + (double)n1 * L[5] + (double)n2 * L[8];
      const double rx = q.dx + sx, ry = q.dy + sy, rz = q.dz + sz;
      const double r2 = rx * rx + ry * ry + rz * rz;
      if (r2 < rc2) {
        visit.pair(lj, rx, ry, rz, r2);
        ++k;
      }
    }
    if (++n2 > q.hi2) {
      n2 = q.lo2;
      if (++n1 > q.hi1) {
        n1 = q.lo1;
        ++n0;
      }
    }
  }
}

// Two-phase list of one atom for nearest cells: phase A walks all atoms j
// with the cheap test only (the FP32 nearest-image box and distance) and
// records the candidates j in the atom's LDS row; phase B tests only the
// candidates with the exact FP64 pair vector and rewrites the row in place
// (kept entries never outrun the candidates).  A free cluster's test is the
// exact FP64 distance, so its walk hands the neighbours to visit directly.
// Returns the candidate count (> K means the row overflowed).
template <typename Visit>
__device__ inline int small_two_phase(const CfgInfo& c, const SmallAtoms& sa, int n, int li, double rc2, int K,
                                      uint8_t* row, Visit&& visit) {
  const double4 pi = sa.x[li];
  int nc = 0;
  if (!c.pbc) {
    // a cluster's cheap test is already the exact one: the candidates are the
    // neighbours, handed to visit in order (no second phase)
    lds_sweep(sa.x, n, [&](int lj, double4 pj) {
      const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      if ((lj != li) & (r2 < rc2)) {
        visit.pair(lj, dx, dy, dz, r2);
        ++nc;
      }
    });
    return nc;
  }
  const float w0 = (float)c.w[0] + 1e-3f, w1 = (float)c.w[1] + 1e-3f, w2 = (float)c.w[2] + 1e-3f;
  const float4 ui = sa.u[li];
  // FP32 estimate of the nearest-image distance, with a margin far above its
  // rounding error, so that nearly every candidate is a neighbour
  float Lf[9];
  for (int t = 0; t < 9; ++t) Lf[t] = (float)c.L[t];
  const float rcm = (float)sqrt(rc2) + 1e-3f, rcm2 = rcm * rcm;
  lds_sweep(sa.u, n, [&](int lj, float4 uj) {
    const float s0 = uj.x - ui.x, s1 = uj.y - ui.y, s2 = uj.z - ui.z;
    const float f0 = s0 - rintf(s0), f1 = s1 - rintf(s1), f2 = s2 - rintf(s2);
    const float x = f0 * Lf[0] + f1 * Lf[3] + f2 * Lf[6];
    const float y = f0 * Lf[1] + f1 * Lf[4] + f2 * Lf[7];
    const float z = f0 * Lf[2] + f1 * Lf[5] + f2 * Lf[8];
    // the atom's own nearest image is itself (n = 0) and no other image is in range
    const bool skip = (lj == li) | (fabsf(f0) > w0) | (fabsf(f1) > w1) | (fabsf(f2) > w2) |
                      (x * x + y * y + z * z > rcm2);
    if (!skip) {
      if (nc < K) row[nc] = (uint8_t)lj;
      ++nc;
    }
  });
  const int m = nc < K ? nc : K;
  for (int q = 0; q < m; ++q) {
    const int lj = row[q];
    double rx, ry, rz;
    nearest_vector(c, sa, li, lj, rx, ry, rz);
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 < rc2) visit.pair(lj, rx, ry, rz, r2);
  }
  return nc;
}

// LDS list of one atom: local neighbour index per slot, counters.
struct LdsCollect {
  uint8_t* row;
  int K;
  double rmin2;
  int count = 0, below = 0;
  __device__ void pair(int lj, double, double, double, double r2) {
    if (count < K) row[count] = (uint8_t)lj;
    if (r2 < rmin2) ++below;
    ++count;
  }
  __device__ void run_end(int, int) {}
};

// LDS list plus direct records of one atom (periodic cells with several
// images per neighbour, whose write-out would have to enumerate boxes again).
struct LdsAndRecords {
  const NbrArgs& a;
  int64_t i, start;
  const int4* mz;
  uint8_t* row;
  double rmin2;
  int count = 0, below = 0;
  __device__ void pair(int lj, double rx, double ry, double rz, double r2) {
    if (count < a.K) {
      const size_t e = (size_t)count * a.stride + i;
      a.nbr[e] = (int32_t)(start + lj);
      store_pair(a, e, rx, ry, rz, mz[lj].w);
      row[count] = (uint8_t)lj;
    }
    if (r2 < rmin2) ++below;
    ++count;
  }
  __device__ void run_end(int, int) {}
};

// Direct lists (K > kLdsSlots): records, neighbour indices and run starts.
struct SmallEmit {
  const NbrArgs& a;
  int64_t i, start;
  const int4* mz;
  int16_t* my_starts;
  double rmin2;
  int count = 0, below = 0, before = 0;
  __device__ void pair(int lj, double rx, double ry, double rz, double r2) {
    if (count < a.K) {
      const size_t e = (size_t)count * a.stride + i;
      a.nbr[e] = (int32_t)(start + lj);
      store_pair(a, e, rx, ry, rz, mz[lj].w);
    }
    if (r2 < rmin2) ++below;
    ++count;
  }
  __device__ void run_end(int lj, int) {
    if (before < a.K) my_starts[lj] = (int16_t)before;
    before = count;
  }
};

// A workgroup of the small search takes a bundle of configurations, each on
// whole wavefronts of its own (ceil(n / 64) of them, atom li on lane li % 64
// of its (li / 64)-th wavefront), so that few of the workgroup's four
// wavefronts idle and more of them share the CU.  Bundles, from the class
// counts after cfg_order (configurations in descending size, so the classes
// are contiguous there): each 4-wavefront configuration alone; each
// 3-wavefront one with a 1-wavefront one while they last; 2-wavefront ones in
// pairs, an odd one left over with up to two 1-wavefront ones; the remaining
// 1-wavefront ones in fours.  Workgroups past the last bundle find none.
struct SmallSlot {
  int pos;     // position of the wavefront's configuration in cfg_order, -1: idle
  int wave0;   // the configuration's first wavefront in the workgroup
};

__device__ inline SmallSlot bundle_slot(const NbrArgs& a, int b, int wave) {
  const int* cls = a.cfg_order + a.n_cfg;
  const int c1 = cls[0], c2 = cls[1], c3 = cls[2], c4 = cls[3];
  const int s3 = c4, s2 = c4 + c3, s1 = c4 + c3 + c2;   // first positions of the classes
  const int u1a = c3 < c1 ? c3 : c1;                     // 1-wavefront ones beside 3-wavefront ones
  const int p2 = c2 >> 1, odd2 = c2 & 1;
  const int u1b = odd2 ? (c1 - u1a < 2 ? c1 - u1a : 2) : 0;   // beside the odd 2-wavefront one
  int pos[4] = {-1, -1, -1, -1}, nw[4] = {0, 0, 0, 0};
  if (b < c4) {
    pos[0] = b;
    nw[0] = 4;
  } else if (b - c4 < c3) {
    const int q = b - c4;
    pos[0] = s3 + q;
    nw[0] = 3;
    if (q < u1a) {
      pos[1] = s1 + q;
      nw[1] = 1;
    }
  } else if (b - c4 - c3 < p2) {
    const int q = b - c4 - c3;
    pos[0] = s2 + 2 * q;
    pos[1] = s2 + 2 * q + 1;
    nw[0] = nw[1] = 2;
  } else if (b - c4 - c3 - p2 < odd2) {
    pos[0] = s2 + c2 - 1;
    nw[0] = 2;
    for (int t = 0; t < u1b; ++t) {
      pos[1 + t] = s1 + u1a + t;
      nw[1 + t] = 1;
    }
  } else {
    const int q = u1a + u1b + 4 * (b - c4 - c3 - p2 - odd2);
    for (int t = 0; t < 4; ++t)
      if (q + t < c1) {
        pos[t] = s1 + q + t;
        nw[t] = 1;
      }
  }
  int w0 = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (pos[m] >= 0 && wave >= w0 && wave < w0 + nw[m]) return SmallSlot{pos[m], w0};
    w0 += nw[m];
  }
  return SmallSlot{-1, 0};
}

__global__ void __launch_bounds__(kSmallBlock) search_small_kernel(NbrArgs a, int lds_lists) {
  __shared__ double4 sx[kSmallMax];
  __shared__ float4 su[kSmallMax];
  __shared__ int4 smz[kSmallMax];
  __shared__ int32_t scount[kSmallMax];
  __shared__ unsigned long long red[5];
  extern __shared__ uint8_t lists[];   // [kSmallMax][K + 4] when lds_lists
  const int t = threadIdx.x;
  if (t < 5) red[t] = 0;
  // this wavefront's configuration in the workgroup's bundle (none: an idle wavefront)
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const SmallSlot slot = bundle_slot(a, blockIdx.x, wave);
  CfgInfo c{};
  if (slot.pos >= 0) c = a.cfg[a.cfg_order[slot.pos]];
  const int n = c.n;
  const int base = 64 * slot.wave0;   // LDS index of the configuration's first atom
  const int li = slot.pos >= 0 ? 64 * (wave - slot.wave0) + (t & 63) : kSmallMax;
  double4* const sxc = sx + base;
  float4* const suc = su + base;
  int4* const smzc = smz + base;
  int32_t* const scc = scount + base;
  const int KL = a.K + 4;   // row pitch in bytes: rows of consecutive atoms fall in different banks
  uint8_t* const lc = lists + (size_t)base * KL;
  int bad = 0;
  if (li < n) {
    const size_t g = (size_t)(c.start + li);
    const double x = a.pos[3 * g], y = a.pos[3 * g + 1], z = a.pos[3 * g + 2];
    sxc[li] = make_double4(x, y, z, 0.0);
    const int zs = a.species[g];
    if (zs < 0 || zs >= a.n_species) bad = 1;
    int m[3] = {0, 0, 0};
    float u[3] = {0.f, 0.f, 0.f};
    if (c.pbc)
      for (int d = 0; d < 3; ++d) {
        const double f = x * c.inv[0 * 3 + d] + y * c.inv[1 * 3 + d] + z * c.inv[2 * 3 + d];
        const double fl = floor(f);
        u[d] = (float)(f - fl);
        m[d] = (int32_t)fl;
      }
    suc[li] = make_float4(u[0], u[1], u[2], 0.f);
    smzc[li] = make_int4(m[0], m[1], m[2], zs < 0 ? 0 : (zs >= a.n_species ? a.n_species - 1 : zs));
  }
  __syncthreads();
  const SmallAtoms sa{sxc, suc, smzc};
  const double rc2 = a.rcut * a.rcut;
  const double rmin2 = a.rmin * a.rmin;
  const bool nearest = nearest_cell(c);
  // global run starts (direct lists): rows of n int16 at the config's atom offset
  int16_t* run_start = a.run_start + (size_t)c.start * kSmallMax;
  int count = 0, below = 0;
  if (li < n) {
    const int64_t i = c.start + li;
    if (lds_lists) {
      uint8_t* row = lc + (size_t)li * KL;
      LdsCollect col{row, a.K, rmin2};
      if (!c.pbc || nearest) {
        const int nc = small_two_phase(c, sa, n, li, rc2, a.K, row, col);
        // a candidate overflow is reported like a neighbour overflow (the
        // call is repeated with capacity for every candidate)
        if (nc > a.K && col.count <= a.K) col.count = nc;
        count = col.count;
        below = col.below;
      } else {
        LdsAndRecords em{a, i, c.start, smzc, row, rmin2};
        small_candidates(c, sa, n, li, rc2, em);
        count = em.count;
        below = em.below;
      }
    } else {
      SmallEmit em{a, i, c.start, smzc, run_start + (size_t)li * n, rmin2};
      small_candidates(c, sa, n, li, rc2, em);
      count = em.count;
      below = em.below;
    }
    a.count[i] = count < a.K ? count : a.K;
    scc[li] = count < a.K ? count : a.K;
  }
  // counts summed over the wavefront first: one LDS atomic per wavefront
  const int wmax = wave_max(count), wsum = wave_sum(count), wover = wave_sum(count > a.K ? 1 : 0);
  const int wbelow = wave_sum(below), wbad = wave_sum(bad);
  if ((t & 63) == 0) {
    atomicMax(&red[0], (unsigned long long)wmax);
    atomicAdd(&red[1], (unsigned long long)wsum);
    if (wover) atomicAdd(&red[2], (unsigned long long)wover);
    if (wbelow) atomicAdd(&red[3], (unsigned long long)wbelow);
    if (wbad) atomicAdd(&red[4], (unsigned long long)wbad);
  }
  __syncthreads();  // LDS lists and counts of every configuration of the bundle are complete
  if (t == 0) {
    atomicMax(&a.status->max_count, red[0]);
    atomicAdd(&a.status->n_pairs, red[1]);
    if (red[2]) atomicAdd(&a.status->overflow, red[2]);
    if (red[3]) atomicAdd(&a.status->below_rmin, red[3]);
    if (red[4]) atomicAdd(&a.status->bad_species, red[4]);
  }
  // Write-out, also when an atom overflowed its K slots (the call is then
  // repeated with more slots, but the kernels that follow in this attempt
  // read the first K slots of every list, which must hold valid records and
  // reverse indices).  Slot by slot, consecutive atoms store consecutive
  // records (cells with several images per neighbour stored theirs in the
  // search).
  if (!lds_lists || li >= n) return;
  const int64_t i = c.start + li;
  const uint8_t* mine = lc + (size_t)li * KL;
  const int ci = scc[li];
  const bool records = !c.pbc || nearest;
  unsigned long long errs = 0;
  // kWriteGroup entries at a time, their binary searches in lockstep so that
  // the dependent LDS loads of different entries overlap
  constexpr int G = kWriteGroup;
  for (int p0 = 0; p0 < ci; p0 += G) {
    int ljv[G], lo[G], hi[G], rr[G], kk[G];
#pragma unroll
    for (int u = 0; u < G; ++u) ljv[u] = mine[p0 + u < ci ? p0 + u : ci - 1];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      lo[u] = 0;
      hi[u] = scc[ljv[u]];
      rr[u] = 0;
      kk[u] = 1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int p = p0 + u;
      if (p >= ci) continue;
      const int lj = ljv[u];
      const size_t e = (size_t)p * a.stride + i;
      if (records) {
        double rx, ry, rz;
        if (!c.pbc) {
          const double4 pi = sxc[li], pj = sxc[lj];
          rx = pj.x - pi.x; ry = pj.y - pi.y; rz = pj.z - pi.z;
        } else {
          nearest_vector(c, sa, li, lj, rx, ry, rz);
        }
        store_pair(a, e, rx, ry, rz, smzc[lj].w);
        a.nbr[e] = (int32_t)(c.start + lj);
      } else {
        // rank of this image in the run of lj, and the run length
        int r = 0, k = 1;
        while (p - r - 1 >= 0 && mine[p - r - 1] == lj) ++r;
        while (p - r + k < ci && mine[p - r + k] == lj) ++k;
        rr[u] = r;
        kk[u] = k;
      }
    }
    // start of the run of li in each lj's list (ascending local indices);
    // mid <= count <= K stays inside the row of K + 4 bytes
    while (true) {
      bool more = false;
#pragma unroll
      for (int u = 0; u < G; ++u) more |= lo[u] < hi[u];
      if (!more) break;
      int v[G];
#pragma unroll
      for (int u = 0; u < G; ++u) v[u] = lc[(size_t)ljv[u] * KL + ((lo[u] + hi[u]) >> 1)];
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (lo[u] < hi[u]) {
          const int mid = (lo[u] + hi[u]) >> 1;
          if (v[u] < li) lo[u] = mid + 1; else hi[u] = mid;
        }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int p = p0 + u;
      if (p >= ci) continue;
      const int lj = ljv[u];
      const size_t e = (size_t)p * a.stride + i;
      const int64_t j = c.start + lj;
      const int cj = scc[lj];
      const int q = lo[u] + kk[u] - 1 - rr[u];
      if (q < cj && lc[(size_t)lj * KL + q] == (uint8_t)li) {
        a.rev[e] = (int32_t)((size_t)q * a.stride + j);
      } else {
        a.rev[e] = (int32_t)e;
        ++errs;
      }
    }
  }
  if (errs) atomicAdd(&a.status->list_errors, errs);
}

// ---------------------------------------------------------------------------
// Verlet skin: lists built with R_cut + skin are reused while every atom stays
// within skin / 2 of its position at the build (then no pair that was beyond
// R_cut + skin can have come within R_cut).  The records are refreshed from
// the positions on every reuse.

__global__ void __launch_bounds__(kBlock) max_disp_kernel(const double* __restrict__ pos,
                                                          const double* __restrict__ xb, int64_t n,
                                                          unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (i < n) {
    const double dx = pos[3 * i] - xb[3 * i], dy = pos[3 * i + 1] - xb[3 * i + 1], dz = pos[3 * i + 2] - xb[3 * i + 2];
    d2 = dx * dx + dy * dy + dz * dz;
  }
  for (int o = 32; o > 0; o >>= 1) d2 = fmax(d2, __shfl_xor(d2, o, 64));
  __shared__ double part[kBlock / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, part[w]);
    // non-negative doubles order like their bit patterns
    if (m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

// Image shift of slot p of atom i: n = rint((r - (x_j - x_i)) . L^-1).
__global__ void pair_images_kernel(NbrArgs a, short4* img) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= a.n_atoms || p >= a.count[i]) return;
  const CfgInfo& c = a.cfg[a.atom_cfg[i]];
  const size_t e = (size_t)p * a.stride + i;
  const int32_t j = a.nbr[e];
  double rx, ry, rz;
  if (a.fp64) {
    const PairRec<double> q = ((const PairRec<double>*)a.pr)[e];
    rx = q.x; ry = q.y; rz = q.z;
  } else {
    const PairRec<float> q = ((const PairRec<float>*)a.pr)[e];
    rx = q.x; ry = q.y; rz = q.z;
  }
  const double sx = rx - (a.pos[3 * j] - a.pos[3 * i]);
  const double sy = ry - (a.pos[3 * j + 1] - a.pos[3 * i + 1]);
  const double sz = rz - (a.pos[3 * j + 2] - a.pos[3 * i + 2]);
  int n[3] = {0, 0, 0};
  bool bad = false;
  if (c.pbc)
    for (int d = 0; d < 3; ++d) {
      const double v = rint(sx * c.inv[0 * 3 + d] + sy * c.inv[1 * 3 + d] + sz * c.inv[2 * 3 + d]);
      bad = bad || !(fabs(v) <= 32767.0);
      n[d] = bad ? 0 : (int)v;
    }
  if (bad) atomicAdd(&a.status->list_errors, 1ull);
  img[e] = make_short4((short)n[0], (short)n[1], (short)n[2], 0);
}

__global__ void refresh_pairs_kernel(NbrArgs a, const short4* __restrict__ img) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  int below = 0;
  if (i < a.n_atoms && p < a.count[i]) {
    const CfgInfo& c = a.cfg[a.atom_cfg[i]];
    const size_t e = (size_t)p * a.stride + i;
    const int32_t j = a.nbr[e];
    const short4 n = img[e];
    const double* L = c.L;
    const double dx = a.pos[3 * j] - a.pos[3 * i], dy = a.pos[3 * j + 1] - a.pos[3 * i + 1],
                 dz = a.pos[3 * j + 2] - a.pos[3 * i + 2];
    const double sx = (double)n.x * L[0] + (double)n.y * L[3] + (double)n.z * L[6];
    const double sy = (double)n.x * L[1] + (double)n.y * L[4] + (double)n.z * L[7];
    const double sz = (double)n.x * L[2] + (double)n.y * L[5] + (double)n.z * L[8];
    const double rx = dx + sx, ry = dy + sy, rz = dz + sz;
    const double r2 = rx * rx + ry * ry + rz * rz;
    int zj = a.species[j];
    zj = zj < 0 ? 0 : (zj >= a.n_species ? a.n_species - 1 : zj);
    if (r2 < a.rcut * a.rcut) {
      store_pair(a, e, rx, ry, rz, zj);
      if (r2 < a.rmin * a.rmin) below = 1;
    } else {
      store_pair(a, e, a.rcut, 0.0, 0.0, zj);
    }
  }
  below = wave_sum(below);
  if ((threadIdx.x & 63) == 0 && below) atomicAdd(&a.status->below_rmin, (unsigned long long)below);
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

hipError_t zero_words(int32_t* p, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(zero_kernel, grid_for(n), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t max_displacement(const double* pos, const double* xbuild, int64_t n_atoms,
                            unsigned long long* out, hipStream_t s) {
  if (n_atoms > 0) hipLaunchKernelGGL(max_disp_kernel, grid_for(n_atoms), dim3(kBlock), 0, s, pos, xbuild, n_atoms, out);
  return hipGetLastError();
}

hipError_t pair_images(const NbrArgs& a, short4* img, hipStream_t s) {
  if (a.n_atoms == 0 || a.K == 0) return hipSuccess;
  const dim3 g((unsigned)((a.n_atoms + kBlock - 1) / kBlock), (unsigned)a.K);
  hipLaunchKernelGGL(pair_images_kernel, g, dim3(kBlock), 0, s, a, img);
  return hipGetLastError();
}

hipError_t refresh_pairs(const NbrArgs& a, const short4* img, hipStream_t s) {
  if (a.n_atoms == 0 || a.K == 0) return hipSuccess;
  const dim3 g((unsigned)((a.n_atoms + kBlock - 1) / kBlock), (unsigned)a.K);
  hipLaunchKernelGGL(refresh_pairs_kernel, g, dim3(kBlock), 0, s, a, img);
  return hipGetLastError();
}

hipError_t nbr_build(NbrArgs& a, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  if (a.n_cfg > 0)
    hipLaunchKernelGGL(cfg_prepare_kernel, grid_for(a.n_cfg), dim3(kBlock), 0, s, a);
  if (a.n_atoms == 0) return hipGetLastError();
  hipLaunchKernelGGL(atom_cfg_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, s, a);
  // every atom's count is written by this call (atoms of an invalid range keep 0)
  hipLaunchKernelGGL(zero_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, s, a.count, a.n_atoms);
  const int lds_lists = a.K <= kLdsSlots ? 1 : 0;
  const size_t lds = lds_lists ? (size_t)kSmallMax * (a.K + 4) : 0;
  // The searches of small and of large configurations write the rows of
  // disjoint atoms: under graph capture the large ones (bins, cell-list and
  // direct searches, and with LDS lists their reverse indices) form a branch
  // on the side stream beside the small-configuration search, joined back
  // before returning.  Launched eagerly they stay on s: there the two
  // cross-stream waits cost more (about 30 us) than the overlap saves.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return e;
  const bool branch = cap == hipStreamCaptureStatusActive;
  if (!branch) side = s;
  if (branch) {
    e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(zero_kernel, grid_for(a.n_atoms + 1), dim3(kBlock), 0, side, a.bin_count, a.n_atoms + 1);
  hipLaunchKernelGGL(bin_count_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, side, a);
  if (a.n_cfg > 0) hipLaunchKernelGGL(bin_scan_kernel, dim3(a.n_cfg), dim3(256), 0, side, a);
  hipLaunchKernelGGL(bin_fill_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, side, a);
  hipLaunchKernelGGL(bin_sort_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, side, a);
  hipLaunchKernelGGL(search_kernel, grid_for(a.n_atoms), dim3(kBlock), 0, side, a);
  hipLaunchKernelGGL(search_binned_kernel, dim3(kBinnedBlocks), dim3(kBinnedBlock), 0, side, a);
  const dim3 g((unsigned)((a.n_atoms + kBlock - 1) / kBlock), (unsigned)a.K);
  if (lds_lists)
    hipLaunchKernelGGL(reverse_large_kernel, dim3(g.x < kReverseBlocks ? g.x : kReverseBlocks, g.y), dim3(kBlock), 0,
                       side, a);
  e = hipGetLastError();
  if (e == hipSuccess && branch) e = hipEventRecord(join, side);
  if (e != hipSuccess) return e;
  if (a.n_cfg > 0) {
    hipLaunchKernelGGL(cfg_order_kernel, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(search_small_kernel, dim3(a.n_cfg), dim3(kSmallBlock), lds, s, a, lds_lists);
  }
  if (branch) {
    e = hipStreamWaitEvent(s, join, 0);
    if (e != hipSuccess) return e;
  }
  // without LDS lists every list's reverse indices come after both searches
  if (!lds_lists) hipLaunchKernelGGL(reverse_kernel, g, dim3(kBlock), 0, s, a, lds_lists);
  return hipGetLastError();
}

}  // namespace mtp
