// Host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "status.h"

namespace mtp {

// Per-configuration geometry prepared on the device before the neighbour search.
struct CfgInfo {
  double L[9];      // lattice vectors as rows
  double inv[9];    // inverse of L (fractional = x . inv)
  double w[3];      // R_cut / interplanar spacing of each lattice plane family
  int64_t start;    // first atom
  int32_t n;        // atoms
  int32_t pbc;      // 1 periodic, 0 cluster
  int32_t binned;   // 1 if the cell-list search is used
  int32_t nb[3];    // bins per axis (binned configs)
  int64_t bin0;     // first bin of this config in the global bin arrays
};


// Neighbour capacity up to which the small-configuration search builds its
// lists in LDS (above it, it writes them directly and needs run_start).
constexpr int kLdsListSlots = 128;

struct NbrArgs {
  int n_cfg;
  int64_t n_atoms;
  const int64_t* atom_offsets;
  const double* pos;
  const int32_t* species;
  const double* cell;
  const uint8_t* pbc;
  double rcut, rmin;
  int n_species;
  CfgInfo* cfg;          // [n_cfg]
  int32_t* cfg_order;    // [n_cfg + 4] launch order of the small-configuration search, then the
                         // numbers of small configurations of 1, 2, 3 and 4 wavefronts
  int32_t* atom_cfg;     // [n_atoms]
  int32_t* atom_bin;     // [n_atoms] global bin index (binned configs only)
  int32_t* bin_count;    // [n_atoms + 1]  bins of a binned config sit at its atom offset
  int32_t* bin_start;    // [n_atoms + 1]
  int32_t* bin_atoms;    // [n_atoms] atoms sorted by bin, then index
  int32_t* bin_fill;     // [n_atoms + 1] scratch cursor
  int32_t* binned;       // [n_atoms] atoms of binned configurations, in no particular order
  int32_t* large;        // [n_atoms] atoms of configurations that are not small, in no particular order
  int32_t* count;        // [n_atoms] neighbours per atom (clamped to K)
  int stride;            // ELL pitch (>= n_atoms)
  int K;                 // ELL slots per atom
  int32_t* nbr;          // [K * stride] neighbour home index of slot p of atom i at p * stride + i
  void* pr;              // [K * stride] PairRec<double> or PairRec<float>
  int fp64;              // pair record type
  int32_t* rev;          // [K * stride] ELL index of the reverse pair
  int16_t* run_start;    // [n_atoms][256] scratch of the small-configuration search when
                         // K > kLdsListSlots (else unused, may be null)
  Status* status;
};

// Neighbour search without host synchronisation: prepare configs and bins,
// fill the ELL lists up to K slots (counting overflow), reverse indices.
// Under graph capture the large configurations' searches run on `side`
// (forked from and joined back to s with the two events); the results are
// complete in s order either way.
hipError_t nbr_build(NbrArgs& a, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join);

// Verlet skin (lists built with R_cut + skin and reused while every atom
// stays within skin / 2 of its position at the build).
// Largest squared displacement |x_i - x_build_i|^2 over the atoms, as the
// bits of a non-negative double in *out (which must start at zero).
hipError_t max_displacement(const double* pos, const double* xbuild, int64_t n_atoms,
                            unsigned long long* out, hipStream_t s);
// After a build: the image shift n of every stored pair (r = x_j - x_i + n.L),
// as int16 triples in img [K * stride] (entry 3 unused).
hipError_t pair_images(const NbrArgs& a, short4* img, hipStream_t s);
// Pair records of every stored pair recomputed from the positions and img,
// the same expression as the search; a pair at or beyond R_cut = a.rcut gets
// the record (R_cut, 0, 0), whose radial factor (R_cut - r)^2 and its
// derivative vanish, so it adds exactly nothing.  Counts pairs below R_min.
hipError_t refresh_pairs(const NbrArgs& a, const short4* img, hipStream_t s);

// Sets n 32-bit words to zero with a kernel (capturable, unlike memset nodes).
hipError_t zero_words(int32_t* p, int64_t n, hipStream_t s);

// Forces F_i = own_i - sum over slots g_rev(p), own_i = sum_p g_p summed by
// the last adjoint pass ([3][stride], FP64); g packed [K * stride][3];
// nothing is launched when forces is null.
hipError_t gather_forces(int fp64, int64_t n_atoms, int stride, const int32_t* count,
                         const int32_t* rev, const void* g, const double* own, double* forces, hipStream_t s);

// Per-configuration sums of site energies, virials and B (kernel order ->
// file order through perm, which maps file index -> kernel index), over the
// validated atom ranges of cfg, as chunked row sums (reduce.hip): the work
// items come from reduce_items (once per batch, after the search), and
// partial holds reduce_max_items x reduce_rows doubles (per stream when
// several reductions run at once).
struct ReduceItems {
  int max_items;            // reduce_max_items(n_cfg, n_atoms)
  const int32_t* item_start;  // [n_cfg + 1]
  const int32_t* item_cfg;    // [max_items]
  double* partial;          // [max_items][rows]
};
int reduce_max_items(int n_cfg, int64_t n_atoms);
int reduce_rows(int has_virial, int m, bool b);
hipError_t reduce_items(int n_cfg, const CfgInfo* cfg, int max_items, int32_t* item_start, int32_t* item_cfg,
                        hipStream_t s);
hipError_t reduce_configs(int fp64, int n_cfg, const CfgInfo* cfg, int stride,
                          const void* site, const void* atom_virial, const void* B, int m,
                          int b_stride, const int32_t* perm, double* energy, double* virial,
                          double* b, double* site_out, const ReduceItems& items, hipStream_t s);

// Normal equations in xi (fit.hip).  Ja is column-major [m + 1][R]: columns
// 0..m-1 the Jacobian, column m the targets.
hipError_t fit_rows(int n_cfg, int64_t N, int64_t R, const CfgInfo* cfg, const int32_t* atom_cfg, double we,
                    double wf, double ws, int scaling, const double* Et, const double* Ft, const double* Wt,
                    double* w, double* y, hipStream_t s);
int gram_splits(int n, int64_t R);
hipError_t gram(int n, int64_t R, const double* Ja, const double* w, double* P, int splits, int accumulate,
                double* H, double* g, double* yy, hipStream_t s);
hipError_t fill_eye(int fp64, int m, void* eye, hipStream_t s);
hipError_t solve_prepare(int m, const double* H, double* D, double* W2, hipStream_t s);
hipError_t solve_apply(int m, const double* inv, const double* D, const double* g, double* xi, hipStream_t s);

// Weights (a, b, c) of energy, force and stress terms of one configuration
// of n atoms under a weighting of eq. Fitting: 0 molecules (as written),
// 1 structures (eq. train-structures), 2 vibrations (eq. train-vibrations).
__device__ inline void weights(int scaling, double n, double we, double wf, double ws, double& a, double& b,
                               double& c) {
  if (scaling == 1) {
    a = we / (n * n); b = wf / n; c = ws / (n * n);
  } else if (scaling == 2) {
    a = we / n; b = wf; c = ws / n;
  } else {
    a = we; b = wf; c = ws;
  }
}

// Residuals of the training loss (per configuration and per atom).
struct LossResidualArgs {
  int n_cfg;
  int64_t N;
  int stride;
  const CfgInfo* cfg;
  const int32_t* atom_cfg;
  const double* E;    // [n_cfg] predictions
  const double* F;    // [N][3]
  const double* W;    // [n_cfg][9]
  const double* Et;   // targets
  const double* Ft;
  const double* Wt;
  double we, wf, ws;
  int scaling;        // 0 molecules, 1 structures, 2 vibrations
  double* a_cfg;      // [n_cfg]
  double* wf_cfg;     // [n_cfg]
  double* eps_cfg;    // [n_cfg][9]
  double* loss_cfg;   // [n_cfg]
  double* loss_atom;  // [N]
};
// Rows dE_k/dtheta of the nonlinear grade (loss.hip): theta_rows_prepare sets
// a = 1, u = 0, eps = 0 for the loss kernels; theta_rows_finish sums their
// per-pair c coefficients per configuration into rows[k][m + t] and copies
// b_k (file order) into rows[k][0 .. m).
struct ThetaRowArgs {
  int n_cfg;
  const CfgInfo* cfg;
  int stride, K;
  const int32_t* count;
  const int32_t* species;
  int n_mu, n_species, nq;
  double rmin, rcut;
  int m, n_c;
  double* rows;   // [n_cfg][m + n_c]
};
hipError_t theta_rows_prepare(int fp64, int64_t N, int stride, void* a_atom, void* u, void* eps_atom, hipStream_t s);
hipError_t theta_rows_finish(int fp64, const ThetaRowArgs& a, const void* pr, const void* pa, const void* pb,
                             const double* b, hipStream_t s);

hipError_t loss_residuals(LossResidualArgs& r, int fp64, void* a_atom, void* u, void* eps_atom, hipStream_t s);
// Loss and gradient from the per-configuration and per-atom loss terms, the
// per-atom xi terms and the per-workgroup c partials, all sums in a fixed
// order; part: loss_finish_scratch_doubles(m) doubles of device scratch.
hipError_t loss_finish(int fp64, int n_cfg, int64_t N, int stride, int m, int n_c, int n_blocks,
                       const double* loss_cfg, const double* loss_atom, const void* xi_terms, const int32_t* perm,
                       const double* cpart, double* part, double* loss, double* grad, hipStream_t s);
int loss_finish_scratch_doubles(int m);
// dL/dx [N][3] from the forces F of the evaluation, a per atom and the
// per-pair values hvp of the position passes (see grad_pos_kernel).
hipError_t loss_grad_pos(int fp64, int64_t N, int stride, const int32_t* count, const int32_t* rev, const void* hvp,
                         const void* a_atom, const double* F, double* out, hipStream_t s);

// MaxVol selection (section 2.3): the largest |C_ij| and where it is.
struct MaxvolPick {
  double value;
  int32_t i, j;
};
// Pivot rows of Gaussian elimination with partial pivoting of W [K][m]
// (columns equilibrated first; W and perm [K] are overwritten), ascending.
hipError_t maxvol_pivot_rows(int K, int m, double* W, int32_t* perm, int32_t* rows, int* singular, hipStream_t s);
// [A | I] [m][2m] with A = pool[rows].
hipError_t maxvol_gather(int m, const double* pool, const int32_t* rows, double* W, hipStream_t s);
// Largest entry over the per-row maxima (lowest row on ties).
hipError_t maxvol_pick(int K, const double* rowmax, const int32_t* rowarg, MaxvolPick* out, hipStream_t s);
// Rank-one update of C [K][m] for the swap in *pick; rows[pick->j] = pick->i.
hipError_t maxvol_swap(int K, int m, double* C, const MaxvolPick* pick, double* colj, double* rowi, int32_t* rows,
                       hipStream_t s);

// Velocity Verlet: v += (dt/2) F/m (masses per species, 1/m in amu^-1 on
// the device); with drift also x += dt v.
// Kinetic energy per configuration (md.hip), eV.
hipError_t md_kinetic(int n_cfg, int64_t n_atoms, const int64_t* offsets, const int32_t* species, int S,
                      const double* inv_mass, const double* vel, double* ekin, hipStream_t s);
// FIRE relaxation step per configuration (md.hip); state [n_cfg][4].
struct FireParams {
  double dt_max, f_inc, f_dec, alpha_start, f_alpha;
  double n_min;
};
hipError_t md_fire(int n_cfg, int64_t n_atoms, const int64_t* offsets, const int32_t* species, int S,
                   const double* inv_mass, double* pos, double* vel, const double* F, double* state,
                   const FireParams& fp, hipStream_t s);
hipError_t md_kick(int64_t n, const int32_t* species, int S, const double* inv_mass, double* pos, double* vel,
                   const double* F, double dt, int drift, hipStream_t s);

// Dense FP64 helpers of the grade.
hipError_t gauss_jordan_inverse(int m, double* work /*[m][2m]*/, double* inv, int* singular,
                                hipStream_t s);
hipError_t grade_rows(int n, int m, const double* b, const double* Ainv, double* gamma,
                      int32_t* argmax, double* c, hipStream_t s);
// Fixed device scratch of mtp_grade_from_b_noalloc (grade.hip): room for c
// of n x m doubles with n m <= kGradeScratchDoubles (16 MiB per GPU).
constexpr size_t kGradeScratchDoubles = size_t(1) << 21;
constexpr int kMaxGradeDevices = 256;
// Device address of that array on `device`, which must be the current
// device; looked up once per device and cached.
hipError_t grade_scratch_address(int device, double** out);
// Per row of c [n][m]: max |c| and its first index.
hipError_t row_maxima(int n, int m, const double* c, double* gamma, int32_t* argmax, hipStream_t s);

}  // namespace mtp
