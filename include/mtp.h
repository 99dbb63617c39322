/*
 * libmtp: Moment Tensor Potential evaluation on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every compute entry point is asynchronous on the HIP stream it is
 * given unless stated otherwise.  Pointers marked "device" must point to
 * memory of the model's device; the caller owns every batch and output
 * buffer; the model owns its parameters, its active-set inverse and a
 * grow-only workspace.  One model must not be used from two host threads at
 * once.  Functions return 0 on success or a negative MTP_E_* code; the text
 * of the last error on the calling thread is returned by mtp_last_error().
 *
 * The method is that of Novikov, Gubaev, Podryabinkin and Shapeev, "The MLIP
 * package: Moment Tensor Potentials with MPI and Active Learning" (2020),
 * section 2 ("Theory"); each entry point names the part it implements.
 */
#ifndef MTP_H
#define MTP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mtp_model mtp_model;

/* Return codes. */
enum {
  MTP_OK = 0,
  MTP_E_ARG = -1,      /* invalid argument (null pointer, size, species, ...) */
  MTP_E_FILE = -2,     /* potential file missing or malformed */
  MTP_E_HIP = -3,      /* a HIP runtime call failed */
  MTP_E_CAPACITY = -4, /* a size exceeds a documented limit */
  MTP_E_BASIS = -5,    /* the potential's basis is not compiled into this library */
  MTP_E_STATE = -6     /* call order violated (e.g. grade without an active set) */
};

/* Arithmetic of the evaluation kernels. */
typedef enum {
  MTP_FP64 = 0,              /* everything in FP64 */
  MTP_FP32 = 1,              /* pair vectors rounded from FP64 to FP32, FP32 arithmetic */
  MTP_FP32_COMPENSATED = 2,  /* as MTP_FP32, moments summed with an error-free TwoSum */
  MTP_MIXED = 3              /* moments M_{mu,nu} in FP32 from the FP64 pair
                                vectors (rounded per pair), stored in FP32;
                                contractions, dV/dM, the adjoint (g = dV/dr),
                                forces, virials, site energies and b in FP64.
                                Evaluation only (mtp_eval, mtp_eval_async,
                                mtp_grade) */
} mtp_precision;

/* Loss weightings of section 2.2: eq. Fitting as written, eq.
 * train-structures, eq. train-vibrations (the paper's default). */
typedef enum {
  MTP_SCALE_MOLECULES = 0,
  MTP_SCALE_STRUCTURES = 1,
  MTP_SCALE_VIBRATIONS = 2
} mtp_scaling;

/* A batch of configurations.  All pointers are device pointers. */
typedef struct {
  int32_t n_configs;
  int64_t n_atoms;              /* total over the batch */
  const int64_t* atom_offsets;  /* [n_configs + 1], atom_offsets[0] = 0, non-decreasing */
  const double* pos;            /* [n_atoms][3] Cartesian positions, Angstrom */
  const int32_t* species;       /* [n_atoms] type index z_i in [0, n_species) */
  const double* cell;           /* [n_configs][3][3] lattice vectors as rows, Angstrom */
  const uint8_t* pbc;           /* [n_configs] 1 = periodic in 3D, 0 = free cluster */
} mtp_batch;

/* Outputs of mtp_eval; every pointer is a device pointer or NULL (not wanted). */
typedef struct {
  double* energy;       /* [n_configs] E = sum_i V(n_i), eV (eq. E_MTP) */
  double* forces;       /* [n_atoms][3] F = -dE/dx, eV/Angstrom */
  double* virial;       /* [n_configs][3][3] W_ab = dE/d eps_ab for r -> (I + eps) r, eV;
                           the stress of a periodic cell is W / volume */
  double* site_energy;  /* [n_atoms] V(n_i), eV (eq. V_MTP) */
  double* b;            /* [n_configs][m] b_alpha = sum_i B_alpha(n_i) (eq. matrix-B),
                           in the basis order of the potential file */
} mtp_out;

/* Basic facts about a loaded potential. */
typedef struct {
  int32_t level;        /* lev_max */
  int32_t m;            /* number of basis functions = |xi| */
  int32_t n_mu;         /* number of radial functions f_mu */
  int32_t n_species;
  int32_t n_q;          /* radial basis size N_Q */
  int32_t n_c;          /* |c| = n_mu * n_species^2 * n_q */
  double r_min;         /* Angstrom */
  double r_cut;         /* Angstrom */
  int32_t n_schedules;  /* FP64 schedules of the evaluation kernels (mtp_set_schedule) */
  int32_t reserved;
} mtp_info;

/*
 * Reads a potential (functional form of section 2.1 plus theta = {xi, c})
 * from a text file and prepares it on HIP device `device`.
 * File format: "mtp355 1", then level, species_count, radial_basis_size,
 * min_dist, max_dist, the moment list (mu nu), the connected contractions
 * (vertices as moment indices, edges "u v k"), the basis functions (lists of
 * contraction indices), radial_coeffs c[mu][z_i][z_j][beta] and xi.
 * The basis must be one the library was built for (MTP_E_BASIS otherwise);
 * it is matched up to the order of contractions, functions and vertices.
 * On success *out owns device memory until mtp_free.
 */
int mtp_load(const char* path, int device, mtp_model** out);

/* Fills *info.  Host only, no device work. */
int mtp_model_info(const mtp_model* model, mtp_info* info);

/* Replaces theta = {xi, c} (eqs. V_MTP and f_mu).  Host pointers, file order:
 * c_host [n_mu][S][S][N_Q], xi_host [m].  Either may be NULL (kept).
 * Synchronous (the parameters are in use by the next call on any stream). */
int mtp_set_params(mtp_model* model, const double* c_host, const double* xi_host);

/* Copies theta to host memory (same layouts as mtp_set_params). */
int mtp_get_params(const mtp_model* model, double* c_host, double* xi_host);

/*
 * Energy, forces, virial, site energies and descriptors of every
 * configuration of a batch (section 2.1: eqs. E_MTP, V_MTP, the moments,
 * eqs. f_mu and radial-basis; forces and virial by the adjoint of that
 * chain).  Neighbourhoods hold every atom and periodic image with
 * 0 < |r_ij| < R_cut.  Runs on `stream` (a hipStream_t; NULL = default);
 * it synchronises the stream once to size the neighbour workspace.
 */
int mtp_eval(mtp_model* model, const mtp_batch* batch, const mtp_out* out,
             int precision, void* stream);

/*
 * mtp_eval without any host synchronisation or allocation, for capture into
 * a HIP graph and replay: the workspace (including the neighbour capacity)
 * must have been sized by an earlier mtp_eval on the same batch or a larger
 * one (MTP_E_STATE otherwise).  Conditions the synchronous call would report
 * (invalid offsets or species, more neighbours than the capacity) are only
 * recorded on the device; mtp_status returns them.  Timing is not recorded.
 */
int mtp_eval_async(mtp_model* model, const mtp_batch* batch, const mtp_out* out,
                   int precision, void* stream);

/*
 * Sets the active set of section 2.3: A (device, [m][m] FP64, row j = b of
 * active configuration j, columns in file basis order).  A^{-1} is formed
 * on the device by FP64 Gauss-Jordan elimination with partial pivoting and
 * kept in the model.  Fails with MTP_E_ARG if A is numerically singular
 * (a pivot below 1e-13 once every column is scaled to max |entry| = 1).
 * Synchronises `stream`.
 */
int mtp_set_active_set(mtp_model* model, const double* A_dev, void* stream);

/*
 * Extrapolation grade of section 2.3 for rows b (device, [n][m] FP64, file
 * order): c = b A^{-1}, gamma = max_j |c_j|, argmax = the row of A that the
 * MaxVol step would replace (lowest index on ties).  gamma_dev [n] FP64,
 * argmax_dev [n] int32, c_dev [n][m] FP64 or NULL.
 */
int mtp_grade_from_b(mtp_model* model, int32_t n, const double* b_dev, double* gamma_dev,
                     int32_t* argmax_dev, double* c_dev, void* stream);

/*
 * mtp_grade_from_b without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): the
 * product c = b A^{-1} goes to a fixed device array of the library (16 MiB
 * per GPU, held until the process ends) instead of memory the model would
 * allocate, so n * m must not exceed 2^21 (MTP_E_CAPACITY otherwise, before
 * anything is launched).  gamma_dev [n] FP64 and argmax_dev [n] int32 as in
 * mtp_grade_from_b; c is not returned.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (on different streams, or from
 * different models) race, so order them on one stream.  MTP_E_STATE without
 * an active set.  Asynchronous on `stream`.
 */
int mtp_grade_from_b_noalloc(mtp_model* model, int32_t n, const double* b_dev, double* gamma_dev,
                             int32_t* argmax_dev, void* stream);

/* mtp_eval for b followed by mtp_grade_from_b, per configuration. */
int mtp_grade(mtp_model* model, const mtp_batch* batch, double* gamma_dev, int32_t* argmax_dev,
              int precision, void* stream);

/*
 * Rows of the nonlinear grade of section 2.3: the matrix B generalised from
 * b = dE/dxi to the derivatives of each configuration's energy in all
 * parameters theta = (xi, c), at the current theta.  rows_dev (device,
 * [n_configs][m + n_c] FP64, caller-owned): columns 0..m-1 are b_k (file
 * basis order), columns m.. are dE_k/dc in the layout of c,
 * [n_mu][S][S][N_Q].  Runs the evaluation and the loss-gradient kernels with
 * unit energy weights and no force or stress terms.  precision FP64 or FP32
 * (FP32 kernels, FP64 sums).  MTP_E_ARG for an empty batch; errors of
 * mtp_eval otherwise.  Synchronises `stream` (as mtp_eval does).
 */
int mtp_theta_rows(mtp_model* model, const mtp_batch* batch, int precision, double* rows_dev, void* stream);

/*
 * Active set of the nonlinear grade: A (device, [n_cols][n_cols] FP64, row j =
 * the theta row of active configuration j restricted to n_cols columns that
 * the caller chose, 1 <= n_cols <= m + n_c).  The full rows are never of full
 * rank: scaling c_mu by lambda and every xi_alpha by lambda^-k (k the number
 * of moments of radial function mu in basis function alpha) leaves E
 * unchanged, one linear relation among the columns per mu, so some c columns
 * must be left out.  Inverted and kept like the linear active set
 * (mtp_set_active_set), independently of it.  MTP_E_ARG for n_cols out of
 * range or a numerically singular A.  Synchronises `stream`.
 */
int mtp_set_active_set_theta(mtp_model* model, int32_t n_cols, const double* A_dev, void* stream);

/*
 * Nonlinear grade of section 2.3 for theta rows restricted to the active
 * set's columns (device, [n][n_cols] FP64): c = row A^{-1}, gamma =
 * max_j |c_j|, argmax as in mtp_grade_from_b.  gamma_dev [n] FP64,
 * argmax_dev [n] int32.  MTP_E_STATE without an active set
 * (mtp_set_active_set_theta).
 */
int mtp_grade_theta(mtp_model* model, int32_t n, const double* rows_dev, double* gamma_dev,
                    int32_t* argmax_dev, void* stream);

/*
 * Training loss of section 2.2 (eq. Fitting; weighting `scaling` = molecules,
 * structures (eq. train-structures) or vibrations (eq. train-vibrations)) and
 * its gradient with respect to theta = {xi, c}.  Targets (device, FP64):
 * E_t [n_configs] eV, F_t [n_atoms][3] eV/Angstrom, W_t [n_configs][3][3] the
 * extensive virial stress in eV (volume * stress; ignored for clusters, which
 * have no stress term).  Outputs (device): loss_dev [1]; grad_dev [m + n_c]:
 * dL/dxi in the file's basis order, then dL/dc in the layout
 * c[mu][z_i][z_j][beta].  The gradient is formed by forward-mode tangents of
 * the moments and of the contraction's reverse sweep (directional
 * derivatives along the force and virial residuals).  grad_pos_dev (device,
 * may be NULL): dL/dx [n_atoms][3] in eV/Angstrom, the gradient in the atomic
 * positions at fixed cells: -a_k F_i from the energy term plus the
 * Hessian-vector product of E with the force and stress residuals, formed by
 * the same tangents and a dual-number pass over the pair gradients.
 * precision: MTP_FP64 or MTP_FP32.  Synchronises `stream` once (inside the
 * evaluation).
 */
int mtp_loss_grad(mtp_model* model, const mtp_batch* batch, const double* E_t, const double* F_t,
                  const double* W_t, double w_e, double w_f, double w_s, int scaling, int precision,
                  double* loss_dev, double* grad_dev, double* grad_pos_dev, void* stream);

/*
 * Normal equations of section 2.2, eq. Fitting, in xi at the model's current
 * radial coefficients c.  E, forces and the virial are linear in xi, so the
 * loss of mtp_loss_grad (same targets, weights and scaling) equals
 *   L(xi) = xi^T H xi - 2 g^T xi + yy,
 * H = J^T W J [m][m], g = J^T W y [m], yy = y^T W y, where J holds the
 * energies, forces and virials of every basis function alone (xi = e_alpha)
 * and W the per-row weights of the scaling.  Outputs (device, FP64, file
 * basis order): H_dev row-major [m][m] (exactly symmetric), g_dev [m] or
 * NULL, yy_dev [1] or NULL; with accumulate = 1 the values are added to what
 * the buffers hold (summing over batches of a training set larger than one
 * batch), with 0 they are overwritten.  J is evaluated in `precision`
 * (MTP_FP64 or MTP_FP32) and held in the model's workspace:
 * 8 (m + 1)(10 n_configs + 3 n_atoms) bytes, plus two more sets of the
 * evaluation's per-atom buffers: the columns run on three internal streams
 * forked from and joined back to `stream`, so the outputs are ready in
 * `stream` order.  Synchronises `stream` once.
 */
int mtp_normal_equations(mtp_model* model, const mtp_batch* batch, const double* E_t, const double* F_t,
                         const double* W_t, double w_e, double w_f, double w_s, int scaling, int precision,
                         int accumulate, double* H_dev, double* g_dev, double* yy_dev, void* stream);

/*
 * Minimiser xi_dev [m] (device, FP64, file order) of xi^T H xi - 2 g^T xi for
 * H, g of mtp_normal_equations: H is scaled to unit diagonal and inverted by
 * Gauss-Jordan elimination with partial pivoting in FP64.  Returns MTP_E_ARG
 * (xi_dev untouched in meaning) when the scaled H is numerically singular,
 * e.g. when a basis function vanishes on every configuration of the set.
 * Does not change the model's xi (see mtp_set_params).  Synchronises
 * `stream`.
 */
int mtp_solve_normal(mtp_model* model, const double* H_dev, const double* g_dev, double* xi_dev, void* stream);

/*
 * Schedules of the evaluation kernels.  Level by level the FP64 kernels are
 * compiled in several schedules: different cuts of the per-atom work
 * (moments, reverse sweep, adjoint) into passes that fit the register file,
 * trading recomputation per pair against wavefronts per SIMD.  All compute
 * the same quantities (they differ only in summation order).  FP32 has one
 * schedule; the FP64 part of MTP_MIXED follows the FP64 schedules (with the
 * contraction passes of schedule 0 for the fused ones, as for any evaluation
 * from stored moments).
 *
 * mtp_set_schedule selects one for every evaluation (MTP_E_ARG for an index
 * outside 0 .. schedules - 1).  mtp_autotune builds the lists of `batch`,
 * times each schedule's evaluation kernels `repeats` times with HIP events
 * on `stream` (after one untimed launch), once without and once with the
 * per-atom basis values that descriptor sums b need, keeps the fastest of
 * each kind for `precision` (evaluations that ask for b use the second) and
 * returns the first's index in *chosen (may be NULL); ms_out[k] (k < n_out,
 * may be NULL) receives the best time of schedule k in milliseconds without
 * the basis values, ms_out[schedules + k] with them.  Synchronises
 * `stream`.
 */
int mtp_set_schedule(mtp_model* model, int precision, int schedule);
int mtp_autotune(mtp_model* model, const mtp_batch* batch, int precision, int repeats, float* ms_out, int n_out,
                 int* chosen, void* stream);

/*
 * Device-side counters of the last mtp_eval on this model: pairs closer than
 * R_min (the radial polynomial is then evaluated outside [R_min, R_cut]) and
 * neighbour-list inconsistencies (pairs whose reverse pair was not found;
 * always 0 unless memory was corrupted).  Returns MTP_E_ARG or
 * MTP_E_CAPACITY when the last (asynchronous) evaluation met invalid input
 * or exceeded the neighbour capacity, and MTP_E_STATE when its lists were
 * inconsistent (its forces are then wrong); mtp_eval returns the same codes.
 * Synchronises `stream`.
 */
int mtp_status(mtp_model* model, void* stream, int64_t* n_below_rmin, int64_t* n_list_errors);

/*
 * MaxVol selection of an active set (section 2.3: the step of Goreinov et
 * al. behind the query strategy) from a pool of descriptor rows: pool_dev
 * (device, [n_pool][m] FP64, file basis order, e.g. b of candidate
 * configurations from mtp_eval).  rows_dev (device, [m] int32): with
 * init = 1 it holds the starting rows (distinct pool indices), with
 * init = 0 the library picks them (the pivot rows of Gaussian elimination
 * with partial pivoting of the column-equilibrated pool, ascending).  Then,
 * while the largest |c_ij| of C = pool A^{-1}, A = pool[rows], exceeds
 * 1 + delta (lowest i, then j, on ties) and fewer than max_swaps swaps were
 * made (max_swaps < 0: 100 m), rows[j] becomes i; |det A| grows by |c_ij|
 * each time.  On return rows_dev holds the selection in position order and
 * *n_swaps (host, may be NULL) the number of swaps.  C is updated by rank-one
 * steps and recomputed from A^{-1} every 32 swaps and before stopping.  It
 * synchronises `stream` once per swap; the model's active set is not
 * changed (pass pool[rows] to mtp_set_active_set).  MTP_E_ARG for a pool
 * of fewer than m rows, invalid starting rows or a singular selection.
 */
int mtp_maxvol(mtp_model* model, int32_t n_pool, const double* pool_dev, int32_t* rows_dev, int init,
               double delta, int32_t max_swaps, int32_t* n_swaps, void* stream);

/*
 * mtp_maxvol for the nonlinear grade: the pool holds theta rows (from
 * mtp_theta_rows) restricted to n_cols columns of the caller's choice
 * (device, [n_pool][n_cols] FP64, 1 <= n_cols <= m + n_c), and n_cols rows
 * are selected (rows_dev [n_cols] int32).  Same algorithm, ties, errors and
 * synchronisation as mtp_maxvol; pass pool[rows] to mtp_set_active_set_theta.
 */
int mtp_maxvol_theta(mtp_model* model, int32_t n_cols, int32_t n_pool, const double* pool_dev, int32_t* rows_dev,
                     int init, double delta, int32_t max_swaps, int32_t* n_swaps, void* stream);

/*
 * One half step of velocity Verlet for the molecular dynamics in which the
 * active learning of section 2.3 runs: vel += (dt/2) F / m for every atom
 * and, when drift != 0, then pos += dt vel.  Device arrays: species [n]
 * int32, pos [n][3] and vel [n][3] FP64 (Angstrom, Angstrom/fs, updated in
 * place), forces [n][3] FP64 (eV/A, from mtp_eval); mass_host [S] in atomic
 * mass units; dt in fs.  A step is kick+drift, mtp_eval at the new
 * positions, kick.  Asynchronous on `stream`, except that a call with
 * masses different from the previous call's first synchronises it to copy
 * them to the device.
 */
int mtp_md_kick(mtp_model* model, int64_t n_atoms, const int32_t* species_dev, double* pos_dev, double* vel_dev,
                const double* forces_dev, const double* mass_host, double dt_fs, int drift, void* stream);

/*
 * One step of FIRE relaxation (the relaxations of the active-learning
 * scheme of section 2.3 run to a minimum of the potential; FIRE is the method
 * of Bitzek et al., Phys. Rev. Lett. 97, 170201 (2006)), every configuration
 * of a batch independently: with P = F . v over the configuration, if P >= 0
 * v <- (1 - alpha) v + alpha |v| F/|F| and, after more than n_min such steps
 * in a row, dt <- min(f_inc dt, dt_max), alpha <- f_alpha alpha; if P < 0,
 * v <- 0, dt <- f_dec dt, alpha <- alpha_start.  Then v += dt F / m and
 * pos += dt v.  Device arrays: atom_offsets [n_configs + 1] int64, species
 * [n_atoms] int32, pos and vel [n_atoms][3] FP64 (updated in place), forces
 * [n_atoms][3] FP64 (eV/A, from mtp_eval at pos), state [n_configs][4] FP64
 * (dt in fs, alpha, the count of steps with P >= 0, unused; the caller sets
 * dt0, alpha_start, 0 before the first step).  mass_host [S] amu;
 * params_host = {dt_max, n_min, f_inc, f_dec, alpha_start, f_alpha}.
 * MTP_E_ARG for null arrays or parameters out of range.  Asynchronous on
 * `stream` except for new masses, as mtp_md_kick.
 */
int mtp_fire_step(mtp_model* model, int32_t n_configs, const int64_t* atom_offsets_dev, int64_t n_atoms,
                  const int32_t* species_dev, double* pos_dev, double* vel_dev, const double* forces_dev,
                  const double* mass_host, double* state_dev, const double* params_host, void* stream);

/*
 * Kinetic energy of every configuration for the MD of section 2.3:
 * ekin_dev[k] = sum over its atoms of m |v|^2 / 2 in eV (device [n_configs]
 * FP64), summed in a fixed order.  atom_offsets [n_configs + 1] int64,
 * species [n_atoms] int32, vel [n_atoms][3] FP64 (Angstrom/fs), mass_host [S]
 * amu.  Asynchronous on `stream` except for new masses, as mtp_md_kick.
 */
int mtp_kinetic_energy(mtp_model* model, int32_t n_configs, const int64_t* atom_offsets_dev, int64_t n_atoms,
                       const int32_t* species_dev, const double* vel_dev, const double* mass_host, double* ekin_dev,
                       void* stream);

/* Counters and device timings of the last mtp_eval on a model. */
typedef struct {
  int64_t n_atoms;          /* atoms of the last batch */
  int64_t n_pairs;          /* neighbour pairs (i, j, image) of the last batch */
  int32_t max_neighbours;   /* largest neighbour count of one atom */
  int32_t level;
  double flops_pair_fwd;    /* algorithmic flops per pair of the compiled schedule, N_Q = 8:
                               radial functions, monomials, moment sums */
  double flops_pair_bwd;    /* per pair: adjoint g = dV/dr_ij, virial */
  double flops_atom;        /* per atom: contractions, basis products and their reverse */
  float ms_neighbours;      /* device time of the neighbour search (-1 when timing is off) */
  float ms_eval;            /* evaluation kernels (moments, contractions, adjoint) */
  float ms_forces;          /* force gather */
  float ms_reduce;          /* per-configuration sums: they run on a second stream beside
                               the gather, so this is the time they add after it */
  int32_t lists_reused;     /* 1 if the last mtp_eval refreshed the lists of an earlier call (skin) */
  int32_t list_builds;      /* neighbour-list builds since the skin was last set */
} mtp_stats;

/*
 * Verlet skin for repeated evaluation of one batch whose atoms move a
 * little between calls (MD steps).  With skin > 0 (Angstrom, at most R_cut),
 * mtp_eval builds the neighbour lists out to R_cut + skin and later calls
 * on the same batch arrays (the same device pointers and sizes) reuse them
 * while every atom is within skin / 2 of its position at the build: the
 * pair vectors are then recomputed from the positions, pairs beyond R_cut
 * contributing nothing, and the results are those of a fresh search up to
 * rounding.  Moving more than skin / 2, or a different batch, rebuilds.  The
 * cells, species and pbc flags of a batch must not change in place while its
 * lists are reused (set the skin again to discard them).  The check costs
 * one extra synchronisation per call; mtp_eval_async ignores the skin and
 * always searches.  skin = 0 (the default) searches on every call.
 * MTP_E_ARG outside [0, R_cut].
 */
int mtp_set_skin(mtp_model* model, double skin);

/* Turns HIP-event timing of the phases of mtp_eval on (enable = 1) or off.
 * Events are recorded on the stream of each call. */
int mtp_set_timing(mtp_model* model, int enable);

/* Fills *stats for the last mtp_eval; synchronises that call's stream. */
int mtp_get_stats(mtp_model* model, mtp_stats* stats);

/* Releases the model and its device memory. */
void mtp_free(mtp_model* model);

/* Message of the last failing call on this thread ("" if none). */
const char* mtp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MTP_H */
