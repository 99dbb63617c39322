// A basis compiled into the library: its structure (for matching a potential
// file) and the launcher of its evaluation kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace mtp {

// Flags of launch_eval: also write every B_alpha; keep the moments already in
// args.M (or args.M32; same pairs and radial coefficients) instead of
// recomputing them; leave the moments in args.M (schedules that keep them in
// registers skip that store otherwise) for a later reuse or for the loss
// kernels; compute the moments only (the first half of the mixed-precision
// path); with kEvalNuMask, bits kEvalNuShift.. of the flags mark the moment
// degrees nu whose dV/dM can be nonzero (the rest is known to be zero, as for
// xi = e_alpha in the normal equations): adjoint passes past the last one
// holding such a degree, and reverse passes feeding none of those that run,
// are skipped.
enum : unsigned {
  kEvalWantB = 1u,
  kEvalReuseMoments = 2u,
  kEvalStoreMoments = 4u,
  kEvalMomentsOnly = 8u,
  kEvalNuMask = 16u,
  kEvalNuShift = 8u
};

struct BasisVariant {
  const char* name;
  int level;
  int n_moments;
  const int* moments;            // [n_moments][2] = (mu, nu)
  int n_graphs;
  const int* graph_key_offsets;  // [n_graphs + 1]
  const int* graph_keys;         // canonical keys, concatenated
  int m;                         // basis size
  const int* func_offsets;       // [m + 1]
  const int* func_factors;       // contraction indices, concatenated
  int C;                         // moment components held per atom
  int n_mu;
  int nu_max;
  double flops_pair_fwd;         // algorithmic flops per pair (N_Q = 8), forward
  double flops_pair_bwd;         // per pair, adjoint
  double flops_atom;             // per atom, contraction forward + reverse
  // precision: 0 = FP64, 1 = FP32, 2 = FP32 with compensated moment sums,
  // 3 = FP32 moments from the FP64 pair records (args.pr64), with
  // kEvalMomentsOnly: the first half of the mixed-precision path
  // schedule: index of the FP64 pass split (0 .. n_schedules - 1; FP32 has only 0)
  hipError_t (*launch_eval)(int precision, unsigned flags, int schedule, const void* args, hipStream_t stream);
  // loss-gradient kernels after an evaluation that left M and G in place
  hipError_t (*launch_loss)(int precision, const void* eval_args, const void* loss_args, hipStream_t stream);
  int block;                     // atoms per workgroup of the per-atom kernels
  int n_schedules;               // FP64 schedules compiled (pass splits)
  int partial_rows;              // table-driven bases: rows per atom of args.Gpart for the
                                 // wavefront-split contraction (0: none)
};

extern const BasisVariant* const kVariants[];
extern const int kNumVariants;

}  // namespace mtp
