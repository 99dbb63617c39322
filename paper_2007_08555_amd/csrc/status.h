// Device status word of an evaluation and its mapping to a return code.
// Plain C++ (no HIP types), so the mapping can be compiled and tested on a
// host without a GPU.
#pragma once
#include <stdint.h>

#include "mtp.h"

namespace mtp {

// Device counters read by mtp_status and by mtp_eval after its kernels.
struct Status {
  unsigned long long below_rmin;
  unsigned long long list_errors;
  unsigned long long max_count;   // largest neighbour count of the last search
  unsigned long long bad_offsets; // atom_offsets not monotone from 0 to n_atoms
  unsigned long long bad_species; // species index outside [0, n_species)
  unsigned long long n_pairs;     // total neighbour pairs of the last search
  unsigned long long overflow;    // atoms with more neighbours than the ELL capacity
  unsigned long long n_binned;    // atoms of binned configurations (entries of NbrArgs::binned)
  unsigned long long n_large;     // atoms of configurations above the small-search size (NbrArgs::large)
};

// Return code (MTP_OK when the evaluation is usable, else an MTP_E_* value)
// of a finished evaluation's status, and the message for mtp_last_error.
// Invalid input comes first (MTP_E_ARG), then an exceeded neighbour
// capacity (MTP_E_CAPACITY), then neighbour lists that are not symmetric
// (MTP_E_STATE: a pair whose reverse pair was not found, so its force
// contribution is wrong).  Pairs below R_min are not an error.
inline int status_code(const Status& st, const char** msg) {
  const char* m = "";
  int code = MTP_OK;
  if (st.bad_offsets) {
    code = MTP_E_ARG;
    m = "atom_offsets must be non-decreasing from 0 to n_atoms";
  } else if (st.bad_species) {
    code = MTP_E_ARG;
    m = "species index outside [0, species_count)";
  } else if (st.overflow) {
    code = MTP_E_CAPACITY;
    m = "an atom had more neighbours than the neighbour workspace holds";
  } else if (st.list_errors) {
    code = MTP_E_STATE;
    m = "neighbour lists are inconsistent (a pair without its reverse pair): forces would be wrong";
  }
  if (msg) *msg = m;
  return code;
}

}  // namespace mtp
