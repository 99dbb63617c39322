// Host-only check of the mapping from the device status word to the return
// codes of mtp_eval and mtp_status.
#include <cstdio>
#include <cstring>

#include "status.h"

static int failures = 0;

static void expect(const char* what, const mtp::Status& st, int code, const char* needle) {
  const char* msg = nullptr;
  const int got = mtp::status_code(st, &msg);
  if (got != code || !msg || (needle && !std::strstr(msg, needle))) {
    std::printf("FAIL %s: code %d (want %d), message '%s'\n", what, got, code, msg ? msg : "(null)");
    ++failures;
  }
}

int main() {
  mtp::Status st{};
  expect("clean", st, MTP_OK, "");
  st.below_rmin = 5;  // pairs below R_min are reported, not an error
  st.n_pairs = 100;
  expect("below rmin", st, MTP_OK, "");
  st.list_errors = 1;
  expect("list errors", st, MTP_E_STATE, "reverse pair");
  st.overflow = 3;
  expect("overflow before list errors", st, MTP_E_CAPACITY, "neighbours");
  st.bad_species = 1;
  expect("bad species first", st, MTP_E_ARG, "species");
  st.bad_offsets = 1;
  expect("bad offsets first", st, MTP_E_ARG, "atom_offsets");
  mtp::Status only{};
  only.list_errors = 7;
  expect("list errors alone", only, MTP_E_STATE, "forces would be wrong");
  if (failures == 0) std::printf("status mapping ok\n");
  return failures == 0 ? 0 : 1;
}
