// Batched circuits and the entangling-gate decomposition driver (Section 4).
#include "juqcs_internal.hpp"

using namespace juqcs;

struct juqcs_batch {
  int dummy;
};

extern "C" {

juqcs_status juqcs_batch_create(juqcs_batch** out, int, const int*, const juqcs_gate*,
                                const int64_t*, void*, const uint64_t*, const juqcs_plan_opts*) {
  if (out) *out = nullptr;
  set_error("batch execution not built yet");
  return JUQCS_ERR_UNSUPPORTED;
}

juqcs_status juqcs_batch_run(juqcs_batch*, void*) {
  set_error("batch execution not built yet");
  return JUQCS_ERR_UNSUPPORTED;
}

juqcs_status juqcs_batch_stats(const juqcs_batch*, int64_t*, int64_t*, int64_t*) {
  set_error("batch execution not built yet");
  return JUQCS_ERR_UNSUPPORTED;
}

juqcs_status juqcs_batch_destroy(juqcs_batch* b) {
  delete b;
  return JUQCS_OK;
}

juqcs_status juqcs_branch_amplitudes(int, const juqcs_gate*, size_t, const uint8_t*,
                                     const uint64_t*, size_t, int, double*, void*) {
  set_error("branch decomposition not built yet");
  return JUQCS_ERR_UNSUPPORTED;
}

}  // extern "C"
