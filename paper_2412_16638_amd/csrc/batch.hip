// batch.hip -- batched form of include/mprk.h (many independent problems per launch).
#include <hip/hip_runtime.h>

#include "../../include/mprk.h"
#include "runtime_internal.hpp"

using namespace mprk;

extern "C" int32_t mprk_batch_create(int32_t, const mprk_problem*, const mprk_tableau*,
                                     const mprk_precisions*, void*, mprk_batch** out) {
  if (out) *out = nullptr;
  return set_error(MPRK_EUNSUPPORTED, "batched form not built yet");
}
extern "C" int64_t mprk_batch_workspace_bytes(const mprk_batch*) {
  return set_error(MPRK_EUNSUPPORTED, "batched form not built yet");
}
extern "C" int32_t mprk_batch_bind(mprk_batch*, double* const*, void*, int64_t) {
  return set_error(MPRK_EUNSUPPORTED, "batched form not built yet");
}
extern "C" int32_t mprk_batch_step(mprk_batch*, int32_t) {
  return set_error(MPRK_EUNSUPPORTED, "batched form not built yet");
}
extern "C" int32_t mprk_batch_stats_sync(mprk_batch*, int32_t, mprk_stats*) {
  return set_error(MPRK_EUNSUPPORTED, "batched form not built yet");
}
extern "C" void mprk_batch_destroy(mprk_batch*) {}
