// Batched solves: placeholder until the persistent kernel lands.
#include "gabp_internal.h"

namespace gabp {

gabp_status batched_create(Ctx* c, int32_t, const int32_t*) {
  return fail(c, GABP_E_ARG, "batched solves are not built yet");
}

gabp_status batched_solve(Ctx* c, const int32_t*, const int64_t*, const double*, double*, double, int32_t,
                          gabp_info*) {
  return fail(c, GABP_E_ARG, "batched solves are not built yet");
}

void batched_destroy(Ctx*) {}

}  // namespace gabp
