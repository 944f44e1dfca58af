// Batched execution of independent jobs (include/lsr.h, lsr_batch_*).
#include "../../include/lsr.h"

extern "C" {

lsr_status lsr_batch_create(lsr_job* const*, int32_t, const double*, const int32_t*, lsr_batch**) {
  return LSR_E_UNSUPPORTED;
}
lsr_status lsr_batch_step(lsr_batch*, int32_t) { return LSR_E_UNSUPPORTED; }
lsr_status lsr_batch_destroy(lsr_batch*) { return LSR_E_UNSUPPORTED; }

}  // extern "C"
