// Learned machine-pair selector (filled in below).
#include "internal.h"

namespace pfsp {
void selector_free(Ctx *c) { (void)c; }
int launch_learned(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                   hipStream_t s) {
  (void)pool; (void)ub; (void)out_lb; (void)out_prune; (void)s;
  return set_err(c, PFSP_EINVAL, "no selector loaded");
}
}  // namespace pfsp
