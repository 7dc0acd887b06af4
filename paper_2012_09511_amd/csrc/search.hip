// Device depth-first search (filled in below).
#include "internal.h"

namespace pfsp {
void search_free(Ctx *c) { (void)c; }
}  // namespace pfsp

extern "C" int pfsp_search(pfsp_ctx *h, int32_t ub0, int64_t budget_nodes, int lb_kind,
                           pfsp_result *res) {
  (void)ub0; (void)budget_nodes; (void)lb_kind; (void)res;
  if (!h) return PFSP_EINVAL;
  return pfsp::set_err(&h->impl, PFSP_EINVAL, "search not available yet");
}
