// Bounding without allocation: pfsp_bound_children_noalloc.
//
// The LB2 kinds stage each parent's front, back and remaining loads (3m int32
// per parent) in a workspace between the costs kernel and the bound kernel.
// pfsp_bound_children grows that workspace with hipMalloc on demand; this
// entry point takes it from a fixed device array instead, for callers that
// must not allocate (HIP graph capture, serving loops).  Each GPU holds its
// own copy of the array from the moment the library's code is loaded on it
// until the process ends; its device address is looked up once per device
// when a context is created there.
#include <mutex>

#include "internal.h"

namespace pfsp {

namespace {

constexpr size_t kScratchInts = size_t(16) << 20;  // 64 MiB per GPU

static __device__ __align__(256) int scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Called by pfsp_create with c->device current: the device address of this
// device's copy of the scratch array (never the host-side symbol itself).
int noalloc_attach(Ctx *c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return set_err(c, PFSP_ERANGE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[c->device]) {
    int *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_err(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[c->device] = ptr;
  }
  c->scratch = g_scratch_ptr[c->device];
  return PFSP_OK;
}

size_t noalloc_scratch_ints() { return kScratchInts; }

}  // namespace pfsp

using namespace pfsp;

extern "C" int pfsp_bound_children_noalloc(pfsp_ctx *h, const pfsp_pool *pool, int lb_kind,
                                           int32_t ub, int32_t *out_lb, uint8_t *out_prune) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!pool) return set_err(c, PFSP_EINVAL, "null pool");
  if (lb_kind != PFSP_LB1 && lb_kind != PFSP_LB2_FULL && lb_kind != PFSP_LB2_SUBSET)
    return set_err(c, PFSP_EINVAL,
                   "pfsp_bound_children_noalloc takes PFSP_LB1, PFSP_LB2_FULL or PFSP_LB2_SUBSET");
  if (pool->count < 0) return set_err(c, PFSP_EINVAL, "negative count");
  if (workspace_ints(c, pool->count) > kScratchInts)
    return set_err(c, PFSP_ERANGE,
                   "pool too large for the fixed workspace: count * 3m must be <= " +
                       std::to_string(kScratchInts));
  if (!c->scratch) return set_err(c, PFSP_EDEVICE, "scratch address not set up");
  // The shared bound path with the workspace pointed at this device's
  // scratch array (its capacity covers the pool, so nothing is allocated) and
  // without event timing (events are created per launch).
  int *const costs = c->d_costs;
  const size_t cap = c->costs_cap;
  const int64_t timing = c->timing;
  c->d_costs = c->scratch;
  c->costs_cap = kScratchInts;
  c->timing = 0;
  const int rc = pfsp_bound_children(h, pool, lb_kind, ub, out_lb, out_prune);
  c->d_costs = costs;
  c->costs_cap = cap;
  c->timing = timing;
  return rc;
}
