// C ABI entry points (declared in include/pfsp.h): argument checks, device
// memory ownership and launch plumbing.  Every step of the bounding path runs
// in the HIP kernels of stage.hip, bound.hip, search.hip and selector.hip.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace pfsp {

int set_err(Ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_err(Ctx *c, hipError_t e, const char *what) {
  std::string s = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return set_err(c, PFSP_EDEVICE, s);
}

static void free_instance(Ctx *c) {
  (void)hipFree(c->d_p);
  (void)hipFree(c->d_T);
  (void)hipFree(c->d_ent);
  (void)hipFree(c->d_entq);
  (void)hipFree(c->d_entw);
  (void)hipFree(c->d_pu);
  (void)hipFree(c->d_pv);
  c->d_p = c->d_T = nullptr;
  c->d_ent = nullptr;
  c->d_entq = nullptr;
  c->d_entw = nullptr;
  c->d_pu = c->d_pv = nullptr;
  free(c->p_host);
  c->p_host = nullptr;
  c->n = c->m = c->P = 0;
  (void)hipFree(c->d_static_mask);
  c->d_static_mask = nullptr;
  c->static_words = c->static_pairs = 0;
}

void collect_timings(Ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto &e = c->ktime[p.name];
      e.first += ms;
      e.second += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->pending.clear();
}

}  // namespace pfsp

using namespace pfsp;

extern "C" {

const char *pfsp_last_error(pfsp_ctx *c) {
  if (!c) return "null context";
  return c->impl.err.c_str();
}

int pfsp_create(pfsp_ctx **out, int device, void *hip_stream) {
  if (!out) return PFSP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PFSP_EDEVICE;
  if (device < 0 || device >= ndev) return PFSP_EINVAL;
  pfsp_ctx *h = new (std::nothrow) pfsp_ctx();
  if (!h) return PFSP_ENOMEM;
  Ctx *c = &h->impl;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return PFSP_EDEVICE;
  }
  c->stream = (hipStream_t)hip_stream;
  static bool attrs = false;
  if (!attrs) {
    init_bound_attributes();
    init_selector_attributes();
    attrs = true;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->cu_count = prop.multiProcessorCount;
  if (hipMalloc(&c->d_flag, 16) != hipSuccess || hipMemset(c->d_flag, 0, 16) != hipSuccess) {
    (void)hipFree(c->d_flag);
    delete h;
    return PFSP_ENOMEM;
  }
  if (noalloc_attach(c) != PFSP_OK) {
    (void)hipFree(c->d_flag);
    delete h;
    return PFSP_EDEVICE;
  }
  *out = h;
  return PFSP_OK;
}

void pfsp_destroy(pfsp_ctx *h) {
  if (!h) return;
  Ctx *c = &h->impl;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  search_free(c);
  selector_free(c);
  free_instance(c);
  collect_timings(c);
  (void)hipFree(c->d_costs);
  (void)hipFree(c->d_flag);
  delete h;
}

int pfsp_load_instance(pfsp_ctx *h, int32_t n, int32_t m, const int32_t *p) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (!p) return set_err(c, PFSP_EINVAL, "p is NULL");
  if (n < 2 || n > kMaxN || m < 1 || m > kMaxM)
    return set_err(c, PFSP_ERANGE, "n must be in [2,255] and m in [1,64]");
  int64_t maxp = 0;
  for (int64_t x = 0; x < (int64_t)n * m; ++x) {
    if (p[x] < 0) return set_err(c, PFSP_ERANGE, "negative processing time");
    if (p[x] > maxp) maxp = p[x];
  }
  if ((int64_t)(n + m - 1) * maxp >= (int64_t(1) << 30))
    return set_err(c, PFSP_ERANGE, "(n + m - 1) * max(p) must stay below 2^30");
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  search_free(c);
  free_instance(c);
  c->n = n;
  c->m = m;
  c->P = m * (m - 1) / 2;
  c->maxp = (int)maxp;
  // packed 8-byte pair entries need a, b < 2^16 and lag < 2^24
  c->narrow = maxp < 65536 && (int64_t)(m > 2 ? m - 2 : 0) * maxp < (1 << 24);
  c->l16 = c->narrow && (int64_t)(m > 1 ? m - 1 : 0) * maxp < (1 << 16);
  c->x16 = c->l16 && (int64_t)(n + m) * maxp < (1 << 15);
  c->p_host = (int *)malloc((size_t)n * m * 4);
  if (!c->p_host) return set_err(c, PFSP_ENOMEM, "host allocation failed");
  memcpy(c->p_host, p, (size_t)n * m * 4);
  const size_t P = c->P > 0 ? c->P : 1;
  if (hipMalloc(&c->d_p, (size_t)n * m * 4) != hipSuccess ||
      hipMalloc(&c->d_T, (size_t)m * 4) != hipSuccess ||
      hipMalloc(&c->d_pu, P) != hipSuccess || hipMalloc(&c->d_pv, P) != hipSuccess ||
      (c->narrow ? hipMalloc(&c->d_ent, (size_t)n * P * 8)
                 : hipMalloc(&c->d_entw, (size_t)n * P * 16)) != hipSuccess) {
    free_instance(c);
    return set_err(c, PFSP_ENOMEM, "device allocation failed");
  }
  PFSP_HIP(c, hipMemcpyAsync(c->d_p, p, (size_t)n * m * 4, hipMemcpyHostToDevice, c->stream));
  int rc = stage_instance(c);
  if (rc == PFSP_OK && c->narrow && c->x16 && n > 32 && n <= 128)
    rc = stage_quick(c, c->stream, n, m, c->d_ent, &c->d_entq);
  if (rc) {
    free_instance(c);
    return rc;
  }
  return PFSP_OK;
}

int pfsp_pair_count(pfsp_ctx *h) {
  if (!h) return PFSP_EINVAL;
  if (h->impl.n == 0) return PFSP_ENOINST;
  return h->impl.P;
}

int pfsp_bound_children(pfsp_ctx *h, const pfsp_pool *pool, int lb_kind, int32_t ub,
                        int32_t *out_lb, uint8_t *out_prune) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!pool) return set_err(c, PFSP_EINVAL, "null pool");
  if (pool->count < 0) return set_err(c, PFSP_EINVAL, "negative count");
  if (pool->n != c->n) return set_err(c, PFSP_EINVAL, "pool.n differs from the loaded n");
  if (lb_kind < PFSP_LB1 || lb_kind > PFSP_LB2_LEARNED)
    return set_err(c, PFSP_EINVAL, "unknown lb_kind");
  if (lb_kind != PFSP_LB1 && c->m < 2)
    return set_err(c, PFSP_ERANGE, "LB2 kinds need m >= 2");
  if (pool->count == 0) return PFSP_OK;
  if (!out_lb || !out_prune) return set_err(c, PFSP_EINVAL, "null output");
  if (!pool->perm || !pool->d1 || !pool->d2) return set_err(c, PFSP_EINVAL, "null pool array");
  if (lb_kind == PFSP_LB2_SUBSET &&
      (!pool->pair_mask || pool->mask_words < (c->P + 31) / 32))
    return set_err(c, PFSP_EINVAL, "subset bound needs pair_mask with ceil(P/32) words");
  if (lb_kind == PFSP_LB1 && pool->argpair_out)
    return set_err(c, PFSP_EINVAL, "argpair_out needs an LB2 kind");
  PFSP_HIP(c, hipSetDevice(c->device));
  DevPool dp;
  dp.count = pool->count;
  dp.n = pool->n;
  dp.perm = pool->perm;
  dp.d1 = pool->d1;
  dp.d2 = pool->d2;
  dp.mask = pool->pair_mask;
  dp.mask_words = pool->mask_words;
  dp.dir = pool->dir_out;
  dp.argpair = pool->argpair_out;
  if (lb_kind == PFSP_LB2_LEARNED) {
    return launch_learned(c, dp, ub, out_lb, out_prune, c->stream);
  }
  return launch_bound(c, dp, lb_kind, ub, out_lb, out_prune, c->stream);
}

int pfsp_pair_mask(pfsp_ctx *h, int variant, uint32_t *mask_out, int32_t words) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!mask_out || words < (c->P + 31) / 32)
    return set_err(c, PFSP_EINVAL, "mask_out needs ceil(P/32) words");
  if (variant != PFSP_PAIRS_ADJACENT && variant != PFSP_PAIRS_LAST)
    return set_err(c, PFSP_EINVAL, "unknown pair variant");
  const int m = c->m;
  for (int w = 0; w < words; ++w) mask_out[w] = 0u;
  for (int k = 0; k + 1 < m; ++k) {
    const int u = k, v = variant == PFSP_PAIRS_ADJACENT ? k + 1 : m - 1;
    const int q = u * (2 * m - u - 1) / 2 + (v - u - 1);
    mask_out[q >> 5] |= 1u << (q & 31);
  }
  return PFSP_OK;
}

int pfsp_search_set_pairs(pfsp_ctx *h, const uint32_t *mask, int32_t words) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  const int need = (c->P + 31) / 32;
  if (!mask || words < need) return set_err(c, PFSP_EINVAL, "mask needs ceil(P/32) words");
  std::vector<uint32_t> mk(mask, mask + need);
  if (c->P & 31) mk[need - 1] &= (1u << (c->P & 31)) - 1u;  // bits past the last pair
  int count = 0;
  for (uint32_t w : mk) count += __builtin_popcount(w);
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  if (!c->d_static_mask) {
    if (hipMalloc(&c->d_static_mask, (size_t)need * 4) != hipSuccess) {
      c->d_static_mask = nullptr;
      return set_err(c, PFSP_ENOMEM, "device allocation failed");
    }
  }
  PFSP_HIP(c, hipMemcpy(c->d_static_mask, mk.data(), (size_t)need * 4, hipMemcpyHostToDevice));
  c->static_words = need;
  c->static_pairs = count;
  return PFSP_OK;
}

int pfsp_check(pfsp_ctx *h) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  int flag[4] = {0, 0, 0, 0};
  PFSP_HIP(c, hipMemcpy(flag, c->d_flag, 16, hipMemcpyDeviceToHost));
  if (flag[0]) {
    PFSP_HIP(c, hipMemset(c->d_flag, 0, 16));
    return set_err(c, PFSP_EINVAL, "a pool row had d1 + d2 >= n");
  }
  return PFSP_OK;
}

int pfsp_neh(pfsp_ctx *h, int32_t *perm_out, int32_t *cmax_out) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!perm_out || !cmax_out) return set_err(c, PFSP_EINVAL, "null argument");
  return neh_host(c->n, c->m, c->p_host, perm_out, cmax_out);
}

static int64_t *opt_slot(Ctx *c, const char *key) {
  if (!strcmp(key, "pool_batch")) return &c->pool_batch;
  if (!strcmp(key, "poll_every")) return &c->poll_every;
  if (!strcmp(key, "pool_capacity")) return &c->pool_capacity;
  if (!strcmp(key, "use_graph")) return &c->use_graph;
  if (!strcmp(key, "learned_topk")) return &c->learned_topk;
  if (!strcmp(key, "learned_exact")) return &c->learned_exact;
  if (!strcmp(key, "timing")) return &c->timing;
  if (!strcmp(key, "force_generic")) return &c->force_generic;
  if (!strcmp(key, "lb2_waves")) return &c->lb2_waves;
  if (!strcmp(key, "subset_group")) return &c->subset_group;
  if (!strcmp(key, "search_filter")) return &c->search_filter;
  if (!strcmp(key, "wide_lb2")) return &c->wide_lb2;
  if (!strcmp(key, "lb2_blocks_per_cu")) return &c->lb2_blocks_per_cu;
  if (!strcmp(key, "log_capacity")) return &c->log_capacity;
  if (!strcmp(key, "log_stride")) return &c->log_stride;
  if (!strcmp(key, "deep_r")) return &c->deep_r;
  if (!strcmp(key, "lb1_r")) return &c->lb1_r;
  if (!strcmp(key, "heuristic_threads")) return &c->heuristic_threads;
  if (!strcmp(key, "heuristic_seed")) return &c->heuristic_seed;
  return nullptr;
}

int pfsp_set_option(pfsp_ctx *h, const char *key, int64_t value) {
  if (!h || !key) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  int64_t *s = opt_slot(c, key);
  if (!s) return set_err(c, PFSP_EINVAL, std::string("unknown option ") + key);
  if (!strcmp(key, "pool_batch") && (value < 1 || value > (1 << 24)))
    return set_err(c, PFSP_ERANGE, "pool_batch must be in [1, 2^24]");
  if (!strcmp(key, "poll_every") && (value < 1 || value > 4096))
    return set_err(c, PFSP_ERANGE, "poll_every must be in [1, 4096]");
  if (!strcmp(key, "pool_capacity") && value < 0)
    return set_err(c, PFSP_ERANGE, "pool_capacity must be >= 0");
  if (!strcmp(key, "log_capacity") && (value < 0 || value > (int64_t(1) << 31)))
    return set_err(c, PFSP_ERANGE, "log_capacity must be in [0, 2^31]");
  if (!strcmp(key, "log_stride") && (value < 1 || value > (1 << 24)))
    return set_err(c, PFSP_ERANGE, "log_stride must be in [1, 2^24]");
  if (!strcmp(key, "lb2_blocks_per_cu") && (value < 0 || value > 64))
    return set_err(c, PFSP_ERANGE, "lb2_blocks_per_cu must be in [0, 64]");
  if (!strcmp(key, "subset_group") && value != 0 && value != 1 && value != 2 && value != 4)
    return set_err(c, PFSP_ERANGE, "subset_group must be 0, 1, 2 or 4");
  if (!strcmp(key, "heuristic_threads") && (value < 0 || value > 256))
    return set_err(c, PFSP_ERANGE, "heuristic_threads must be in [0, 256]");
  if (!strcmp(key, "deep_r") && (value < 0 || value > 16))
    return set_err(c, PFSP_ERANGE, "deep_r must be in [0, 16]");
  if (!strcmp(key, "lb1_r") && (value < 0 || value > 255))
    return set_err(c, PFSP_ERANGE, "lb1_r must be in [0, 255]");
  if (!strcmp(key, "lb2_waves") && (value < 0 || value > 16))
    return set_err(c, PFSP_ERANGE, "lb2_waves must be in [0, 16]");
  if (!strcmp(key, "learned_topk") && (value < 1 || value > 2016))
    return set_err(c, PFSP_ERANGE, "learned_topk must be in [1, 2016]");
  if ((!strcmp(key, "use_graph") || !strcmp(key, "learned_exact") || !strcmp(key, "timing") ||
       !strcmp(key, "search_filter") || !strcmp(key, "wide_lb2") ||
       !strcmp(key, "force_generic")) &&
      value != 0 && value != 1)
    return set_err(c, PFSP_EINVAL, "flag options take 0 or 1");
  if (!strcmp(key, "pool_batch") || !strcmp(key, "pool_capacity") ||
      !strcmp(key, "log_capacity"))
    search_free(c);
  *s = value;
  return PFSP_OK;
}

int pfsp_get_option(pfsp_ctx *h, const char *key, int64_t *value) {
  if (!h || !key || !value) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  int64_t *s = opt_slot(c, key);
  if (!s) return set_err(c, PFSP_EINVAL, std::string("unknown option ") + key);
  *value = *s;
  return PFSP_OK;
}

int pfsp_autotune(pfsp_ctx *h, const pfsp_pool *pool, int lb_kind, int32_t ub, int32_t *out_lb,
                  uint8_t *out_prune, int32_t reps, char *report, int32_t report_len) {
  if (!h || !pool) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (lb_kind != PFSP_LB2_FULL && lb_kind != PFSP_LB2_SUBSET && lb_kind != PFSP_LB2_LEARNED)
    return set_err(c, PFSP_EINVAL, "the autotuner shapes the LB2 kernels");
  if (reps < 1) reps = 3;
  PFSP_HIP(c, hipSetDevice(c->device));
  const int64_t save_w = c->lb2_waves, save_g = c->lb2_blocks_per_cu, save_t = c->timing;
  c->timing = 0;
  hipEvent_t e0, e1;
  PFSP_HIP(c, hipEventCreate(&e0));
  PFSP_HIP(c, hipEventCreate(&e1));
  struct Cand {
    int w, g;
    double ms;
  };
  std::vector<Cand> res;
  int rc = PFSP_OK;
  for (int w : {0, 1, 2, 3, 4, 6, 8, 12, 16})
    for (int g : {0, 2, 4, 8, 16, 32}) {
      c->lb2_waves = w;
      c->lb2_blocks_per_cu = g;
      rc = pfsp_bound_children(h, pool, lb_kind, ub, out_lb, out_prune);  // warm-up
      if (rc) break;
      std::vector<double> ts;
      for (int r = 0; r < reps && rc == PFSP_OK; ++r) {
        if (hipEventRecord(e0, c->stream) != hipSuccess) rc = PFSP_EDEVICE;
        if (!rc) rc = pfsp_bound_children(h, pool, lb_kind, ub, out_lb, out_prune);
        if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = PFSP_EDEVICE;
        float ms = 0.f;
        if (!rc && (hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = PFSP_EDEVICE;
        ts.push_back(ms);
      }
      if (rc) break;
      std::sort(ts.begin(), ts.end());
      res.push_back({w, g, ts[ts.size() / 2]});
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = save_t;
  if (rc || res.empty()) {
    c->lb2_waves = save_w;
    c->lb2_blocks_per_cu = save_g;
    return rc ? rc : set_err(c, PFSP_EINVAL, "no candidate ran");
  }
  Cand best = res[0];
  double dflt = -1;
  for (const Cand &x : res) {
    if (x.ms < best.ms) best = x;
    if (x.w == 0 && x.g == 0) dflt = x.ms;
  }
  c->lb2_waves = best.w;
  c->lb2_blocks_per_cu = best.g;
  if (report && report_len > 0) {
    std::string js = "{\"best\": {\"lb2_waves\": " + std::to_string(best.w) +
                     ", \"lb2_blocks_per_cu\": " + std::to_string(best.g) +
                     ", \"ms\": " + std::to_string(best.ms) + "}, \"default_ms\": " +
                     std::to_string(dflt) + ", \"candidates\": " + std::to_string(res.size()) +
                     "}";
    snprintf(report, (size_t)report_len, "%s", js.c_str());
  }
  return PFSP_OK;
}

int pfsp_kernel_time(pfsp_ctx *h, const char *kernel, double *total_ms, int64_t *launches,
                     int reset) {
  if (!h || !kernel || !total_ms || !launches) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  collect_timings(c);
  auto it = c->ktime.find(kernel);
  *total_ms = it == c->ktime.end() ? 0.0 : it->second.first;
  *launches = it == c->ktime.end() ? 0 : it->second.second;
  if (reset) c->ktime.clear();
  return PFSP_OK;
}

}  // extern "C"
