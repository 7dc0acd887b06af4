// Batched bounding of several instances of different (n, m) in one launch
// sequence, and the autotuner that picks its tile and block shapes.
//
// Parents of all instances sit in one pool (rows of a common stride, grouped
// by instance).  One k_lb1m launch computes every parent's front, back and
// remaining work (or, for LB1, the whole decomposition); then one persistent
// k_lb2m launch per instance class (n <= 20, n <= 64, packed pair entries)
// drains a device queue of (instance, parent range) tiles, restaging its LDS
// tables only when the instance changes; instances outside those classes use
// the generic kernels.  The whole sequence is captured once as a HIP graph and
// replayed while the buffers and the grouping stay the same.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "internal.h"

namespace pfsp {

// LDS budget of the persistent multi-instance kernels (160 KiB minus their
// few bytes of static LDS)
constexpr size_t kLdsM = 160 * 1024 - 64;

struct MultiInst {
  int n = 0, m = 0, P = 0, narrow = 1, l16 = 1, x16 = 1;
  int cls = -1;  // 0 quick (n <= 20), 1 scan (n <= 64), 2, 3 wide (n <= 64, 128), -1 generic
  int *d_p = nullptr, *d_T = nullptr;
  uint2 *d_ent = nullptr, *d_entq = nullptr;
  uint4 *d_entw = nullptr;
  uint8_t *d_pu = nullptr, *d_pv = nullptr;
  DevInst view() const {
    DevInst I;
    I.n = n; I.m = m; I.P = P; I.narrow = narrow; I.l16 = l16; I.x16 = x16;
    I.p = d_p; I.T = d_T; I.ent = d_ent; I.entw = d_entw; I.pu = d_pu; I.pv = d_pv;
    I.entq = d_entq;
    return I;
  }
};

struct MultiKey {
  int kind = 0;
  const void *perm = nullptr, *d1 = nullptr, *d2 = nullptr, *lb = nullptr, *pr = nullptr,
             *dir = nullptr;
  int stride = 0;
  std::vector<long long> seg;
  int tile = 0, waves0 = 0, waves1 = 0, gridk = 0;
  bool operator==(const MultiKey &o) const {
    return kind == o.kind && perm == o.perm && d1 == o.d1 && d2 == o.d2 && lb == o.lb &&
           pr == o.pr && dir == o.dir && stride == o.stride && seg == o.seg && tile == o.tile &&
           waves0 == o.waves0 && waves1 == o.waves1 && gridk == o.gridk;
  }
};

}  // namespace pfsp

struct pfsp_multi {
  pfsp::Ctx *c = nullptr;
  std::vector<pfsp::MultiInst> in;
  pfsp::DevInst *d_insts = nullptr;
  int nmax = 0, mmax = 0;
  hipStream_t stream = nullptr;
  // shape (0 = automatic)
  int tile = 256, waves[2] = {0, 0}, grid_per_cu = 0;
  // buffers
  long long *d_seg = nullptr;
  int *d_ubs = nullptr;
  int *d_costs = nullptr;
  size_t costs_cap = 0;
  pfsp::MultiTile *d_tiles = nullptr;
  size_t tiles_cap = 0;
  int first[5] = {0, 0, 0, 0, 0};  // tile ranges of the four fast classes
  int *d_queue = nullptr;  // [4] tile counters
  // graph cache
  pfsp::MultiKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace pfsp {

static void multi_drop_graph(pfsp_multi *mt) {
  if (mt->gexec) (void)hipGraphExecDestroy(mt->gexec);
  if (mt->graph) (void)hipGraphDestroy(mt->graph);
  mt->gexec = nullptr;
  mt->graph = nullptr;
  mt->key = MultiKey();
}

static int class_of(const MultiInst &x, const Ctx *c) {
  if (!x.narrow || c->force_generic) return -1;
  if (x.n <= 20 && x.l16) return 0;
  if (x.d_entq && x.n <= 64) return 2;
  if (x.d_entq && x.n <= 128) return 3;
  if (x.n <= 64) return 1;
  return -1;
}

constexpr int kNumCls = 4;
static const int kClassNmax[kNumCls] = {20, 64, 64, 128};
static const int kClassWide[kNumCls] = {0, 0, 1, 1};

// waves per block that the class kernel's launch bounds allow (the quick
// class with 16-bit X: four per SIMD)
static int max_waves(int cls, int x16) {
  static const int w[kNumCls] = {12, 8, 8, 4};
  return cls == 0 && x16 ? 16 : w[cls];
}

// Class layout: the largest padded pair count, job count and machine count
// of the instances of the class, and whether all of them allow 16-bit X.
static void class_layout(const pfsp_multi *mt, int cls, int &ppad, int &nj, int &mm, int &x16) {
  ppad = 64;
  nj = 1;
  mm = 1;
  x16 = 1;
  for (const MultiInst &x : mt->in)
    if (x.cls == cls) {
      ppad = std::max(ppad, (x.P + 63) / 64 * 64);
      nj = std::max(nj, x.n);
      mm = std::max(mm, x.m);
      x16 = x16 && x.x16;
    }
}

static int auto_waves(int cls, int ppad, int nj, int mm, int x16) {
  int waves = 1, best = 0;
  for (int w = max_waves(cls, x16); w >= 1; --w) {
    const size_t l = lb2m_lds_bytes(kClassNmax[cls], ppad, nj, mm, w, x16, kClassWide[cls]);
    const int per_cu = l <= kLdsM ? (int)((kLdsM) / l) * w : 0;
    if (per_cu > best) {
      best = per_cu;
      waves = w;
    }
  }
  return waves;
}

// Tiles of the fast classes, grouped by instance, uploaded synchronously
// (never inside a graph capture).
static int multi_tiles(pfsp_multi *mt, const std::vector<long long> &seg) {
  Ctx *c = mt->c;
  const int K = (int)mt->in.size();
  std::vector<MultiTile> tiles;
  for (int cls = 0; cls < kNumCls; ++cls) {
    mt->first[cls] = (int)tiles.size();
    for (int k = 0; k < K; ++k) {
      if (mt->in[k].cls != cls) continue;
      for (long long b = seg[k]; b < seg[k + 1]; b += mt->tile) {
        MultiTile t;
        t.inst = k;
        t.begin = (int)b;
        t.end = (int)std::min<long long>(b + mt->tile, seg[k + 1]);
        t.pad = 0;
        tiles.push_back(t);
      }
    }
  }
  mt->first[kNumCls] = (int)tiles.size();
  PFSP_HIP(c, hipStreamSynchronize(mt->stream));
  if (tiles.size() > mt->tiles_cap) {
    multi_drop_graph(mt);
    (void)hipFree(mt->d_tiles);
    mt->d_tiles = nullptr;
    mt->tiles_cap = 0;
    if (hipMalloc(&mt->d_tiles, tiles.size() * sizeof(MultiTile)) != hipSuccess)
      return set_err(c, PFSP_ENOMEM, "tile list allocation failed");
    mt->tiles_cap = tiles.size();
  }
  if (!tiles.empty())
    PFSP_HIP(c, hipMemcpy(mt->d_tiles, tiles.data(), tiles.size() * sizeof(MultiTile),
                          hipMemcpyHostToDevice));
  return PFSP_OK;
}

static int multi_enqueue(pfsp_multi *mt, int kind, const uint8_t *perm, const uint8_t *d1,
                         const uint8_t *d2, int stride, const std::vector<long long> &seg,
                         int *out_lb, uint8_t *out_prune, uint8_t *dir) {
  Ctx *c = mt->c;
  hipStream_t s = mt->stream;
  const int K = (int)mt->in.size();
  const long long total = seg[K];
  int rc = launch_lb1m(c, mt->d_insts, mt->d_seg, K, total, perm, d1, d2, stride, mt->nmax,
                       mt->mmax,
                       mt->d_ubs, out_lb, out_prune, dir, mt->d_costs, kind == PFSP_LB1, s);
  if (rc || kind == PFSP_LB1) return rc;
  for (int cls = 0; cls < kNumCls; ++cls) {
    if (mt->first[cls + 1] == mt->first[cls]) continue;
    FastClassLaunch L;
    L.nmax = kClassNmax[cls];
    L.wide = kClassWide[cls];
    class_layout(mt, cls, L.ppad, L.nmax_jobs, L.mmax, L.x16);
    L.tiles = mt->d_tiles + mt->first[cls];
    L.ntiles = mt->first[cls + 1] - mt->first[cls];
    L.queue = mt->d_queue + cls;
    L.cstride = 3 * mt->mmax;  // k_lb1m's row stride, not the class's
    const int pref = mt->waves[cls == 0 ? 0 : 1];  // small: the quick class; large: the rest
    L.waves = pref > 0 ? std::min(pref, max_waves(cls, L.x16))
                       : auto_waves(cls, L.ppad, L.nmax_jobs, L.mmax, L.x16);
    while (L.waves > 1 && lb2m_lds_bytes(L.nmax, L.ppad, L.nmax_jobs, L.mmax, L.waves, L.x16,
                                         L.wide) > kLdsM)
      --L.waves;
    const size_t lds =
        lb2m_lds_bytes(L.nmax, L.ppad, L.nmax_jobs, L.mmax, L.waves, L.x16, L.wide);
    const int per_cu = std::max(1, (int)((kLdsM) / std::max<size_t>(lds, 1)));
    const int gpc = mt->grid_per_cu > 0 ? mt->grid_per_cu : per_cu;
    L.grid = std::max(1, std::min(L.ntiles, c->cu_count * gpc));
    rc = launch_lb2m(c, L, mt->d_insts, perm, d1, d2, stride, mt->d_ubs, mt->d_costs, out_lb,
                     out_prune, dir, s);
    if (rc) return rc;
  }
  // instances outside the fast classes
  for (int k = 0; k < K; ++k) {
    if (mt->in[k].cls >= 0 || seg[k + 1] == seg[k]) continue;
    DevPool pool;
    pool.count = (int)(seg[k + 1] - seg[k]);
    pool.n = stride;
    pool.perm = perm + (size_t)seg[k] * stride;
    pool.d1 = d1 + seg[k];
    pool.d2 = d2 + seg[k];
    pool.mask = nullptr;
    pool.mask_words = 0;
    pool.dir = dir + seg[k];
    pool.argpair = nullptr;
    pool.ub_dev = mt->d_ubs + k;
    rc = launch_generic_instance(c, mt->in[k].view(), pool, 0,
                                 mt->d_costs + (size_t)seg[k] * 3 * mt->mmax,
                                 out_lb + (size_t)seg[k] * 2 * stride,
                                 out_prune + (size_t)seg[k] * 2 * stride, s);
    if (rc) return rc;
  }
  return PFSP_OK;
}

static int multi_check_args(pfsp_multi *mt, int kind, const uint8_t *perm, const uint8_t *d1,
                            const uint8_t *d2, int stride, const int64_t *seg_begin,
                            const int32_t *ub, int32_t *out_lb, uint8_t *out_prune,
                            uint8_t *dir, std::vector<long long> &seg) {
  Ctx *c = mt->c;
  const int K = (int)mt->in.size();
  if (kind != PFSP_LB1 && kind != PFSP_LB2_FULL)
    return set_err(c, PFSP_EINVAL, "multi-instance bounds support PFSP_LB1 and PFSP_LB2_FULL");
  if (!seg_begin || !ub) return set_err(c, PFSP_EINVAL, "null segment or incumbent array");
  seg.assign(seg_begin, seg_begin + K + 1);
  if (seg[0] != 0) return set_err(c, PFSP_EINVAL, "seg_begin[0] must be 0");
  for (int k = 0; k < K; ++k) {
    if (seg[k + 1] < seg[k]) return set_err(c, PFSP_EINVAL, "seg_begin must not decrease");
    if (seg[k + 1] > seg[k] && mt->in[k].n > stride)
      return set_err(c, PFSP_EINVAL, "stride is smaller than an instance's n");
  }
  if (seg[K] > 0x7fffffffLL) return set_err(c, PFSP_ERANGE, "too many parents");
  if (kind != PFSP_LB1)
    for (int k = 0; k < K; ++k)
      if (seg[k + 1] > seg[k] && mt->in[k].m < 2)
        return set_err(c, PFSP_ERANGE, "LB2 needs m >= 2");
  if (seg[K] > 0 && (!perm || !d1 || !d2 || !out_lb || !out_prune || !dir))
    return set_err(c, PFSP_EINVAL, "null pool or output");
  if (stride < 2 || stride > kMaxN) return set_err(c, PFSP_ERANGE, "stride out of range");
  return PFSP_OK;
}

static int multi_run(pfsp_multi *mt, int kind, const uint8_t *perm, const uint8_t *d1,
                     const uint8_t *d2, int stride, const std::vector<long long> &seg,
                     const int32_t *ub, int32_t *out_lb, uint8_t *out_prune, uint8_t *dir) {
  Ctx *c = mt->c;
  const int K = (int)mt->in.size();
  const long long total = seg[K];
  // buffers
  const size_t need = (size_t)(total > 0 ? total : 1) * 3 * mt->mmax;
  if (need > mt->costs_cap) {
    PFSP_HIP(c, hipStreamSynchronize(mt->stream));
    multi_drop_graph(mt);
    (void)hipFree(mt->d_costs);
    mt->d_costs = nullptr;
    mt->costs_cap = 0;
    if (hipMalloc(&mt->d_costs, need * 4) != hipSuccess)
      return set_err(c, PFSP_ENOMEM, "multi-instance workspace allocation failed");
    mt->costs_cap = need;
  }
  PFSP_HIP(c, hipMemcpyAsync(mt->d_seg, seg.data(), (K + 1) * sizeof(long long),
                             hipMemcpyHostToDevice, mt->stream));
  PFSP_HIP(c, hipMemcpyAsync(mt->d_ubs, ub, K * sizeof(int), hipMemcpyHostToDevice, mt->stream));
  PFSP_HIP(c, hipStreamSynchronize(mt->stream));  // host sources may be temporaries
  if (total == 0) return PFSP_OK;
  MultiKey key;
  key.kind = kind;
  key.perm = perm; key.d1 = d1; key.d2 = d2;
  key.lb = out_lb; key.pr = out_prune; key.dir = dir;
  key.stride = stride;
  key.seg = seg;
  key.tile = mt->tile; key.waves0 = mt->waves[0]; key.waves1 = mt->waves[1];
  key.gridk = mt->grid_per_cu;
  if (!c->use_graph || c->timing) {
    multi_drop_graph(mt);
    int rc = multi_tiles(mt, seg);
    if (rc) return rc;
    return multi_enqueue(mt, kind, perm, d1, d2, stride, seg, out_lb, out_prune, dir);
  }
  if (!(mt->gexec && mt->key == key)) {
    multi_drop_graph(mt);
    int rt = multi_tiles(mt, seg);
    if (rt) return rt;
    PFSP_HIP(c, hipStreamBeginCapture(mt->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = 1;
    int rc = multi_enqueue(mt, kind, perm, d1, d2, stride, seg, out_lb, out_prune, dir);
    c->capturing = 0;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(mt->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_err(c, e, "hipStreamEndCapture");
    mt->graph = g;
    PFSP_HIP(c, hipGraphInstantiate(&mt->gexec, g, nullptr, nullptr, 0));
    mt->key = key;
  }
  PFSP_HIP(c, hipGraphLaunch(mt->gexec, mt->stream));
  return PFSP_OK;
}

}  // namespace pfsp

using namespace pfsp;

extern "C" {

int pfsp_multi_create(pfsp_ctx *h, int32_t count, const int32_t *n, const int32_t *m,
                      const int32_t *const *p, pfsp_multi **out) {
  if (!h || !out) return PFSP_EINVAL;
  *out = nullptr;
  Ctx *c = &h->impl;
  if (count < 1 || count > 65535 || !n || !m || !p)
    return set_err(c, PFSP_EINVAL, "count must be in [1, 65535] with n, m, p arrays");
  PFSP_HIP(c, hipSetDevice(c->device));
  pfsp_multi *mt = new (std::nothrow) pfsp_multi();
  if (!mt) return set_err(c, PFSP_ENOMEM, "host allocation failed");
  mt->c = c;
  mt->in.resize(count);
  int rc = PFSP_OK;
  if (hipStreamCreateWithFlags(&mt->stream, hipStreamNonBlocking) != hipSuccess)
    rc = set_err(c, PFSP_EDEVICE, "stream creation failed");
  for (int k = 0; k < count && rc == PFSP_OK; ++k) {
    MultiInst &x = mt->in[k];
    if (n[k] < 2 || n[k] > kMaxN || m[k] < 1 || m[k] > kMaxM || !p[k]) {
      rc = set_err(c, PFSP_ERANGE, "instance n must be in [2,255] and m in [1,64]");
      break;
    }
    int64_t maxp = 0;
    for (int64_t t = 0; t < (int64_t)n[k] * m[k]; ++t) {
      if (p[k][t] < 0) rc = set_err(c, PFSP_ERANGE, "negative processing time");
      maxp = std::max<int64_t>(maxp, p[k][t]);
    }
    if (rc) break;
    if ((int64_t)(n[k] + m[k] - 1) * maxp >= (int64_t(1) << 30)) {
      rc = set_err(c, PFSP_ERANGE, "(n + m - 1) * max(p) must stay below 2^30");
      break;
    }
    x.n = n[k];
    x.m = m[k];
    x.P = x.m * (x.m - 1) / 2;
    x.narrow = maxp < 65536 && (int64_t)(x.m > 2 ? x.m - 2 : 0) * maxp < (1 << 24);
    x.l16 = x.narrow && (int64_t)(x.m > 1 ? x.m - 1 : 0) * maxp < (1 << 16);
    x.x16 = x.l16 && (int64_t)(x.n + x.m) * maxp < (1 << 15);
    const size_t P = x.P > 0 ? x.P : 1;
    if (hipMalloc(&x.d_p, (size_t)x.n * x.m * 4) != hipSuccess ||
        hipMalloc(&x.d_T, (size_t)x.m * 4) != hipSuccess || hipMalloc(&x.d_pu, P) != hipSuccess ||
        hipMalloc(&x.d_pv, P) != hipSuccess ||
        (x.narrow ? hipMalloc(&x.d_ent, (size_t)x.n * P * 8)
                  : hipMalloc(&x.d_entw, (size_t)x.n * P * 16)) != hipSuccess) {
      rc = set_err(c, PFSP_ENOMEM, "device allocation failed");
      break;
    }
    if (hipMemcpy(x.d_p, p[k], (size_t)x.n * x.m * 4, hipMemcpyHostToDevice) != hipSuccess) {
      rc = set_err(c, PFSP_EDEVICE, "copy failed");
      break;
    }
    rc = stage_tables(c, mt->stream, x.n, x.m, x.d_p, x.d_T, x.d_ent, x.d_entw, x.d_pu, x.d_pv,
                      x.narrow);
    if (rc == PFSP_OK && x.narrow && x.x16 && x.n > 20 && x.n <= 128 && x.P > 0 &&
        c->wide_lb2 && !c->force_generic)
      rc = stage_quick(c, mt->stream, x.n, x.m, x.d_ent, &x.d_entq);
    x.cls = class_of(x, c);
    mt->nmax = std::max(mt->nmax, x.n);
    mt->mmax = std::max(mt->mmax, x.m);
  }
  if (rc == PFSP_OK) {
    std::vector<DevInst> views(count);
    for (int k = 0; k < count; ++k) views[k] = mt->in[k].view();
    if (hipMalloc(&mt->d_insts, count * sizeof(DevInst)) != hipSuccess ||
        hipMalloc(&mt->d_seg, (count + 1) * sizeof(long long)) != hipSuccess ||
        hipMalloc(&mt->d_ubs, count * sizeof(int)) != hipSuccess ||
        hipMalloc(&mt->d_queue, kNumCls * sizeof(int)) != hipSuccess)
      rc = set_err(c, PFSP_ENOMEM, "device allocation failed");
    else if (hipMemcpy(mt->d_insts, views.data(), count * sizeof(DevInst),
                       hipMemcpyHostToDevice) != hipSuccess)
      rc = set_err(c, PFSP_EDEVICE, "copy failed");
  }
  if (rc) {
    pfsp_multi_destroy(mt);
    return rc;
  }
  *out = mt;
  return PFSP_OK;
}

void pfsp_multi_destroy(pfsp_multi *mt) {
  if (!mt) return;
  if (mt->stream) (void)hipStreamSynchronize(mt->stream);
  multi_drop_graph(mt);
  for (MultiInst &x : mt->in) {
    void *bufs[] = {x.d_p, x.d_T, x.d_ent, x.d_entq, x.d_entw, x.d_pu, x.d_pv};
    for (void *b : bufs) (void)hipFree(b);
  }
  void *bufs[] = {mt->d_insts, mt->d_seg, mt->d_ubs, mt->d_costs, mt->d_tiles, mt->d_queue};
  for (void *b : bufs) (void)hipFree(b);
  if (mt->stream) (void)hipStreamDestroy(mt->stream);
  delete mt;
}

int pfsp_multi_bound(pfsp_multi *mt, int lb_kind, const uint8_t *perm, const uint8_t *d1,
                     const uint8_t *d2, int32_t stride, const int64_t *seg_begin,
                     const int32_t *ub, int32_t *out_lb, uint8_t *out_prune, uint8_t *dir_out) {
  if (!mt) return PFSP_EINVAL;
  Ctx *c = mt->c;
  std::vector<long long> seg;
  int rc = multi_check_args(mt, lb_kind, perm, d1, d2, stride, seg_begin, ub, out_lb, out_prune,
                            dir_out, seg);
  if (rc) return rc;
  PFSP_HIP(c, hipSetDevice(c->device));
  // the pool may still be written by work queued on the ctx stream
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  rc = multi_run(mt, lb_kind, perm, d1, d2, stride, seg, ub, out_lb, out_prune, dir_out);
  if (rc) return rc;
  PFSP_HIP(c, hipStreamSynchronize(mt->stream));
  return PFSP_OK;
}

int pfsp_multi_set_shape(pfsp_multi *mt, int32_t tile, int32_t waves_small, int32_t waves_large,
                         int32_t blocks_per_cu) {
  if (!mt) return PFSP_EINVAL;
  Ctx *c = mt->c;
  if (tile < 1 || tile > (1 << 20) || waves_small < 0 || waves_small > 16 || waves_large < 0 ||
      waves_large > 8 || blocks_per_cu < 0 || blocks_per_cu > 64)
    return set_err(c, PFSP_ERANGE, "shape out of range");
  mt->tile = tile;
  mt->waves[0] = waves_small;
  mt->waves[1] = waves_large;
  mt->grid_per_cu = blocks_per_cu;
  return PFSP_OK;
}

// Times every candidate shape on the given batch (median of `reps` graph
// replays each) and keeps the fastest; writes a JSON report.
int pfsp_multi_autotune(pfsp_multi *mt, int lb_kind, const uint8_t *perm, const uint8_t *d1,
                        const uint8_t *d2, int32_t stride, const int64_t *seg_begin,
                        const int32_t *ub, int32_t *out_lb, uint8_t *out_prune, uint8_t *dir_out,
                        int32_t reps, char *report, int32_t report_len) {
  if (!mt) return PFSP_EINVAL;
  Ctx *c = mt->c;
  std::vector<long long> seg;
  int rc = multi_check_args(mt, lb_kind, perm, d1, d2, stride, seg_begin, ub, out_lb, out_prune,
                            dir_out, seg);
  if (rc) return rc;
  if (reps < 1) reps = 3;
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));  // the pool may be written on the ctx stream
  const int tiles[] = {64, 128, 256, 512, 1024};
  const int wv[] = {0, 2, 4, 8, 12, 16};
  const int gpc[] = {0, 2, 4, 8};
  struct Cand {
    int tile, w, g;
    double ms;
  };
  std::vector<Cand> res;
  hipEvent_t e0, e1;
  PFSP_HIP(c, hipEventCreate(&e0));
  PFSP_HIP(c, hipEventCreate(&e1));
  const int saved_timing = (int)c->timing;
  c->timing = 0;
  for (int t : tiles)
    for (int w : wv)
      for (int g : gpc) {
        mt->tile = t;
        mt->waves[0] = mt->waves[1] = w;
        mt->grid_per_cu = g;
        rc = multi_run(mt, lb_kind, perm, d1, d2, stride, seg, ub, out_lb, out_prune, dir_out);
        if (rc) break;
        std::vector<double> ts;
        for (int r = 0; r < reps; ++r) {
          PFSP_HIP(c, hipEventRecord(e0, mt->stream));
          rc = multi_run(mt, lb_kind, perm, d1, d2, stride, seg, ub, out_lb, out_prune, dir_out);
          if (rc) break;
          PFSP_HIP(c, hipEventRecord(e1, mt->stream));
          PFSP_HIP(c, hipEventSynchronize(e1));
          float ms = 0.f;
          PFSP_HIP(c, hipEventElapsedTime(&ms, e0, e1));
          ts.push_back(ms);
        }
        if (rc) break;
        std::sort(ts.begin(), ts.end());
        res.push_back({t, w, g, ts[ts.size() / 2]});
      }
  c->timing = saved_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const Cand best = *std::min_element(res.begin(), res.end(),
                                      [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
  double default_ms = -1;
  for (const Cand &x : res)
    if (x.tile == 256 && x.w == 0 && x.g == 0) default_ms = x.ms;
  mt->tile = best.tile;
  mt->waves[0] = mt->waves[1] = best.w;
  mt->grid_per_cu = best.g;
  if (report && report_len > 0) {
    std::string js = "{\"best\": {\"tile\": " + std::to_string(best.tile) +
                     ", \"waves\": " + std::to_string(best.w) +
                     ", \"blocks_per_cu\": " + std::to_string(best.g) +
                     ", \"ms\": " + std::to_string(best.ms) +
                     "}, \"default_ms\": " + std::to_string(default_ms) +
                     ", \"candidates\": " + std::to_string(res.size()) + "}";
    snprintf(report, (size_t)report_len, "%s", js.c_str());
  }
  return PFSP_OK;
}

}  // extern "C"
