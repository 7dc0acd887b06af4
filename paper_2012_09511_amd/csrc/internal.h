// Internal declarations of the gfx950 flow-shop bounding library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/pfsp.h"

namespace pfsp {

constexpr int kMaxN = 255;
constexpr int kMaxM = 64;
// Sentinel below every reachable bound value: instances are limited to
// (n + m - 1) * max(p) < 2^30, so NEG minus any processing time stays above
// INT32_MIN and NEG plus any path length stays negative.
constexpr int kNeg = -(1 << 30);
constexpr int kInt32Max = 0x7fffffff;

// Device view of a staged instance (Section 2.4: pre-sorted two-machine
// schedules for every machine pair).
struct DevInst {
  int n, m, P;
  int narrow;              // 1: ent holds packed 8-byte entries, else entw
  int l16;                 // 1: (m - 1) * max p < 2^16, so every a + lag fits 16 bits (NMAX <= 32)
  int x16;                 // 1: l16 and (n + m) * max p < 2^15 (quick kernels store X in 16 bits)
  const int *p;            // [n][m] processing times
  const int *T;            // [m] per-machine totals
  const uint2 *ent;        // [n][P] narrow entries: x = a | b << 16, y = lag | k << 24
  const uint4 *entw;       // [n][P] wide entries: {a, b, lag, k}
  const uint2 *entq;       // [P/64 passes][n][64] quick entries (n > 32, x16), else null
  const uint8_t *pu;       // [P] first machine of pair
  const uint8_t *pv;       // [P] second machine of pair
};

// Parent batch as seen by the kernels.
struct DevPool {
  int count, n;                 // count: rows (grid size); see count_dev
  const int *count_dev = nullptr;  // if set, the number of valid rows is *count_dev (<= count)
  const int *ub_dev = nullptr;     // if set, the prune threshold is *ub_dev
  const uint8_t *perm, *d1, *d2;
  const uint32_t *mask;
  int mask_words;
  int mask_stride = -1;         // words between rows of mask (-1: mask_words; 0: one row for all)
  uint8_t *dir;
  int16_t *argpair;
  const int *index = nullptr;  // if set, launch row i bounds pool row index[i]
  // depth bins of full LB2 (r = n - d1 - d2): 0 every row; 1 the rows with
  // r > bin_r or r < 1 (the full-scan kernels); 2 the rows with 1 <= r <= bin_r
  // (the deep kernel).  A kernel leaves the other bin's rows untouched.
  int bin = 0, bin_r = 0;
};

// Search-step filter of the costs kernels (row i of the pool):
//  - a dead record (alive[i] == 0, lazy re-check) is skipped;
//  - a parent all of whose children (both directions) have LB1 >= *ub_dev
//    cannot keep a child under any LB2 kind (LB2 >= LB1): its prune row is
//    written here (all pruned, direction 0) and it is left out of the bound
//    kernels;
//  - every other parent is appended to rows[0 .. *open) (any order).
//  - rows_deep (optional): open rows with 1 <= r <= deep_r unscheduled jobs go
//    to rows_deep[0 .. *open_deep) instead (the deep LB2 kernel).
//  - rows_lb1 (optional): open rows with 1 <= r <= lb1_r go to
//    rows_lb1[0 .. *open_lb1) instead, before the deep split (their children
//    are bounded with LB1: the bound chosen by depth).
struct CostFilter {
  const uint8_t *alive;
  const int *ub_dev;
  uint8_t *out_prune;
  uint8_t *dir;
  int *rows;
  int *open;
  int *rows_deep = nullptr;
  int *open_deep = nullptr;
  int deep_r = 0;
  int *rows_lb1 = nullptr;
  int *open_lb1 = nullptr;
  int lb1_r = 0;
};

struct Selector;   // learned pair selector state (selector.hip)
struct SearchState;

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // instance
  int n = 0, m = 0, P = 0;
  int maxp = 0;
  int *p_host = nullptr;
  int *d_p = nullptr, *d_T = nullptr;
  uint2 *d_ent = nullptr;
  uint2 *d_entq = nullptr;  // staged for the wide kernels when n > 32 and x16
  uint4 *d_entw = nullptr;
  uint8_t *d_pu = nullptr, *d_pv = nullptr;
  int narrow = 1;
  int l16 = 1;
  int x16 = 1;
  // workspace: parent front/back/remaining [count][3][m]
  int *d_costs = nullptr;
  size_t costs_cap = 0;
  int *d_flag = nullptr;   // [4] device status words: [0] invalid-row flag
  int *scratch = nullptr;  // this device's fixed workspace (pfsp_bound_children_noalloc)
  // fixed pair set of PFSP_LB2_SUBSET searches (pfsp_search_set_pairs)
  uint32_t *d_static_mask = nullptr;
  int static_words = 0, static_pairs = 0;
  // options
  int64_t pool_batch = 65536;
  int64_t poll_every = 8;
  int64_t pool_capacity = 0;
  int64_t use_graph = 1;
  int64_t learned_topk = 16;
  int64_t learned_exact = 0;
  int64_t timing = 0;
  int64_t force_generic = 0;
  int64_t lb2_waves = 0;      // waves per block of the LB2 kernel (0 = automatic)
  int64_t lb2_blocks_per_cu = 0;  // persistent LB2 blocks per CU (0 = 16)
  int64_t subset_group = 0;   // parents per wave of subset LB2 (0/1 = one, 2, 4)
  int64_t search_filter = 1;  // LB2 search steps bound only parents with a child LB1 < ub
  int64_t log_capacity = 0;   // search node log size in records (0 = off)
  int64_t log_stride = 1;     // log every log_stride-th decomposed node of a batch
  int64_t wide_lb2 = 1;       // full LB2 for 32 < n <= 128 with 16-bit X takes k_lb2w
  int64_t deep_r = 8;         // full LB2: parents with at most deep_r jobs left take k_lb2d
  int64_t lb1_r = 0;          // LB2 searches: parents with at most lb1_r jobs left use LB1
  int64_t heuristic_threads = 0;  // host threads improving the incumbent during searches
  int64_t heuristic_seed = 1;
  struct Pending {
    const char *name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;              // launches whose events are not read yet
  std::map<std::string, std::pair<double, int64_t>> ktime;  // name -> (ms, launches)
  int capturing = 0;                         // a HIP graph capture is in progress
  Selector *sel = nullptr;
  SearchState *search = nullptr;
  std::vector<unsigned char> ivm_ckpt;  // checkpoint of the last IVM search stopped on its budget
  int cu_count = 256;
  DevInst inst() const {
    DevInst I;
    I.n = n; I.m = m; I.P = P; I.narrow = narrow; I.l16 = l16; I.x16 = x16;
    I.p = d_p; I.T = d_T; I.ent = d_ent; I.entw = d_entw; I.pu = d_pu; I.pv = d_pv;
    I.entq = d_entq;
    return I;
  }
};

int set_err(Ctx *c, int code, const std::string &msg);
int hip_err(Ctx *c, hipError_t e, const char *what);
#define PFSP_HIP(c, call)                         \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_err((c), e_, #call); \
  } while (0)

// Event bracketing of kernel launches (option "timing"); no-ops otherwise or
// while a graph is being captured.
struct KTimer {
  Ctx *c;
  hipStream_t s;
  const char *name;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(Ctx *c_, hipStream_t s_, const char *name_) : c(c_), s(s_), name(name_) {
    if (c->timing && !c->capturing && hipEventCreate(&a) == hipSuccess &&
        hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, s);
    else
      a = b = nullptr;
  }
  ~KTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      c->pending.push_back({name, a, b});
    }
  }
};
void collect_timings(Ctx *c);

// stage.hip
int stage_instance(Ctx *c);
int stage_tables(Ctx *c, hipStream_t s, int n, int m, const int *d_p, int *d_T, uint2 *d_ent,
                 uint4 *d_entw, uint8_t *d_pu, uint8_t *d_pv, int narrow);
// Quick-format copy of the narrow pair table for the wide kernels: entries
// {(b - a) in the low 16 bits | job << 24, job | (a + lag) << 16} (job <
// 128) in [pass][position][64 lanes] order, pairs >= P repeating pair 0;
// allocates *d_entq.  Synchronous.
int stage_quick(Ctx *c, hipStream_t s, int n, int m, const uint2 *d_ent, uint2 **d_entq);
// bound.hip
int ensure_costs(Ctx *c, int count);
int launch_bound(Ctx *c, const DevPool &pool, int kind, int ub, int *out_lb,
                 uint8_t *out_prune, hipStream_t s);
int launch_costs(Ctx *c, const DevPool &pool, hipStream_t s, const CostFilter *f = nullptr);
// FNV-1a hash of the loaded instance (n, m, p): checkpoints name their instance.
uint64_t instance_hash(const Ctx *c);

// Parents per wave for subset bounds of at most k pairs per parent: option
// "subset_group" if set, else by k and n.
int subset_group_for(const Ctx *c, int k);
// group: parents per wave for subset bounds (1, 2 or 4; 0 = option "subset_group")
int launch_bound_costs_ready(Ctx *c, const DevPool &pool, int kind, int ub, int *out_lb,
                             uint8_t *out_prune, hipStream_t s, int group = 0);
size_t lb2_lds_bytes(const Ctx *c, int waves);
// Depth threshold of the deep LB2 kernel for this context and kind (0: the
// kernel does not apply; every parent takes the other LB2 kernels).
int deep_bin_r(const Ctx *c, int kind, bool log);
// Full LB2 with the rows split by depth: the deep kernel takes the rows with
// at most deep_bin_r jobs left, the full-scan kernel the others (costs ready).
int launch_lb2_binned(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                      hipStream_t s);
// The deep kernel alone on a pool all of whose rows have 1 <= r <= deep_bin_r.
int launch_lb2d(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                hipStream_t s);
// Workspace of pfsp_bound_children in int32: 3m costs per parent.
size_t workspace_ints(const Ctx *c, int count);
void init_bound_attributes();
void init_selector_attributes();
// multi-instance launches (bound.hip)
struct MultiTile {
  int inst, begin, end, pad;
};
struct FastClassLaunch {
  int nmax;                 // compiled job bound of the class (20, 64 or 128)
  int wide = 0;             // 1: the wide kernel (16-bit X, entries from entq)
  int ppad, nmax_jobs, mmax;  // LDS layout of the class
  const MultiTile *tiles;   // device, grouped by instance
  int ntiles;
  int *queue;               // device tile counter (zeroed by the launcher)
  int waves, grid;
  int cstride;              // ints per parent row of the costs workspace (3 * largest m)
  int x16;                  // every instance of the class allows 16-bit X
};
size_t lb2m_lds_bytes(int nmax, int ppad, int nmax_jobs, int mmax, int waves, int x16,
                      int wide);
int launch_generic_instance(Ctx *c, const DevInst &I, const DevPool &pool, int ub, int *costs,
                            int *out_lb, uint8_t *out_prune, hipStream_t s);
int launch_lb1m(Ctx *c, const DevInst *insts, const long long *seg, int ninst, long long total,
                const uint8_t *perm, const uint8_t *d1, const uint8_t *d2, int stride, int nmax,
                int mmax, const int *ubs, int *out_lb, uint8_t *out_prune, uint8_t *dir,
                int *costs, int write_out, hipStream_t s);
int launch_lb2m(Ctx *c, const FastClassLaunch &L, const DevInst *insts, const uint8_t *perm,
                const uint8_t *d1, const uint8_t *d2, int stride, const int *ubs,
                const int *costs, int *out_lb, uint8_t *out_prune, uint8_t *dir, hipStream_t s);
// selector.hip
int launch_learned(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                   hipStream_t s);
int launch_learned_ready(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                   hipStream_t s);
int learned_prepare(Ctx *c, int rows);
// 0: no selector, 1: float model, 2: integer model (changes the captured step)
int selector_mode(const Ctx *c);
void selector_free(Ctx *c);
// search.hip
void search_free(Ctx *c);
// noalloc.hip: looks up this device's scratch array address (device current)
int noalloc_attach(Ctx *c);
// neh.cpp
int neh_host(int n, int m, const int *p, int *perm_out, int *cmax_out);

}  // namespace pfsp

struct pfsp_ctx {
  pfsp::Ctx impl;
};
