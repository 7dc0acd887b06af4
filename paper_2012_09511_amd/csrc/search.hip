// Depth-first branch-and-bound on the device (Sections 2.2-2.5).
//
// The paper keeps K integer-vector-matrix explorers per GPU and balances them
// by work stealing (Sections 2.5, 3.1-3.4).  Here the open subproblems live in
// one device stack of node records (perm[n], d1, d2, lb); every step pops the
// top `pool_batch` records, decomposes them with the bounding kernels of
// bound.hip (both children sets, MinMin, prune flags), and pushes each
// parent's surviving children back in list order with the leftmost child on
// top, parents nearer the top of the stack ending nearer the top.  Popping
// from the top keeps the search depth-first while every step still feeds the
// GPU a full batch; balancing is implicit because all parents share the stack.
//
// Step = k_pop -> k_gather -> the costs kernel with its LB1 filter -> the LB2
// kernels (and k_lb1 for the LB1 band) -> k_count_scan -> k_scan_top -> k_push.  All sizes and the incumbent are read from a control
// block in device memory, so the step is captured once as a HIP graph and
// replayed; the host reads the control block every `poll_every` steps.
//
// Pruning (Section 2.2): a child is discarded iff LB >= incumbent.  A popped
// record whose stored LB is no longer below the incumbent is dropped without
// being decomposed (lazy re-check).  A leaf child (no unscheduled job left)
// carries its makespan as LB; if it is below the step's incumbent it lowers
// the incumbent with atomicMin and the best leaf of the step is recorded.
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "heuristic.h"
#include "internal.h"

namespace pfsp {

struct SearchCtl {
  int top;         // records on the stack
  int count;       // records popped this step
  int base;        // stack index of the first popped record
  int ub;          // incumbent (lowered by atomicMin)
  int ub_step;     // incumbent at the start of the step: prune threshold
  int overflow;    // a push would have exceeded the capacity
  int newbest;     // a leaf improved the incumbent since the last poll
  int pad0;
  unsigned long long step_best;  // (makespan << 32) | batch index of the step's best leaf
  long long nodes;               // decomposed nodes
  long long children;            // bounded children
  long long steps;               // steps that popped at least one record
  long long log_count;           // decomposed nodes offered to the node log
};

struct SearchState {
  int n = 0, N = 0;
  long long cap = 0;
  hipStream_t stream = nullptr;
  // stack
  uint8_t *s_perm = nullptr, *s_d1 = nullptr, *s_d2 = nullptr;
  int *s_lb = nullptr;
  // batch
  uint8_t *b_perm = nullptr, *b_d1 = nullptr, *b_d2 = nullptr, *b_dir = nullptr;
  int *b_lb = nullptr;
  uint8_t *b_alive = nullptr;
  int *out_lb = nullptr;
  uint8_t *out_prune = nullptr;
  int *cnt = nullptr, *offs = nullptr, *bsum = nullptr;
  uint8_t *best_perm = nullptr;
  SearchCtl *ctl = nullptr, *ctl_host = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<long long> graph_key;  // options the captured step depends on
  // LB2 steps: parents that survive the costs kernels' LB1 filter (those with
  // few jobs left in rows_deep, counted in open[1], for the deep kernel; with
  // option lb1_r, those with at most lb1_r in rows_lb1, counted in open[2],
  // for LB1)
  int *rows = nullptr, *open = nullptr, *rows_deep = nullptr, *rows_lb1 = nullptr;
  // node log (option log_capacity > 0): every log_stride-th decomposed node
  uint8_t *l_perm = nullptr, *l_d1 = nullptr, *l_d2 = nullptr;
  long long log_cap = 0;
  // records moved to host memory from the bottom of the device stack (the
  // shallowest open nodes, needed only once everything above them is done)
  std::vector<uint8_t> h_perm, h_d1, h_d2;
  std::vector<int> h_lb;
  // the search that pfsp_search_dump / pfsp_search_resume continue
  int32_t ub0 = 0;
  int kind = 0;
  int resumable = 0;  // the last search stopped on its budget
};

constexpr int kScanBlock = 1024;  // parents per k_count_scan block (256 threads x 4)

__global__ void k_clear(int *p) { *p = 0; }
__global__ void k_lower_ub(SearchCtl *c, int v) { atomicMin(&c->ub, v); }
// Takes the step's batch from the top of the stack and clears the counters of
// the LB1 filter's lists.
__global__ void k_pop(SearchCtl *c, int N, int *open) {
  const int top = c->top;
  const int count = top < N ? top : N;
  c->count = count;
  c->base = top - count;
  c->top = top - count;
  c->ub_step = c->ub;
  c->step_best = ~0ull;
  if (count > 0) c->steps += 1;
  open[0] = 0;
  open[1] = 0;
  open[2] = 0;
}

__global__ void k_gather(const SearchCtl *__restrict__ c, int n, const uint8_t *__restrict__ s_perm,
                         const uint8_t *__restrict__ s_d1, const uint8_t *__restrict__ s_d2,
                         const int *__restrict__ s_lb, uint8_t *__restrict__ b_perm,
                         uint8_t *__restrict__ b_d1, uint8_t *__restrict__ b_d2,
                         int *__restrict__ b_lb, uint8_t *__restrict__ b_alive) {
  const int count = c->count, base = c->base, ub = c->ub_step;
  const long long total = (long long)count * n;
  const uint8_t *src = s_perm + (size_t)base * n;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x)
    b_perm[x] = src[x];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    b_d1[i] = s_d1[base + i];
    b_d2[i] = s_d2[base + i];
    const int lb = s_lb[base + i];
    b_lb[i] = lb;
    b_alive[i] = lb < ub;  // lazy re-check against the current incumbent
  }
}

// Appends every stride-th decomposed node of the batch to the node log.
__global__ void k_log(SearchCtl *__restrict__ c, int n, const uint8_t *__restrict__ b_perm,
                      const uint8_t *__restrict__ b_d1, const uint8_t *__restrict__ b_d2,
                      const uint8_t *__restrict__ b_alive, int stride, long long cap,
                      uint8_t *__restrict__ l_perm, uint8_t *__restrict__ l_d1,
                      uint8_t *__restrict__ l_d2) {
  const int count = c->count;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || !b_alive[i] || i % stride) return;
  const long long slot = (long long)atomicAdd((unsigned long long *)&c->log_count, 1ull);
  if (slot >= cap) return;
  for (int x = 0; x < n; ++x) l_perm[slot * n + x] = b_perm[(size_t)i * n + x];
  l_d1[slot] = b_d1[i];
  l_d2[slot] = b_d2[i];
}

// Per parent: node statistics, leaf incumbent updates, and the number of
// surviving non-leaf children of the chosen direction (cnt); then the
// exclusive scan of cnt within blocks of kScanBlock parents (offs, and the
// block totals in bsum).  A thread takes four consecutive parents.
__device__ __forceinline__ int survivors(SearchCtl *__restrict__ c, int n, int i, int ub,
                                         const uint8_t *__restrict__ b_d1,
                                         const uint8_t *__restrict__ b_d2,
                                         const uint8_t *__restrict__ b_dir,
                                         const int *__restrict__ out_lb,
                                         const uint8_t *__restrict__ out_prune) {
  const int r = n - b_d1[i] - b_d2[i];
  const int dir = b_dir[i];
  const int *lb = out_lb + ((size_t)i * 2 + dir) * n;
  const uint8_t *pr = out_prune + ((size_t)i * 2 + dir) * n;
  int s = 0;
  if (r == 1) {  // leaf children: the bound is the makespan (pruned: not below ub)
    const int v = lb[0];
    if (!pr[0] && v < ub) {
      atomicMin(&c->ub, v);
      atomicMin(&c->step_best, ((unsigned long long)(unsigned)v << 32) | (unsigned)i);
    }
  } else if ((n & 3) == 0) {  // rows start on 4-byte boundaries: a word per 4 flags
    const uint32_t *pw = (const uint32_t *)pr;
    for (int w = 0; 4 * w < r; ++w) {
      const int valid = min(4, r - 4 * w);  // flags are 0 or 1
      const uint32_t keep = 0x01010101u >> (8 * (4 - valid));
      s += valid - __popc(pw[w] & keep);
    }
  } else {
    for (int q = 0; q < r; ++q) s += pr[q] == 0;
  }
  return s;
}

__global__ void __launch_bounds__(256)
k_count_scan(SearchCtl *__restrict__ c, int n, const uint8_t *__restrict__ b_d1,
             const uint8_t *__restrict__ b_d2, const uint8_t *__restrict__ b_alive,
             const uint8_t *__restrict__ b_dir, const int *__restrict__ out_lb,
             const uint8_t *__restrict__ out_prune, int *__restrict__ cnt,
             int *__restrict__ offs, int *__restrict__ bsum) {
  __shared__ int sh[256];
  __shared__ unsigned long long sn, sc;
  const int count = c->count, ub = c->ub_step;
  const int base = blockIdx.x * kScanBlock;
  if (base >= count) return;
  if (threadIdx.x == 0) sn = sc = 0;
  int v[4], tot = 0;
  unsigned long long nodes = 0, children = 0;
  for (int k = 0; k < 4; ++k) {
    const int i = base + threadIdx.x * 4 + k;
    int s = 0;
    if (i < count && b_alive[i]) {
      nodes += 1;
      children += 2 * (n - b_d1[i] - b_d2[i]);
      s = survivors(c, n, i, ub, b_d1, b_d2, b_dir, out_lb, out_prune);
    }
    if (i < count) cnt[i] = s;
    v[k] = s;
    tot += s;
  }
  sh[threadIdx.x] = tot;
  __syncthreads();  // also orders the clear of sn, sc before the sums below
  if (nodes) {
    atomicAdd(&sn, nodes);
    atomicAdd(&sc, children);
  }
  for (int o = 1; o < 256; o <<= 1) {  // inclusive Hillis-Steele scan of thread totals
    const int x = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tot;
  for (int k = 0; k < 4; ++k) {
    const int i = base + threadIdx.x * 4 + k;
    if (i < count) offs[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = sh[255];
  if (threadIdx.x == 0 && sn) {  // the scan's barriers order every add before this read
    atomicAdd((unsigned long long *)&c->nodes, sn);
    atomicAdd((unsigned long long *)&c->children, sc);
  }
}

// Exclusive scan of the block sums; sets the new stack top (or the overflow flag).
__global__ void __launch_bounds__(1024)
k_scan_top(SearchCtl *__restrict__ c, int *__restrict__ bsum, long long cap) {
  __shared__ int sh[1024];
  const int count = c->count;
  const int nb = (count + kScanBlock - 1) / kScanBlock;
  const int per = (nb + 1023) / 1024;
  int tot = 0;
  for (int k = 0; k < per; ++k) {
    const int b = threadIdx.x * per + k;
    if (b < nb) tot += bsum[b];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int x = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tot;
  for (int k = 0; k < per; ++k) {
    const int b = threadIdx.x * per + k;
    if (b < nb) {
      const int x = bsum[b];
      bsum[b] = run;
      run += x;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long top = (long long)c->base + sh[1023];
    if (top > cap) {
      c->overflow = 1;
      c->top = c->base;
    } else {
      c->top = (int)top;
    }
  }
}

// One wave per parent: the prune flags and bounds of 64 children are read at
// once, the survivors of the chosen direction ranked by a ballot (leftmost
// child on top of the stack), their indices put in LDS; then the survivors'
// records are written floor(64 / n) at a time, each by n consecutive lanes on
// consecutive bytes.  The step's best leaf is stored too.
__global__ void __launch_bounds__(256)
k_push(SearchCtl *__restrict__ c, int n, const uint8_t *__restrict__ b_perm,
       const uint8_t *__restrict__ b_d1, const uint8_t *__restrict__ b_d2,
       const uint8_t *__restrict__ b_dir, const int *__restrict__ out_lb,
       const uint8_t *__restrict__ out_prune, const int *__restrict__ cnt,
       const int *__restrict__ offs, const int *__restrict__ bsum, uint8_t *__restrict__ s_perm,
       uint8_t *__restrict__ s_d1, uint8_t *__restrict__ s_d2, int *__restrict__ s_lb,
       uint8_t *__restrict__ best_perm) {
  __shared__ int sq[4][64];  // per wave: child index of each survivor rank
  const int count = c->count;
  if (c->overflow) return;
  const int lane = threadIdx.x & 63;
  int *const rank_q = sq[threadIdx.x >> 6];
  const int waves = (gridDim.x * blockDim.x) >> 6;
  const unsigned long long sb = c->step_best;
  // record writers: G groups of n lanes (n <= 64), else the whole wave
  const int G = n <= 64 ? 64 / n : 1;
  const int gi = n <= 64 ? lane / n : 0, xl = n <= 64 ? lane - gi * n : lane;
  const int xstep = n <= 64 ? n : 64;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < count; i += waves) {
    const uint8_t *row = b_perm + (size_t)i * n;
    if (sb != ~0ull && (int)(sb & 0xffffffffu) == i) {
      // the step's best leaf: a one-job parent's only child is its own permutation
      for (int x = lane; x < n; x += 64) best_perm[x] = row[x];
      if (lane == 0) c->newbest = 1;
    }
    const int s = cnt[i];
    if (s == 0) continue;
    const int a = b_d1[i], b = b_d2[i], r = n - a - b, dir = b_dir[i];
    const int *lb = out_lb + ((size_t)i * 2 + dir) * n;
    const uint8_t *pr = out_prune + ((size_t)i * 2 + dir) * n;
    const long long dst = (long long)c->base + bsum[i / kScanBlock] + offs[i];
    int done = 0;  // survivors among earlier chunks of 64 children
    for (int q0 = 0; q0 < r; q0 += 64) {
      const int ql = q0 + lane;
      const bool live = ql < r && pr[ql] == 0;
      const int lbv = live ? lb[ql] : 0;
      const uint64_t bal = __ballot(live);
      if (live)
        rank_q[__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0))] = ql;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int nl = __popcll(bal);
      for (int t0 = 0; t0 < nl; t0 += G) {
        const int tt = t0 + gi;
        const bool act = gi < G && tt < nl;
        const int q = rank_q[act ? tt : t0];
        const int lq = __shfl(lbv, q - q0, 64);
        if (act) {
          const long long pos = dst + (s - 1 - (done + tt));
          uint8_t *out = s_perm + pos * n;
          const int j = row[a + q];
          for (int x = xl; x < n; x += xstep) {
            int v;
            if (x < a || x >= a + r) {
              v = row[x];
            } else if (dir == 0) {  // sigma1 j | U \ j | sigma2
              v = x == a ? j : (x <= a + q ? row[x - 1] : row[x]);
            } else {  // sigma1 | U \ j | j sigma2
              v = x == a + r - 1 ? j : (x < a + q ? row[x] : row[x + 1]);
            }
            out[x] = (uint8_t)v;
          }
          if (xl == 0) {
            s_d1[pos] = (uint8_t)(a + (dir == 0));
            s_d2[pos] = (uint8_t)(b + (dir == 1));
            s_lb[pos] = lq;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // rank_q is rewritten by the next chunk
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      done += nl;
    }
  }
}

__global__ void k_init_root(SearchCtl *c, int n, int ub0, uint8_t *s_perm, uint8_t *s_d1,
                            uint8_t *s_d2, int *s_lb) {
  const int x = threadIdx.x;
  for (int j = x; j < n; j += blockDim.x) s_perm[j] = (uint8_t)j;
  if (x == 0) {
    s_d1[0] = 0;
    s_d2[0] = 0;
    s_lb[0] = (int)0x80000000;  // the root is always decomposed
    c->top = 1;
    c->count = 0;
    c->base = 0;
    c->ub = ub0;
    c->ub_step = ub0;
    c->overflow = 0;
    c->newbest = 0;
    c->step_best = ~0ull;
    c->nodes = 0;
    c->children = 0;
    c->steps = 0;
    c->log_count = 0;
  }
}

void search_free(Ctx *c) {
  SearchState *S = c->search;
  if (!S) return;
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->graph) (void)hipGraphDestroy(S->graph);
  void *bufs[] = {S->s_perm, S->s_d1, S->s_d2, S->s_lb, S->b_perm, S->b_d1, S->b_d2, S->b_dir,
                  S->b_lb, S->b_alive, S->out_lb, S->out_prune, S->cnt, S->offs, S->bsum,
                  S->best_perm, S->ctl, S->l_perm, S->l_d1, S->l_d2, S->rows, S->open,
                  S->rows_deep, S->rows_lb1};
  for (void *p : bufs) (void)hipFree(p);
  if (S->ctl_host) (void)hipHostFree(S->ctl_host);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
  c->search = nullptr;
}

static int search_alloc(Ctx *c) {
  const int n = c->n;
  const int N = (int)c->pool_batch;
  long long cap = c->pool_capacity;
  if (cap <= 0) cap = (long long)N * (n * (n + 1) / 2 + 1);
  if (cap > 0x7fffffffLL) cap = 0x7fffffffLL;
  SearchState *S = c->search;
  if (S && S->n == n && S->N == N && S->cap == cap && S->log_cap == c->log_capacity)
    return PFSP_OK;
  search_free(c);
  S = new (std::nothrow) SearchState();
  if (!S) return set_err(c, PFSP_ENOMEM, "host allocation failed");
  c->search = S;
  S->n = n;
  S->N = N;
  S->cap = cap;
  const int nb = (N + kScanBlock - 1) / kScanBlock;
  bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
  auto alloc = [&](void **p, size_t bytes) {
    if (ok && hipMalloc(p, bytes ? bytes : 1) != hipSuccess) ok = false;
  };
  alloc((void **)&S->s_perm, (size_t)cap * n);
  alloc((void **)&S->s_d1, (size_t)cap);
  alloc((void **)&S->s_d2, (size_t)cap);
  alloc((void **)&S->s_lb, (size_t)cap * 4);
  alloc((void **)&S->b_perm, (size_t)N * n);
  alloc((void **)&S->b_d1, (size_t)N);
  alloc((void **)&S->b_d2, (size_t)N);
  alloc((void **)&S->b_dir, (size_t)N);
  alloc((void **)&S->b_lb, (size_t)N * 4);
  alloc((void **)&S->b_alive, (size_t)N);
  alloc((void **)&S->out_lb, (size_t)N * 2 * n * 4);
  alloc((void **)&S->out_prune, (size_t)N * 2 * n);
  alloc((void **)&S->cnt, (size_t)N * 4);
  alloc((void **)&S->offs, (size_t)N * 4);
  alloc((void **)&S->bsum, (size_t)nb * 4);
  alloc((void **)&S->best_perm, (size_t)n);
  alloc((void **)&S->ctl, sizeof(SearchCtl));
  alloc((void **)&S->rows, (size_t)N * 4);
  alloc((void **)&S->rows_deep, (size_t)N * 4);
  alloc((void **)&S->rows_lb1, (size_t)N * 4);
  alloc((void **)&S->open, 12);
  S->log_cap = c->log_capacity;
  if (S->log_cap > 0) {
    alloc((void **)&S->l_perm, (size_t)S->log_cap * n);
    alloc((void **)&S->l_d1, (size_t)S->log_cap);
    alloc((void **)&S->l_d2, (size_t)S->log_cap);
  }
  if (ok && hipHostMalloc((void **)&S->ctl_host, sizeof(SearchCtl), hipHostMallocDefault) !=
                hipSuccess)
    ok = false;
  if (!ok) {
    search_free(c);
    return set_err(c, PFSP_ENOMEM, "search buffers do not fit in device memory");
  }
  // the bound workspace is sized here: nothing may allocate during capture
  return ensure_costs(c, N);
}

// Enqueues one search step on the search stream.
static int enqueue_step(Ctx *c, int kind) {
  SearchState *S = c->search;
  const int n = c->n, N = S->N;
  hipStream_t s = S->stream;
  const int nb = (N + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_pop, dim3(1), dim3(1), 0, s, S->ctl, N, S->open);
  const int gg = (int)(((long long)N * n + 255) / 256 < 4096 ? ((long long)N * n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_gather, dim3(gg), dim3(256), 0, s, S->ctl, n, S->s_perm, S->s_d1, S->s_d2,
                     S->s_lb, S->b_perm, S->b_d1, S->b_d2, S->b_lb, S->b_alive);
  if (S->log_cap > 0)
    hipLaunchKernelGGL(k_log, dim3((N + 255) / 256), dim3(256), 0, s, S->ctl, n, S->b_perm,
                       S->b_d1, S->b_d2, S->b_alive, (int)c->log_stride, S->log_cap, S->l_perm,
                       S->l_d1, S->l_d2);
  DevPool pool;
  pool.count = N;
  pool.n = n;
  pool.count_dev = &S->ctl->count;
  pool.ub_dev = &S->ctl->ub_step;
  pool.perm = S->b_perm;
  pool.d1 = S->b_d1;
  pool.d2 = S->b_d2;
  pool.mask = nullptr;
  pool.mask_words = 0;
  if (kind == PFSP_LB2_SUBSET) {  // one pair set for every node
    pool.mask = c->d_static_mask;
    pool.mask_words = c->static_words;
    pool.mask_stride = 0;
  }
  pool.dir = S->b_dir;
  pool.argpair = nullptr;
  int rc;
  if (kind != PFSP_LB1 && c->search_filter) {
    // parents whose children all have LB1 >= ub are closed by the costs
    // kernel (LB2 >= LB1 cannot keep a child); only the others are bounded
    // parents with few jobs left go to a list of their own for the deep kernel
    // and, with lb1_r, those with at most lb1_r to one bounded with LB1 (the
    // bound chosen by depth; Section 2.4 ranks LB1 the cheaper, weaker one)
    const int deep = deep_bin_r(c, kind, false);
    const int lb1_r = (int)c->lb1_r;
    CostFilter f{S->b_alive, &S->ctl->ub_step, S->out_prune, S->b_dir, S->rows, S->open};
    if (deep) {
      f.rows_deep = S->rows_deep;
      f.open_deep = S->open + 1;
      f.deep_r = deep;
    }
    if (lb1_r > 0) {
      f.rows_lb1 = S->rows_lb1;
      f.open_lb1 = S->open + 2;
      f.lb1_r = lb1_r;
    }
    rc = launch_costs(c, pool, s, &f);
    if (rc) return rc;
    if (lb1_r > 0) {
      DevPool lp = pool;
      lp.index = S->rows_lb1;
      lp.count_dev = S->open + 2;
      rc = launch_bound(c, lp, PFSP_LB1, 0, S->out_lb, S->out_prune, s);
      if (rc) return rc;
    }
    DevPool op = pool;
    op.index = S->rows;
    op.count_dev = S->open;
    if (kind == PFSP_LB2_LEARNED) {
      rc = launch_learned_ready(c, op, 0, S->out_lb, S->out_prune, s);
    } else {
      // a fixed selection of at most 32 (16) pairs fills half (a quarter of) a
      // wave: several parents per wave
      const int group = kind == PFSP_LB2_SUBSET ? subset_group_for(c, (int)c->static_pairs) : 0;
      rc = launch_bound_costs_ready(c, op, kind, 0, S->out_lb, S->out_prune, s, group);
      if (!rc && deep) {
        DevPool dp = pool;
        dp.index = S->rows_deep;
        dp.count_dev = S->open + 1;
        rc = launch_lb2d(c, dp, 0, S->out_lb, S->out_prune, s);
      }
    }
  } else if (kind == PFSP_LB2_LEARNED) {
    rc = launch_learned(c, pool, 0, S->out_lb, S->out_prune, s);
  } else {
    rc = launch_bound(c, pool, kind, 0, S->out_lb, S->out_prune, s);
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_count_scan, dim3(nb), dim3(256), 0, s, S->ctl, n, S->b_d1, S->b_d2,
                     S->b_alive, S->b_dir, S->out_lb, S->out_prune, S->cnt, S->offs, S->bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, S->ctl, S->bsum, S->cap);
  const int pw = (N + 3) / 4 < 8192 ? (N + 3) / 4 : 8192;
  hipLaunchKernelGGL(k_push, dim3(pw), dim3(256), 0, s, S->ctl, n, S->b_perm, S->b_d1, S->b_d2,
                     S->b_dir, S->out_lb, S->out_prune, S->cnt, S->offs, S->bsum, S->s_perm,
                     S->s_d1, S->s_d2, S->s_lb, S->best_perm);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

// Everything enqueue_step's launches depend on besides the buffers.
static std::vector<long long> step_key(const Ctx *c, int kind) {
  const SearchState *S = c->search;
  return {kind, S->log_cap > 0 ? c->log_stride : 0, c->search_filter, c->learned_topk,
          c->learned_exact, c->subset_group, c->lb2_waves, c->lb2_blocks_per_cu,
          c->force_generic, c->wide_lb2, c->deep_r, selector_mode(c), c->static_pairs,
          c->lb1_r};
}

static int build_graph(Ctx *c, int kind) {
  SearchState *S = c->search;
  const std::vector<long long> key = step_key(c, kind);
  if (S->gexec && S->graph_key == key) return PFSP_OK;
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->graph) (void)hipGraphDestroy(S->graph);
  S->gexec = nullptr;
  S->graph = nullptr;
  PFSP_HIP(c, hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = 1;
  int rc = enqueue_step(c, kind);
  c->capturing = 0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(S->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_err(c, e, "hipStreamEndCapture");
  S->graph = g;
  PFSP_HIP(c, hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0));
  S->graph_key = key;
  return PFSP_OK;
}

// Moves the bottom `count` records of the device stack (top records) to the
// end of the host stack and shifts the rest down.  The stream is idle.
static int spill(Ctx *c, long long top, long long count) {
  SearchState *S = c->search;
  const int n = S->n;
  const size_t h = S->h_d1.size();
  S->h_perm.resize((h + count) * n);
  S->h_d1.resize(h + count);
  S->h_d2.resize(h + count);
  S->h_lb.resize(h + count);
  PFSP_HIP(c, hipMemcpy(S->h_perm.data() + h * n, S->s_perm, (size_t)count * n,
                        hipMemcpyDeviceToHost));
  PFSP_HIP(c, hipMemcpy(S->h_d1.data() + h, S->s_d1, count, hipMemcpyDeviceToHost));
  PFSP_HIP(c, hipMemcpy(S->h_d2.data() + h, S->s_d2, count, hipMemcpyDeviceToHost));
  PFSP_HIP(c, hipMemcpy(S->h_lb.data() + h, S->s_lb, (size_t)count * 4, hipMemcpyDeviceToHost));
  // [count, top) -> [0, top - count) in chunks of at most count records: each
  // chunk's source lies above its destination and above every later write
  for (long long b = 0; b < top - count; b += count) {
    const long long len = std::min(count, top - count - b);
    PFSP_HIP(c, hipMemcpy(S->s_perm + b * n, S->s_perm + (b + count) * n, (size_t)len * n,
                          hipMemcpyDeviceToDevice));
    PFSP_HIP(c, hipMemcpy(S->s_d1 + b, S->s_d1 + b + count, len, hipMemcpyDeviceToDevice));
    PFSP_HIP(c, hipMemcpy(S->s_d2 + b, S->s_d2 + b + count, len, hipMemcpyDeviceToDevice));
    PFSP_HIP(c, hipMemcpy(S->s_lb + b, S->s_lb + b + count, (size_t)len * 4,
                          hipMemcpyDeviceToDevice));
  }
  return PFSP_OK;
}

// Puts the top `count` host records back as the device stack's [0, count).
static int refill(Ctx *c, long long count) {
  SearchState *S = c->search;
  const int n = S->n;
  const size_t h = S->h_d1.size() - count;
  PFSP_HIP(c, hipMemcpy(S->s_perm, S->h_perm.data() + h * n, (size_t)count * n,
                        hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemcpy(S->s_d1, S->h_d1.data() + h, count, hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemcpy(S->s_d2, S->h_d2.data() + h, count, hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemcpy(S->s_lb, S->h_lb.data() + h, (size_t)count * 4, hipMemcpyHostToDevice));
  S->h_perm.resize(h * n);
  S->h_d1.resize(h);
  S->h_d2.resize(h);
  S->h_lb.resize(h);
  return PFSP_OK;
}

static int set_top(Ctx *c, long long top) {
  SearchState *S = c->search;
  const int t = (int)top;
  PFSP_HIP(c, hipMemcpy((char *)S->ctl + offsetof(SearchCtl, top), &t, sizeof(int),
                        hipMemcpyHostToDevice));
  return PFSP_OK;
}

// Replays search steps from the current device state until the tree is
// exhausted (device and host stacks empty) or the budget is spent.
// Host threads that improve the incumbent while the search runs (option
// heuristic_threads); stopped and joined when the search returns.
struct HeurRun {
  Heuristic h;
  bool on = false;
  ~HeurRun() {
    if (on) h.finish();
  }
};

static void heur_start(Ctx *c, HeurRun &hr) {
  if (c->heuristic_threads <= 0) return;
  const int n = c->n, m = c->m;
  std::vector<int> neh(n);
  int cmax = 0;
  neh_host(n, m, c->p_host, neh.data(), &cmax);
  hr.h.n = n;
  hr.h.m = m;
  hr.h.p.assign(c->p_host, c->p_host + (size_t)n * m);
  hr.h.seed = (uint64_t)c->heuristic_seed;
  hr.h.launch((int)c->heuristic_threads, neh, cmax);
  hr.on = true;
}

// At a poll (stream idle): the top open node completed into a schedule for
// the heuristic threads, and the device incumbent lowered to theirs.
static int heur_poll(Ctx *c, HeurRun &hr, const SearchCtl &hc) {
  SearchState *S = c->search;
  const int n = c->n;
  if (hc.top > 0) {
    uint8_t perm[kMaxN], d[2];
    PFSP_HIP(c, hipMemcpy(perm, S->s_perm + (size_t)(hc.top - 1) * n, n, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(&d[0], S->s_d1 + hc.top - 1, 1, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(&d[1], S->s_d2 + hc.top - 1, 1, hipMemcpyDeviceToHost));
    hr.h.offer(complete_node(c->p_host, n, c->m, perm, d[0], d[1]));
  }
  const int v = hr.h.best.load();
  if (v < hc.ub) {
    hipLaunchKernelGGL(k_lower_ub, dim3(1), dim3(1), 0, S->stream, S->ctl, v);
    PFSP_HIP(c, hipGetLastError());
  }
  return PFSP_OK;
}

static int run_search(Ctx *c, int lb_kind, int32_t ub0, int64_t budget_nodes, pfsp_result *res,
                      std::chrono::steady_clock::time_point t0) {
  SearchState *S = c->search;
  const int n = c->n;
  int rc;
  HeurRun hr;
  heur_start(c, hr);
  if (c->use_graph) {
    rc = build_graph(c, lb_kind);
    if (rc) return rc;
  }
  const int k = (int)c->poll_every;
  // a step pushes at most N (n - 1) records: at a poll, keep k steps of room
  const long long grow = (long long)k * S->N * (n > 1 ? n - 1 : 1);
  const long long spill_hi = S->cap - grow;
  int status = PFSP_OK;
  long long max_pool = 1;
  int steps = 0;
  S->resumable = 0;
  for (;;) {
    for (int t = 0; t < k; ++t) {
      if (c->use_graph) {
        PFSP_HIP(c, hipGraphLaunch(S->gexec, S->stream));
      } else {
        rc = enqueue_step(c, lb_kind);
        if (rc) return rc;
      }
    }
    PFSP_HIP(c, hipMemcpyAsync(S->ctl_host, S->ctl, sizeof(SearchCtl), hipMemcpyDeviceToHost,
                               S->stream));
    PFSP_HIP(c, hipStreamSynchronize(S->stream));
    const SearchCtl &hc = *S->ctl_host;
    steps = (int)hc.steps;
    const long long held = hc.top + (long long)S->h_d1.size();
    if (held > max_pool) max_pool = held;
    if (hc.overflow) {
      status = set_err(c, PFSP_ENOMEM, "search stack capacity exceeded (raise pool_capacity)");
      break;
    }
    if (budget_nodes > 0 && hc.nodes >= budget_nodes && held > 0) {
      status = PFSP_BUDGET;
      S->resumable = 1;
      break;
    }
    if (hr.on) {
      rc = heur_poll(c, hr, hc);
      if (rc) return rc;
    }
    if (hc.top == 0) {
      if (S->h_d1.empty()) break;
      // the deepest spilled records come back, filling half the room
      const long long x = std::min<long long>((long long)S->h_d1.size(),
                                              std::max<long long>(spill_hi / 2, S->N));
      rc = refill(c, x);
      if (!rc) rc = set_top(c, x);
      if (rc) return rc;
    } else if (spill_hi > S->N && hc.top > spill_hi) {
      const long long x = hc.top - spill_hi / 2;
      rc = spill(c, hc.top, x);
      if (!rc) rc = set_top(c, hc.top - x);
      if (rc) return rc;
    }
  }
  PFSP_HIP(c, hipStreamSynchronize(S->stream));
  PFSP_HIP(c, hipMemcpy(S->ctl_host, S->ctl, sizeof(SearchCtl), hipMemcpyDeviceToHost));
  const SearchCtl hc = *S->ctl_host;
  // the best schedule: the device's best leaf, unless the heuristic threads
  // hold one at least as good (the device incumbent was only lowered to
  // their value, so a device leaf below it is strictly better)
  int best = hc.ub;
  bool from_heur = false;
  if (hr.on) {
    hr.h.finish();
    hr.on = false;
    if (hr.h.best.load() <= best && hr.h.best.load() < ub0) {
      best = hr.h.best.load();
      from_heur = true;
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  res->found = best < ub0;
  res->best_cmax = res->found ? best : ub0;
  res->proven = status == PFSP_OK;
  res->steps = steps;
  res->nodes_decomposed = hc.nodes;
  res->children_bounded = hc.children;
  res->max_pool = max_pool;
  res->seconds = std::chrono::duration<double>(t1 - t0).count();
  if (res->found && res->best_perm) {
    if (from_heur) {
      for (int j = 0; j < n; ++j) res->best_perm[j] = hr.h.best_perm[j];
    } else {
      uint8_t tmp[kMaxN];
      PFSP_HIP(c, hipMemcpy(tmp, S->best_perm, n, hipMemcpyDeviceToHost));
      for (int j = 0; j < n; ++j) res->best_perm[j] = tmp[j];
    }
  }
  return status;
}

static int search_prepare(Ctx *c, int lb_kind, pfsp_result *res) {
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!res) return set_err(c, PFSP_EINVAL, "res is NULL");
  if (lb_kind < PFSP_LB1 || lb_kind > PFSP_LB2_LEARNED)
    return set_err(c, PFSP_EINVAL, "unknown lb_kind");
  if (lb_kind == PFSP_LB2_SUBSET && !c->d_static_mask)
    return set_err(c, PFSP_EINVAL, "PFSP_LB2_SUBSET searches need pfsp_search_set_pairs");
  if (lb_kind != PFSP_LB1 && c->m < 2) return set_err(c, PFSP_ERANGE, "LB2 kinds need m >= 2");
  if (lb_kind != PFSP_LB1 && c->lb1_r > 0 && !c->search_filter)
    return set_err(c, PFSP_EINVAL, "option lb1_r needs search_filter = 1");
  PFSP_HIP(c, hipSetDevice(c->device));
  // the search stream shares the bound workspace with work queued on the ctx stream
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  int rc = search_alloc(c);
  if (rc) return rc;
  if (lb_kind == PFSP_LB2_LEARNED)  // size the selector workspaces before any capture
    rc = learned_prepare(c, c->search->N);
  return rc;
}

}  // namespace pfsp

using namespace pfsp;

extern "C" int pfsp_search(pfsp_ctx *h, int32_t ub0, int64_t budget_nodes, int lb_kind,
                           pfsp_result *res) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (budget_nodes < 0) return set_err(c, PFSP_EINVAL, "negative budget");
  int rc = search_prepare(c, lb_kind, res);
  if (rc) return rc;
  SearchState *S = c->search;
  S->h_perm.clear();
  S->h_d1.clear();
  S->h_d2.clear();
  S->h_lb.clear();
  S->ub0 = ub0;
  S->kind = lb_kind;
  const auto t0 = std::chrono::steady_clock::now();
  hipLaunchKernelGGL(k_init_root, dim3(1), dim3(256), 0, S->stream, S->ctl, c->n, (int)ub0,
                     S->s_perm, S->s_d1, S->s_d2, S->s_lb);
  PFSP_HIP(c, hipGetLastError());
  return run_search(c, lb_kind, ub0, budget_nodes, res, t0);
}

namespace {

struct CkptHeader {
  char magic[8];  // "PFSPCKP1"
  int32_t n, m, kind, ub0, ub, pad;
  uint64_t inst_hash;
  int64_t nodes, children, steps, records;
};

}  // namespace

uint64_t pfsp::instance_hash(const Ctx *c) {  // FNV-1a over n, m and p
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *d, size_t len) {
    const unsigned char *b = (const unsigned char *)d;
    for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&c->n, 4);
  mix(&c->m, 4);
  mix(c->p_host, (size_t)c->n * c->m * 4);
  return h;
}

extern "C" int pfsp_search_dump(pfsp_ctx *h, void *buf, int64_t cap, int64_t *size) {
  if (!h || !size) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  SearchState *S = c->search;
  if (!S || !S->resumable || S->n != c->n)
    return set_err(c, PFSP_EINVAL, "no search stopped on its budget to dump");
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(S->stream));
  PFSP_HIP(c, hipMemcpy(S->ctl_host, S->ctl, sizeof(SearchCtl), hipMemcpyDeviceToHost));
  const SearchCtl hc = *S->ctl_host;
  const int n = c->n;
  const long long hr = (long long)S->h_d1.size(), records = hr + hc.top;
  const int64_t need = (int64_t)sizeof(CkptHeader) + records * (n + 6) + n;
  *size = need;
  if (!buf) return PFSP_OK;
  if (cap < need) return set_err(c, PFSP_ERANGE, "checkpoint buffer too small");
  CkptHeader hd;
  memcpy(hd.magic, "PFSPCKP1", 8);
  hd.n = n;
  hd.m = c->m;
  hd.kind = S->kind;
  hd.ub0 = S->ub0;
  hd.ub = hc.ub;
  hd.pad = 0;
  hd.inst_hash = instance_hash(c);
  hd.nodes = hc.nodes;
  hd.children = hc.children;
  hd.steps = hc.steps;
  hd.records = records;
  unsigned char *o = (unsigned char *)buf;
  memcpy(o, &hd, sizeof(hd));
  o += sizeof(hd);
  // records bottom to top: the host part, then the device stack
  unsigned char *perm = o, *d1 = perm + records * n, *d2 = d1 + records;
  unsigned char *lb = d2 + records;
  if (hr) {
    memcpy(perm, S->h_perm.data(), (size_t)hr * n);
    memcpy(d1, S->h_d1.data(), hr);
    memcpy(d2, S->h_d2.data(), hr);
    memcpy(lb, S->h_lb.data(), (size_t)hr * 4);
  }
  if (hc.top) {
    PFSP_HIP(c, hipMemcpy(perm + hr * n, S->s_perm, (size_t)hc.top * n, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(d1 + hr, S->s_d1, hc.top, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(d2 + hr, S->s_d2, hc.top, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(lb + hr * 4, S->s_lb, (size_t)hc.top * 4, hipMemcpyDeviceToHost));
  }
  PFSP_HIP(c, hipMemcpy(lb + records * 4, S->best_perm, n, hipMemcpyDeviceToHost));
  return PFSP_OK;
}

extern "C" int pfsp_search_resume(pfsp_ctx *h, const void *buf, int64_t size,
                                  int64_t budget_nodes, pfsp_result *res) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (!buf || size < (int64_t)sizeof(CkptHeader))
    return set_err(c, PFSP_EINVAL, "checkpoint too short");
  if (budget_nodes < 0) return set_err(c, PFSP_EINVAL, "negative budget");
  CkptHeader hd;
  memcpy(&hd, buf, sizeof(hd));
  if (memcmp(hd.magic, "PFSPCKP1", 8) != 0) return set_err(c, PFSP_EINVAL, "not a checkpoint");
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (hd.n != c->n || hd.m != c->m || hd.inst_hash != instance_hash(c))
    return set_err(c, PFSP_EINVAL, "checkpoint of another instance");
  const int n = c->n;
  if (hd.records < 0 || size < (int64_t)sizeof(hd) + hd.records * (n + 6) + n)
    return set_err(c, PFSP_EINVAL, "checkpoint truncated");
  int rc = search_prepare(c, hd.kind, res);
  if (rc) return rc;
  SearchState *S = c->search;
  const long long R = hd.records;
  const unsigned char *in = (const unsigned char *)buf + sizeof(hd);
  const unsigned char *perm = in, *d1 = perm + R * n, *d2 = d1 + R, *lb = d2 + R;
  S->h_perm.assign(perm, perm + R * n);
  S->h_d1.assign(d1, d1 + R);
  S->h_d2.assign(d2, d2 + R);
  S->h_lb.resize(R);
  memcpy(S->h_lb.data(), lb, (size_t)R * 4);
  S->ub0 = hd.ub0;
  S->kind = hd.kind;
  const auto t0 = std::chrono::steady_clock::now();
  // the top records onto the device stack, as much as leaves a step's room
  const long long room = std::max<long long>(S->N, S->cap - (long long)S->N * (n > 1 ? n - 1 : 1));
  const long long x = std::min<long long>(R, room);
  if (x) {
    rc = refill(c, x);
    if (rc) return rc;
  }
  SearchCtl hc;
  memset(&hc, 0, sizeof(hc));
  hc.top = (int)x;
  hc.ub = hd.ub;
  hc.ub_step = hd.ub;
  hc.step_best = ~0ull;
  hc.nodes = hd.nodes;
  hc.children = hd.children;
  hc.steps = hd.steps;
  PFSP_HIP(c, hipMemcpy(S->ctl, &hc, sizeof(hc), hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemcpy(S->best_perm, lb + R * 4, n, hipMemcpyHostToDevice));
  return run_search(c, hd.kind, hd.ub0, budget_nodes, res, t0);
}

extern "C" int pfsp_search_log(pfsp_ctx *h, uint8_t *perm_out, uint8_t *d1_out, uint8_t *d2_out,
                               int64_t max_records, int64_t *count) {
  if (!h || !count || max_records < 0) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  SearchState *S = c->search;
  *count = 0;
  if (!S || S->log_cap <= 0) return PFSP_OK;
  if (max_records > 0 && (!perm_out || !d1_out || !d2_out))
    return set_err(c, PFSP_EINVAL, "null output");
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipMemcpyAsync(S->ctl_host, S->ctl, sizeof(SearchCtl), hipMemcpyDeviceToHost,
                             S->stream));
  PFSP_HIP(c, hipStreamSynchronize(S->stream));
  long long k = S->ctl_host->log_count;
  if (k > S->log_cap) k = S->log_cap;
  if (k > max_records) k = max_records;
  if (k > 0) {
    PFSP_HIP(c, hipMemcpy(perm_out, S->l_perm, (size_t)k * S->n, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(d1_out, S->l_d1, (size_t)k, hipMemcpyDeviceToHost));
    PFSP_HIP(c, hipMemcpy(d2_out, S->l_d2, (size_t)k, hipMemcpyDeviceToHost));
  }
  *count = k;
  return PFSP_OK;
}
