/* pfsp.h - C ABI of the MI355X (gfx950) flow-shop bounding library.
 *
 * The library evaluates, on one GPU, the lower bounds of all children of a
 * batch of partial permutation flow-shop schedules, takes the MinMin
 * branching decision and the pruning decision for each parent, and runs a
 * depth-first branch-and-bound built from those steps.  The method is the one
 * of Gmys (2020), "Solving large permutation flow-shop scheduling problems on
 * GPU-accelerated supercomputers":
 *   - problem and makespan recursion:            Section 2.1, Eq. (1)
 *   - nodes (sigma1, sigma2), dynamic branching:  Section 2.3
 *   - MinMin branching heuristic:                 Section 2.3 (Figure 2)
 *   - LB1 (front + remaining + back):             Section 2.4 (Figure 3)
 *   - LB2 (two-machine Johnson bound over machine pairs, pre-sorted orders,
 *     between m and m(m-1)/2 pairs):             Section 2.4
 *   - bounding / pruning / depth-first search:    Sections 2.2, 2.5
 *
 * Conventions shared by every call
 *   - Return value: PFSP_OK (0) on success, a negative PFSP_E* code on error,
 *     PFSP_BUDGET (+1) from pfsp_search when the node budget ran out first.
 *     pfsp_last_error() gives a message for the last failing call on a ctx.
 *   - Processing times are int32 >= 0, row-major p[j*m + k] (job j, machine k).
 *     n in [2, 255], m in [1, 64]; LB2 kinds need m >= 2.  An instance whose
 *     longest possible path (n + m - 1) * max(p) reaches 2^30 is rejected
 *     (PFSP_ERANGE): all bound arithmetic is exact int32 below that limit.
 *   - A node is (perm[n], d1, d2): sigma1 = perm[0, d1), the unscheduled jobs
 *     U = perm[d1, n - d2) in list order, sigma2 = perm[n - d2, n);
 *     d1 + d2 <= n - 1.
 *   - Machine pairs u < v are numbered lexicographically:
 *     idx(u, v) = u*(2m - u - 1)/2 + (v - u - 1), P = m(m-1)/2 pairs.
 *   - Pool and output buffers are DEVICE pointers (e.g. torch tensors on the
 *     ctx's device) owned by the caller; the library never frees them.  Calls
 *     that take device buffers are asynchronous on the ctx stream unless said
 *     otherwise.  The instance is copied into library-owned device memory.
 *   - One ctx per host thread; calls on one ctx must not overlap.
 */
#ifndef PFSP_H
#define PFSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PFSP_OK = 0,
  PFSP_BUDGET = 1,   /* pfsp_search: budget exhausted without a proof */
  PFSP_EINVAL = -1,  /* null pointer, size mismatch, d1 + d2 >= n, bad option */
  PFSP_ENOINST = -2, /* no instance loaded */
  PFSP_ERANGE = -3,  /* n, m, p or a size out of the supported range */
  PFSP_ENOMEM = -4,  /* device or host allocation failed */
  PFSP_EDEVICE = -5  /* a HIP runtime error (message in pfsp_last_error) */
};

typedef enum {
  PFSP_LB1 = 1,         /* one-machine bound (Section 2.4, steps 1-4) */
  PFSP_LB2_FULL = 2,    /* max(LB1, two-machine bound over all P pairs) */
  PFSP_LB2_SUBSET = 3,  /* max(LB1, two-machine bound over the pairs in pair_mask) */
  PFSP_LB2_LEARNED = 4  /* subset chosen per parent by the loaded pair selector */
} pfsp_lb_kind;

typedef struct pfsp_ctx pfsp_ctx;

/* A batch of parent nodes, structure-of-arrays, all device pointers. */
typedef struct {
  int32_t count;              /* number of parents N >= 0 */
  int32_t n;                  /* row stride of perm; must equal the loaded n */
  const uint8_t *perm;        /* [N][n] job ids 0..n-1, each row a permutation */
  const uint8_t *d1;          /* [N] prefix lengths */
  const uint8_t *d2;          /* [N] suffix lengths */
  const uint32_t *pair_mask;  /* PFSP_LB2_SUBSET: [N][mask_words], bit idx(u,v)
                                 selects pair (u, v); otherwise ignored */
  int32_t mask_words;         /* words per row of pair_mask, >= ceil(P / 32) */
  uint8_t *dir_out;           /* [N] or NULL: MinMin choice, 0 = forward, 1 = backward */
  int16_t *argpair_out;       /* [N][2][n] or NULL (LB2 kinds): lowest pair index
                                 attaining each child's pair maximum, -1 if none */
} pfsp_pool;

typedef struct {
  int32_t best_cmax;          /* best makespan found (< ub0) if found, else ub0 */
  int32_t found;              /* 1 iff a schedule with C_max < ub0 was found */
  int32_t proven;             /* 1 iff the tree was exhausted (optimal if found,
                                 otherwise the optimum is >= ub0) */
  int32_t steps;              /* batch steps executed */
  int64_t nodes_decomposed;   /* decomposed nodes, root included */
  int64_t children_bounded;   /* sum over decomposed nodes of 2(n - d) */
  int64_t max_pool;           /* largest pool size seen at a poll */
  double seconds;             /* wall time of the search loop */
  int32_t *best_perm;         /* caller-owned HOST [n], filled when found */
} pfsp_result;

/* Creates a context on HIP device `device`.  hip_stream is a hipStream_t
 * (NULL = the device's null stream) on which every kernel is launched.
 * *out receives the context; it owns all library device memory. */
int pfsp_create(pfsp_ctx **out, int device, void *hip_stream);

/* Releases a context and its device memory (waits for its stream first). */
void pfsp_destroy(pfsp_ctx *c);

/* Message of the last failing call on c (static text if c is NULL). */
const char *pfsp_last_error(pfsp_ctx *c);

/* Loads an instance from HOST memory p[n*m] (Section 2.1) and stages its
 * device tables: per-machine totals, and for every machine pair the
 * Johnson-with-lags order of all n jobs with their (a, b, lag) times
 * (Section 2.4: LB2 uses pre-sorted two-machine schedules).  Synchronous. */
int pfsp_load_instance(pfsp_ctx *c, int32_t n, int32_t m, const int32_t *p);

/* Number of machine pairs P = m(m-1)/2 of the loaded instance, or < 0. */
int pfsp_pair_count(pfsp_ctx *c);

/* Decomposition of every parent of the pool (Section 2.3, Figure 2; Section
 * 2.2 bounding and pruning): both children sets are bounded with `lb_kind`,
 * MinMin chooses the direction, and a child is flagged pruned iff LB >= ub.
 * out_lb [N][2][n] int32 and out_prune [N][2][n] uint8 (device): entry
 * [i][dir][q] is the child of parent i that puts the job perm[i][d1 + q] at
 * the end of sigma1 (dir 0) or the front of sigma2 (dir 1); slots q >= n-d1-d2
 * hold INT32_MAX and prune 1.  A leaf child's LB is its makespan.
 * Asynchronous on the ctx stream.  A row that is not a valid node (d1 + d2 >=
 * n, or perm not a permutation of 0..n-1) gets INT32_MAX / prune 1 in every
 * slot and dir 0, and makes the next pfsp_check report PFSP_EINVAL. */
int pfsp_bound_children(pfsp_ctx *c, const pfsp_pool *pool, int lb_kind, int32_t ub,
                        int32_t *out_lb, uint8_t *out_prune);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * decomposition as pfsp_bound_children for lb_kind PFSP_LB1, PFSP_LB2_FULL or
 * PFSP_LB2_SUBSET, with the per-parent workspace (front, back and remaining
 * loads, 3m int32 per parent) taken from a fixed 64 MiB device array that
 * each GPU holds from the library's load until the process ends, instead of
 * a workspace grown with hipMalloc.  The call allocates nothing (no
 * hipMalloc, hipFree, events or library allocations); the caller still
 * passes the pool and the outputs.  PFSP_ERANGE if count * 3m exceeds 2^24
 * (e.g. 279,620 parents at m = 20); PFSP_EINVAL for PFSP_LB2_LEARNED.  Every
 * call on a GPU
 * uses that GPU's one array: calls whose work overlaps on one GPU (other
 * contexts, other streams) race; calls queued on one stream are ordered.
 * No kernel-time instrumentation.  Asynchronous on the ctx stream. */
int pfsp_bound_children_noalloc(pfsp_ctx *c, const pfsp_pool *pool, int lb_kind, int32_t ub,
                                int32_t *out_lb, uint8_t *out_prune);

/* Waits for the ctx stream and reports PFSP_EINVAL if any pool row seen by
 * pfsp_bound_children since the last check had d1 + d2 >= n (such rows are
 * filled with INT32_MAX / prune 1).  Clears the condition.  Synchronous. */
int pfsp_check(pfsp_ctx *c);

/* Fixed LB2 pair variants (Section 2.4: LB2 variants evaluate between m and
 * m(m-1)/2 two-machine schedules per child).  Writes to HOST mask_out[words]
 * (words >= ceil(P/32)) the bit mask over the loaded instance's pair indices
 * of PFSP_PAIRS_ADJACENT, the m - 1 pairs (k, k + 1), or PFSP_PAIRS_LAST, the
 * m - 1 pairs (k, m - 1).  Host only. */
enum { PFSP_PAIRS_ADJACENT = 1, PFSP_PAIRS_LAST = 2 };
int pfsp_pair_mask(pfsp_ctx *c, int variant, uint32_t *mask_out, int32_t words);

/* The pair set (HOST mask[words], words >= ceil(P/32), bits over the
 * instance's pair indices) with which pfsp_search bounds every node when
 * called with PFSP_LB2_SUBSET: LB = max(LB1, maximum over the set).  Kept
 * until the next pfsp_load_instance.  Synchronous. */
int pfsp_search_set_pairs(pfsp_ctx *c, const uint32_t *mask, int32_t words);

/* Depth-first branch-and-bound on the device (Sections 2.2-2.5) from the
 * root (empty sigma1, sigma2): pools of up to `pool_batch` (option) nodes are
 * popped from a device stack, decomposed with pfsp_bound_children's step,
 * and their surviving children pushed back (leftmost on top); when the stack
 * nears its capacity its bottom (shallowest) records move to host memory and
 * come back once the stack above them has drained.  Looks for a
 * schedule with C_max < ub0 (INT32_MAX: none known).  budget_nodes > 0 stops
 * after about that many decomposed nodes (returns PFSP_BUDGET).  lb_kind as
 * above; PFSP_LB2_SUBSET takes the pair set of pfsp_search_set_pairs for
 * every node.  Waits for the ctx stream first (the search
 * runs on a stream of its own and shares the bound workspace).  Synchronous;
 * res must not be NULL. */
int pfsp_search(pfsp_ctx *c, int32_t ub0, int64_t budget_nodes, int lb_kind,
                pfsp_result *res);

/* Checkpoint of a search that stopped on its node budget (pfsp_search or
 * pfsp_search_resume returned PFSP_BUDGET), for restarting it later, in this
 * process or another, on the same instance (the paper's global checkpoints of
 * Section 4.1, here for one GPU): the open nodes (device stack and any part
 * moved to host memory), the incumbent and best schedule, ub0, the bound
 * kind and the node counters, in a self-describing byte format.  buf NULL:
 * *size receives the bytes needed.  PFSP_ERANGE if cap is smaller.  HOST
 * buffer; synchronous. */
int pfsp_search_dump(pfsp_ctx *c, void *buf, int64_t cap, int64_t *size);

/* Continues the search of a checkpoint (HOST buf[size]) on the loaded
 * instance (PFSP_EINVAL if it is another one) with the checkpoint's bound
 * kind and ub0, under the current options, until the tree is exhausted or
 * budget_nodes (counted from the first start) is reached.  The result counts
 * the nodes of every run since the first start.  Synchronous. */
int pfsp_search_resume(pfsp_ctx *c, const void *buf, int64_t size, int64_t budget_nodes,
                       pfsp_result *res);

/* Depth-first search by `explorers` (a power of 4, at most 4^10)
 * integer-vector-matrix explorers (Section 2.5) on the device, for n <= 64:
 * each explorer owns a work unit, an interval of the factorial-number-system
 * numbering of the n! schedules (Section 2.6), explores it depth first, and
 * every "poll_every" steps, when fewer than 80 % of the explorers held work,
 * the empty ones steal the right half of a busy neighbour's interval on a
 * 4-ary hypercube (Section 3.4: a victim is taken once per phase and must
 * hold more than the average and a minimum length).  Each step bounds every explorer's current node with
 * the kernels of pfsp_bound_children (lb_kind PFSP_LB1 or PFSP_LB2_FULL).
 * Same result and node semantics as pfsp_search (a node re-decomposed by a
 * thief on the way to its interval is not counted again); *steals (HOST, may
 * be NULL) receives the number of work units stolen.  A search stopped on
 * its budget can be dumped (pfsp_search_ivm_dump) and resumed.  Synchronous. */
int pfsp_search_ivm(pfsp_ctx *c, int32_t ub0, int64_t budget_nodes, int lb_kind,
                    int32_t explorers, pfsp_result *res, int64_t *steals);

/* Checkpoint of the last pfsp_search_ivm or pfsp_search_ivm_resume that
 * stopped on its node budget (Section 4.1 checkpoints the explorers' work
 * units; this one holds every explorer's whole state: interval, position,
 * matrix rows, prune bits and stored bounds, so that a resumed search
 * decomposes and counts every node once), with the incumbent, best schedule,
 * ub0, bound kind, explorer count and counters.  Same two-call protocol as
 * pfsp_search_dump (buf NULL: *size receives the bytes needed; PFSP_ERANGE if
 * cap is smaller; PFSP_EINVAL if there is no such search).  About
 * K n (5 n + 10) bytes for K explorers.  HOST buffer; synchronous. */
int pfsp_search_ivm_dump(pfsp_ctx *c, void *buf, int64_t cap, int64_t *size);

/* Continues an IVM checkpoint (HOST buf[size]) on the loaded instance
 * (PFSP_EINVAL if it is another one or the bytes are malformed) with its
 * explorer count, bound kind and ub0, under the current options, until the
 * tree is exhausted or budget_nodes (counted from the first start) is
 * reached; res and *steals count every run since the first start.
 * Synchronous. */
int pfsp_search_ivm_resume(pfsp_ctx *c, const void *buf, int64_t size, int64_t budget_nodes,
                           pfsp_result *res, int64_t *steals);

/* Work-unit arithmetic of the IVM search on HOST digit vectors (factorial
 * number system, Section 2.6): a position in [0, n!] is digits d[0 .. n),
 * digit L in [0, n - L) with weight (n - 1 - L)!, plus a top digit (1 only
 * for n! itself).  op 0: a + b; op 1: b - a (b >= a); op 2: floor(a / 2);
 * op 3: a + (b - a) / 2, the split point of a work unit [a, b).  Writes
 * out[n] and *out_top.  n in [1, 64].  Needs no device. */
int pfsp_factoradic(int op, int32_t n, const uint8_t *a, int32_t atop, const uint8_t *b,
                    int32_t btop, uint8_t *out, int32_t *out_top);

/* The node an IVM designates (Section 2.5): HOST M[n][n] (row L: the jobs
 * schedulable at level L, n - L of them), V[level + 1] (chosen cell per row),
 * D[level + 1] (0: front of sigma1, 1: front of sigma2), level >= 0; writes
 * perm_out[n] (sigma1 | unscheduled in row order | sigma2), *d1, *d2.  Needs
 * no device. */
int pfsp_ivm_decode(int32_t n, const uint8_t *M, const uint8_t *V, const uint8_t *D,
                    int32_t level, uint8_t *perm_out, int32_t *d1, int32_t *d2);

/* Copies up to max_records nodes decomposed by the last pfsp_search (every
 * log_stride-th node of each batch, at most log_capacity; option names above)
 * to HOST perm_out[max_records][n], d1_out, d2_out; *count receives the number
 * copied.  Synchronous. */
int pfsp_search_log(pfsp_ctx *c, uint8_t *perm_out, uint8_t *d1_out, uint8_t *d2_out,
                    int64_t max_records, int64_t *count);

/* Nawaz-Enscore-Ham constructive heuristic on the loaded instance, used for
 * the initial incumbent: jobs by decreasing total time (ties: lower id), each
 * inserted at the first position minimising the partial makespan.  HOST
 * outputs perm_out[n] and *cmax_out.  Synchronous. */
int pfsp_neh(pfsp_ctx *c, int32_t *perm_out, int32_t *cmax_out);

/* Integer options: "pool_batch" (nodes popped per search step, default
 * 65536), "poll_every" (search steps between host polls, default 8),
 * "pool_capacity" (max stacked nodes, default derived from n and pool_batch),
 * "use_graph" (1 = replay the search step as a HIP graph, default 1),
 * "learned_topk" (pairs kept by the selector, default 16; at most 32 with
 * the float selector, 64 with the integer one),
 * "learned_exact" (1 = PFSP_LB2_LEARNED bounds every parent that keeps a
 * child under the selected pairs again with all pairs: the prune flags, and a
 * search's tree, are those of PFSP_LB2_FULL, and so are the bounds and MinMin
 * choice of those parents; a parent whose children the subset prunes
 * entirely keeps the subset's values; default 0),
 * "timing" (1 = bracket every kernel launch with HIP events on the ctx
 * stream, default 0), "lb2_waves" (waves per block of the LB2 kernel, 0..16, 0 =
 * automatic; larger values than a kernel's launch bounds allow are ignored), "lb2_blocks_per_cu" (cap on LB2 blocks per CU, 0 = twice
 * the blocks that fit a CU's LDS for the n <= 32 and subset kernels, 16 for
 * the others),
 * "force_generic" (1 = always use the generic LB2 kernel),
 * "search_filter" (1 = LB2 search steps close every parent whose children
 * all have LB1 >= incumbent in the costs kernel and bound only the others
 * with LB2; the tree is unchanged since LB2 >= LB1; default 1),
 * "subset_group" (parents per wave of subset LB2 for n <= 64 when every
 * stored value fits 16 bits: 2 or 4, each parent then gets 32 or 16 lanes
 * and a selection of up to that many pairs costs one scan pass; 0 = one
 * parent per wave for PFSP_LB2_SUBSET in pfsp_bound_children, and by the
 * number of selected pairs k in searches and for PFSP_LB2_LEARNED: four
 * parents per wave for k <= 16 when 32 < n <= 64, else two for k <= 32),
 * "deep_r" (PFSP_LB2_FULL for n <= 32 with (n + m) max p < 2^15: parents
 * with at most deep_r unscheduled jobs take a kernel that scans only their
 * jobs' positions in each pair's Johnson order, the others the full-scan
 * kernel; 0 = every parent takes the full scan; at most 16; default 8),
 * "lb1_r" (pfsp_search with an LB2 kind: the bound chosen by depth, Section
 * 2.4 ranking LB1 as the cheaper, weaker bound; a popped parent with at most
 * lb1_r unscheduled jobs has its children bounded with LB1, the others with
 * the search's kind; the optimum is unchanged, the tree may grow; needs
 * search_filter = 1 (else pfsp_search returns PFSP_EINVAL); 0..255, default
 * 0 = off; the IVM search ignores it),
 * "heuristic_threads" (host threads that run an iterated greedy local search
 * on the instance while pfsp_search runs, seeded with NEH and with schedules
 * completed from open nodes; a better makespan lowers the device incumbent
 * at the next poll, and the search returns the better of the device's and
 * the threads' schedules; the optimum is unchanged, node counts then depend
 * on timing; default 0 = off), "heuristic_seed" (their random seed),
 * "wide_lb2" (1 = PFSP_LB2_FULL for 32 < n <= 128 with (n + m) max p < 2^15
 * runs the wide kernel, whose entries are staged at pfsp_load_instance;
 * default 1), "log_capacity" (records kept by pfsp_search's node log,
 * 0 = off) and "log_stride" (log every log_stride-th decomposed node of a
 * batch). */
int pfsp_set_option(pfsp_ctx *c, const char *key, int64_t value);
int pfsp_get_option(pfsp_ctx *c, const char *key, int64_t *value);

/* Autotuner for the single-instance LB2 kernels: times pfsp_bound_children on
 * this pool (DEVICE buffers as there) for every candidate of options
 * "lb2_waves" (0,1,2,3,4,6,8,12,16) and "lb2_blocks_per_cu" (0,2,4,8,16,32), median
 * of reps runs each, sets the fastest pair on the context and writes a JSON
 * summary to report (HOST, report_len bytes).  Synchronous. */
int pfsp_autotune(pfsp_ctx *c, const pfsp_pool *pool, int lb_kind, int32_t ub, int32_t *out_lb,
                  uint8_t *out_prune, int32_t reps, char *report, int32_t report_len);

/* Instrumentation (option "timing" = 1): total milliseconds and number of
 * launches of the kernel named `kernel` ("k_lb1", "k_lb2", ...) since the last
 * reset, measured with HIP events recorded on the ctx stream around each
 * launch.  Waits for the ctx stream.  reset != 0 clears all counters after
 * reading. */
int pfsp_kernel_time(pfsp_ctx *c, const char *kernel, double *total_ms, int64_t *launches,
                     int reset);

/* ------------------------------------------------------------------------
 * Several instances of different (n, m) bounded together.  Parents of all
 * instances share one DEVICE pool whose rows have a common stride (>= every
 * n used); the parents of instance k are rows [seg_begin[k], seg_begin[k+1]).
 * Outputs use the same stride: out_lb/out_prune [N][2][stride], slots
 * q >= n - d1 - d2 hold INT32_MAX / prune 1.  The launch sequence (one costs
 * kernel, one persistent LB2 kernel per instance class draining a queue of
 * instance tiles: n <= 20; 20 < n <= 128 with (n + m) max p < 2^15 (the wide
 * kernel, unless "wide_lb2" was 0 at pfsp_multi_create); other n <= 64;
 * generic kernels for the rest) is captured as a
 * HIP graph on first use and replayed while buffers and grouping are
 * unchanged.
 * ------------------------------------------------------------------------ */
typedef struct pfsp_multi pfsp_multi;

/* Stages `count` instances (HOST p[k][n[k]*m[k]]) for batched bounding. */
int pfsp_multi_create(pfsp_ctx *c, int32_t count, const int32_t *n, const int32_t *m,
                      const int32_t *const *p, pfsp_multi **out);

void pfsp_multi_destroy(pfsp_multi *mt);

/* Decomposition of every parent (as pfsp_bound_children, lb_kind PFSP_LB1 or
 * PFSP_LB2_FULL) with incumbent ub[k] (HOST [count]) for instance k;
 * seg_begin is HOST [count + 1] with seg_begin[0] = 0.  Waits for the ctx
 * stream first (the pool may be written there).  Synchronous. */
int pfsp_multi_bound(pfsp_multi *mt, int lb_kind, const uint8_t *perm, const uint8_t *d1,
                     const uint8_t *d2, int32_t stride, const int64_t *seg_begin,
                     const int32_t *ub, int32_t *out_lb, uint8_t *out_prune, uint8_t *dir_out);

/* Launch shape: parents per tile, waves per block of the n <= 20 class (0..16; 16 only
 * when all its instances allow 16-bit X, else at most 12) and of the
 * larger classes (0..8, at most 4 for the n > 64 wide class; 0 = most resident waves),
 * blocks per CU (0 = as many as fit). */
int pfsp_multi_set_shape(pfsp_multi *mt, int32_t tile, int32_t waves_small, int32_t waves_large,
                         int32_t blocks_per_cu);

/* Autotuner: runs pfsp_multi_bound's launch for every candidate shape (tile
 * 64..1024, waves 0/2/4/8/12/16, blocks per CU 0/2/4/8) on this batch, keeps the
 * fastest (median of reps replays) and writes a JSON summary to report. */
int pfsp_multi_autotune(pfsp_multi *mt, int lb_kind, const uint8_t *perm, const uint8_t *d1,
                        const uint8_t *d2, int32_t stride, const int64_t *seg_begin,
                        const int32_t *ub, int32_t *out_lb, uint8_t *out_prune, uint8_t *dir_out,
                        int32_t reps, char *report, int32_t report_len);

/* ------------------------------------------------------------------------
 * Learned machine-pair selector (PFSP_LB2_LEARNED).  Section 2.4 allows LB2
 * variants over any number of machine pairs between m and m(m-1)/2; the
 * maximum over any subset still bounds from below.  The selector scores the
 * 190 pairs of a 20-machine layout from 64 features of a parent node with an
 * MLP 64 -> 64 -> 64 -> 190 (ReLU, weights rounded to bfloat16, fp32
 * accumulation); the `learned_topk` best pairs present on the instance (m <= 20)
 * are bounded exactly.  The float form runs on bf16 matrix cores: each fp32
 * activation enters as bf16(x) plus bf16(x - bf16(x)) (about 16 bits of it),
 * sums are fp32, and pairs rank by a key of the score's leading 24 bits
 * (order-preserving integer form), equal keys to the lower layout index.
 * Parameter layout (fp32, 20670 values): W1[64][64],
 * b1[64], W2[64][64], b2[64], W3[190][64], b3[190]; W[o][i] maps input i to
 * output o.  Layout pair of machines u < v: u*(39 - u)/2 + (v - u - 1).
 * Features of a parent (norm = largest machine load of the instance):
 * [0,20) C1[k]/norm, [20,40) C2[k]/norm, [40,60) R[k]/norm (k < min(m,20),
 * zero beyond), d1/n, d2/n, (n-d1-d2)/n, LB1(parent)/norm.
 * ------------------------------------------------------------------------ */

/* Sets the fp32 master parameters from HOST memory and resets the optimiser. */
int pfsp_selector_set(pfsp_ctx *c, const float *params, int64_t count);

/* Copies the fp32 master parameters to HOST memory (synchronous). */
int pfsp_selector_get(pfsp_ctx *c, float *params, int64_t count);

/* Features of every parent of the pool into DEVICE feat_out[N][64]. */
int pfsp_selector_features(pfsp_ctx *c, const pfsp_pool *pool, float *feat_out);

/* Scores DEVICE x[rows][64] -> DEVICE scores_out[rows][190] with the float
 * form's arithmetic of the learned bound (layout pairs not present on the
 * loaded instance get -inf). */
int pfsp_selector_forward(pfsp_ctx *c, const float *x, int32_t rows, float *scores_out);

/* Top-k (k in [1, 32]) of DEVICE scores[rows][190] (larger first, ties to the
 * lower layout index) as DEVICE bit masks mask_out[rows][ceil(P/32)] over the
 * instance's pair indices, the pair_mask format of PFSP_LB2_SUBSET. */
int pfsp_selector_select(pfsp_ctx *c, const float *scores, int32_t rows, int32_t k,
                         uint32_t *mask_out);

/* Integer-only deployment of the selector.  With these parameters set,
 * PFSP_LB2_LEARNED ranks pairs with an int8 form of the MLP whose sums are
 * exact integers (int8 weights and activations, int32 accumulation):
 *   features  xq[j] = clamp(rint(float(c) * q), 0, 127), c the numerator of
 *             feature j above (C1, C2, R, LB1 with q = sx / norm; d1, d2,
 *             n - d1 - d2 with q = sx / n; float32 products; zero for absent
 *             machines and invalid rows);
 *   hidden    a = b + W xq (int32), h = min(127, (max(a, 0) * M + 2^(S-1)) >> S),
 *             M in [1, 1023], S in [1, 30], per hidden layer;
 *   scores    s = b3 + W3 h2 (int32); the k largest among present pairs, ties
 *             to the lower layout index.
 * blob (HOST int32, 20675 values): sx (float32 bits), M1, S1, M2, S2,
 * W1[64][64], b1[64], W2[64][64], b2[64], W3[190][64], b3[190]; weights in
 * [-127, 127], biases in (-2^19, 2^19) (else PFSP_ERANGE).  blob = NULL
 * returns to the float model.  Synchronous. */
int pfsp_selector_set_quant(pfsp_ctx *c, const int32_t *blob, int64_t count);

/* Pair masks that PFSP_LB2_LEARNED would bound for every parent of the pool
 * (the integer model if set, k in [1, 64], else the float model, k in
 * [1, 32]): DEVICE
 * mask_out[N][ceil(P/32)] over the instance's pair indices. */
int pfsp_selector_infer(pfsp_ctx *c, const pfsp_pool *pool, int32_t k, uint32_t *mask_out);

/* Training targets from argpair_out of an LB2_FULL pfsp_bound_children call on
 * the same pool: DEVICE target_out[N][190] = share of the parent's 2(n-d)
 * children whose LB2 is attained first by each layout pair (all zero if none).
 * Synchronous. */
int pfsp_selector_targets(pfsp_ctx *c, const pfsp_pool *pool, const int16_t *argpair,
                          float *target_out);

/* One training step on DEVICE x[rows][64] and targets[rows][190]: mean soft-
 * target cross-entropy over rows with a non-empty target (masked softmax over
 * present pairs), gradients by backpropagation through the bf16-rounded
 * weights (forward and backward passes and the weight gradients as bf16
 * matrix-core products with fp32 sums, activations and errors entering as
 * bf16 hi + lo pairs; the gradient sums over the rows run in a fixed order),
 * then one Adam step (beta 0.9/0.999, eps 1e-8) of size lr on the master
 * parameters if lr > 0.  *loss_out (HOST, may be NULL) receives the loss
 * before the update; grad_out (DEVICE [20670], may be NULL) the gradient.
 * Synchronous. */
int pfsp_selector_train_step(pfsp_ctx *c, const float *x, const float *target, int32_t rows,
                             float lr, float *loss_out, float *grad_out);

#ifdef __cplusplus
}
#endif
#endif /* PFSP_H */
