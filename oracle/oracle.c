/* Plain CPU oracle for the permutation flow-shop (PFSP) bounds and depth-first
 * branch-and-bound of Gmys (2020), "Solving large permutation flow-shop
 * scheduling problems on GPU-accelerated supercomputers".
 *
 * TEST INFRASTRUCTURE ONLY.  It is loaded by the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark, never by the product path, and it
 * shares no code with the HIP library.  Every quantity is recomputed from its
 * definition for every node (no incremental evaluation, no pre-sorted tables),
 * in 64-bit integers, so that it can be checked against the paper by eye.
 */
#include "oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

#define P_(p, m, j, k) ((int64_t)(p)[(size_t)(j) * (size_t)(m) + (size_t)(k)])
#define MAXN 256
#define MAXM 64

static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* Section 2.1, Eq. (1): completion times of a job sequence, zero at the
 * borders.  Fills C[k] = completion time of the last job of seq on machine k
 * (all zero for an empty sequence). */
void or_front(int m, const int32_t *p, const uint8_t *seq, int len, int64_t *C) {
  for (int k = 0; k < m; ++k) C[k] = 0;
  for (int i = 0; i < len; ++i) {
    int j = seq[i];
    C[0] += P_(p, m, j, 0);
    for (int k = 1; k < m; ++k) C[k] = max64(C[k], C[k - 1]) + P_(p, m, j, k);
  }
}

/* Section 2.1: the makespan C_max = C[last job, last machine] of Eq. (1). */
int64_t or_makespan(int m, const int32_t *p, const uint8_t *seq, int len) {
  int64_t C[MAXM];
  or_front(m, p, seq, len, C);
  return C[m - 1];
}

/* Section 2.4, step 3: the back times of a suffix sigma2.  Cb[k] is the least
 * time between the start of sigma2's first job on machine k and the end of
 * the last operation; it is Eq. (1) applied to sigma2 in reverse job order on
 * the machines taken in reverse order (reversibility of the PFSP). */
void or_back(int m, const int32_t *p, const uint8_t *seq, int len, int64_t *Cb) {
  for (int k = 0; k < m; ++k) Cb[k] = 0;
  for (int i = len - 1; i >= 0; --i) {
    int j = seq[i];
    Cb[m - 1] += P_(p, m, j, m - 1);
    for (int k = m - 2; k >= 0; --k) Cb[k] = max64(Cb[k], Cb[k + 1]) + P_(p, m, j, k);
  }
}

/* Section 2.4, step 4: LB1 = max over machines k of front + remaining + back. */
int64_t or_lb1_parts(int m, const int64_t *C1, const int64_t *R, const int64_t *C2) {
  int64_t lb = C1[0] + R[0] + C2[0];
  for (int k = 1; k < m; ++k) lb = max64(lb, C1[k] + R[k] + C2[k]);
  return lb;
}

/* Time lag between machines u < v for job j: the processing on the machines
 * strictly between them, which the two-machine relaxation treats as
 * non-bottleneck (capacity unbounded). */
static int64_t lag(int m, const int32_t *p, int j, int u, int v) {
  int64_t s = 0;
  for (int q = u + 1; q < v; ++q) s += P_(p, m, j, q);
  return s;
}

/* Johnson's rule (Section 2.1 cites it for m = 2), extended to time lags as
 * used by the two-machine bound of Lageweg et al. (1978), which Section 2.4
 * names as LB2: the jobs with a_j <= b_j come first in ascending order of
 * a_j + l_j, then the others in descending order of b_j + l_j; equal keys keep
 * ascending job id.  a_j = p[j][u], b_j = p[j][v], l_j = lag(j, u, v).
 * Sorts `jobs` in place (insertion sort). */
static int johnson_before(int m, const int32_t *p, int x, int y, int u, int v) {
  int64_t ax = P_(p, m, x, u), bx = P_(p, m, x, v), lx = lag(m, p, x, u, v);
  int64_t ay = P_(p, m, y, u), by = P_(p, m, y, v), ly = lag(m, p, y, u, v);
  int sx = ax <= bx ? 0 : 1, sy = ay <= by ? 0 : 1;
  if (sx != sy) return sx < sy;
  if (sx == 0) {
    if (ax + lx != ay + ly) return ax + lx < ay + ly;
  } else {
    if (bx + lx != by + ly) return bx + lx > by + ly;
  }
  return x < y;
}

void or_johnson_lag_order(int m, const int32_t *p, uint8_t *jobs, int nj, int u, int v) {
  for (int i = 1; i < nj; ++i) {
    uint8_t x = jobs[i];
    int k = i - 1;
    while (k >= 0 && johnson_before(m, p, x, jobs[k], u, v)) {
      jobs[k + 1] = jobs[k];
      --k;
    }
    jobs[k + 1] = x;
  }
}

/* Two-machine evaluation of a fixed job order on machines u, v with heads
 * (hu, hv) and tails (tu, tv):  t_u advances by a_j; t_v waits for
 * t_u + l_j then advances by b_j; the value is max(t_u + tail_u, t_v + tail_v). */
static int64_t pair_eval(int m, const int32_t *p, const uint8_t *order, int nj, int u, int v,
                         int64_t hu, int64_t hv, int64_t tu, int64_t tv) {
  int64_t a = hu, b = hv;
  for (int i = 0; i < nj; ++i) {
    int j = order[i];
    a += P_(p, m, j, u);
    b = max64(b, a + lag(m, p, j, u, v)) + P_(p, m, j, v);
  }
  return max64(a + tu, b + tv);
}

/* Section 2.4 (LB2): the two-machine bound for one machine pair, solved
 * exactly by sorting the unscheduled jobs with Johnson's rule for lags. */
int64_t or_pair_value(int m, const int32_t *p, const uint8_t *jobs, int nj, int u, int v,
                      int64_t hu, int64_t hv, int64_t tu, int64_t tv) {
  uint8_t ord[MAXN];
  memcpy(ord, jobs, (size_t)nj);
  or_johnson_lag_order(m, p, ord, nj, u, v);
  return pair_eval(m, p, ord, nj, u, v, hu, hv, tu, tv);
}

/* Lexicographic next permutation of a byte array; returns 0 after the last. */
static int next_perm(uint8_t *a, int len) {
  int i = len - 2;
  while (i >= 0 && a[i] >= a[i + 1]) --i;
  if (i < 0) return 0;
  int j = len - 1;
  while (a[j] <= a[i]) --j;
  uint8_t t = a[i]; a[i] = a[j]; a[j] = t;
  for (int x = i + 1, y = len - 1; x < y; ++x, --y) { t = a[x]; a[x] = a[y]; a[y] = t; }
  return 1;
}

static int cmp_u8(const void *x, const void *y) {
  return (int)*(const uint8_t *)x - (int)*(const uint8_t *)y;
}

/* Brute force of the same two-machine problem over every order of `jobs`. */
int64_t or_pair_value_bruteforce(int m, const int32_t *p, const uint8_t *jobs, int nj,
                                 int u, int v, int64_t hu, int64_t hv, int64_t tu,
                                 int64_t tv) {
  uint8_t ord[MAXN];
  memcpy(ord, jobs, (size_t)nj);
  qsort(ord, (size_t)nj, 1, cmp_u8);
  int64_t best = INT64_MAX;
  do {
    int64_t x = pair_eval(m, p, ord, nj, u, v, hu, hv, tu, tv);
    if (x < best) best = x;
  } while (next_perm(ord, nj));
  return best;
}

static int pair_index(int m, int u, int v) { return u * (2 * m - u - 1) / 2 + (v - u - 1); }

/* Lower bound of one node (sigma1 = perm[0,d1), U = perm[d1,n-d2),
 * sigma2 = perm[n-d2,n)), all parts recomputed from scratch:
 *  - LB1 (Section 2.4, steps 1-4);
 *  - LB2 (Section 2.4): max over the machine pairs u < v (all of them, or the
 *    pairs whose bit is set in pair_mask) of the two-machine bound with heads
 *    C1[u], C1[v] and tails C2[u], C2[v]; the returned value is max(LB1, LB2).
 * If argpair is given it receives the lowest index of a pair whose
 * two-machine bound exceeds LB1 and attains the returned value, or -1 when
 * the value equals LB1 (no pair is needed to reach it) or no pair is
 * evaluated. */
int64_t or_node_bound(int n, int m, const int32_t *p, const uint8_t *perm, int d1, int d2,
                      int kind, const uint32_t *pair_mask, int32_t *argpair) {
  int64_t C1[MAXM], C2[MAXM], R[MAXM];
  int r = n - d1 - d2;
  const uint8_t *U = perm + d1;
  or_front(m, p, perm, d1, C1);
  or_back(m, p, perm + (n - d2), d2, C2);
  for (int k = 0; k < m; ++k) {
    R[k] = 0;
    for (int i = 0; i < r; ++i) R[k] += P_(p, m, U[i], k);
  }
  int64_t lb = or_lb1_parts(m, C1, R, C2);
  if (argpair) *argpair = -1;
  if (kind == OR_LB1) return lb;
  int64_t best = INT64_MIN;
  for (int u = 0; u < m; ++u)
    for (int v = u + 1; v < m; ++v) {
      int pi = pair_index(m, u, v);
      if (kind == OR_LB2_SUBSET && !(pair_mask[pi >> 5] >> (pi & 31) & 1u)) continue;
      int64_t x = or_pair_value(m, p, U, r, u, v, C1[u], C1[v], C2[u], C2[v]);
      if (x > best) {
        best = x;
        if (argpair) *argpair = pi;
      }
    }
  if (argpair && best <= lb) *argpair = -1;
  return max64(lb, best);
}

/* Best completion of a node by enumerating every order of its unscheduled
 * jobs (exponential; tiny nodes only). */
int64_t or_best_completion(int n, int m, const int32_t *p, const uint8_t *perm, int d1,
                           int d2, uint8_t *best_perm) {
  uint8_t s[MAXN];
  int r = n - d1 - d2;
  memcpy(s, perm, (size_t)n);
  qsort(s + d1, (size_t)r, 1, cmp_u8);
  int64_t best = INT64_MAX;
  do {
    int64_t c = or_makespan(m, p, s, n);
    if (c < best) {
      best = c;
      if (best_perm) memcpy(best_perm, s, (size_t)n);
    }
  } while (next_perm(s + d1, r));
  return best;
}

/* Section 2.3, MinMin: keep the children set in which the smallest LB over
 * both sets occurs fewer times; on equal counts the set with the larger LB
 * sum; forward if the sums are equal too.  Returns 0 = forward, 1 = backward. */
int or_minmin(int r, const int64_t *lbf, const int64_t *lbb) {
  int64_t mn = INT64_MAX, sf = 0, sb = 0;
  int cf = 0, cb = 0;
  for (int q = 0; q < r; ++q) {
    if (lbf[q] < mn) mn = lbf[q];
    if (lbb[q] < mn) mn = lbb[q];
  }
  for (int q = 0; q < r; ++q) {
    cf += lbf[q] == mn;
    cb += lbb[q] == mn;
    sf += lbf[q];
    sb += lbb[q];
  }
  if (cf != cb) return cb < cf ? 1 : 0;
  return sb > sf ? 1 : 0;
}

/* Section 2.3: the children of (sigma1, sigma2) for the unscheduled job at
 * list position q: forward = (sigma1 j, sigma2), backward = (sigma1, j sigma2).
 * The remaining unscheduled jobs keep their list order. */
static void make_child(int n, const uint8_t *perm, int d1, int d2, int q, int dir,
                       uint8_t *out) {
  int r = n - d1 - d2;
  uint8_t j = perm[d1 + q];
  memcpy(out, perm, (size_t)d1);
  int w = d1;
  if (dir == 0) out[w++] = j;
  for (int i = 0; i < r; ++i)
    if (i != q) out[w++] = perm[d1 + i];
  if (dir == 1) out[w++] = j;
  memcpy(out + w, perm + (n - d2), (size_t)d2);
}

/* Decomposition of a batch of parents (Figure 2 of Section 2.3 and the
 * bounding/pruning operators of Section 2.2): both children sets are bounded,
 * MinMin picks a direction, and a child is pruned iff its LB >= ub.  Output
 * slot q of direction dir belongs to the job perm[d1 + q]; slots q >= n-d1-d2
 * hold INT32_MAX and a prune flag of 1.  Returns 0, or -1 on invalid input. */
int or_bound_children(int n, int m, const int32_t *p, int count, const uint8_t *perm,
                      const uint8_t *d1, const uint8_t *d2, int kind, int64_t ub,
                      const uint32_t *pair_mask, int mask_words, int32_t *out_lb,
                      uint8_t *out_prune, uint8_t *out_dir, int32_t *out_argpair,
                      int threads) {
  if (n < 2 || n > 255 || m < 1 || m > MAXM) return -1;
  if (kind != OR_LB1 && m < 2) return -1;
  for (int i = 0; i < count; ++i)
    if ((int)d1[i] + (int)d2[i] >= n) return -1;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads) if (threads > 1)
  for (int i = 0; i < count; ++i) {
    const uint8_t *pp = perm + (size_t)i * n;
    int a = d1[i], b = d2[i], r = n - a - b;
    const uint32_t *mask = pair_mask ? pair_mask + (size_t)i * mask_words : NULL;
    int64_t lb[2][MAXN];
    uint8_t child[MAXN];
    for (int dir = 0; dir < 2; ++dir)
      for (int q = 0; q < n; ++q) {
        size_t o = ((size_t)i * 2 + dir) * n + q;
        if (q >= r) {
          out_lb[o] = INT32_MAX;
          out_prune[o] = 1;
          if (out_argpair) out_argpair[o] = -1;
          continue;
        }
        make_child(n, pp, a, b, q, dir, child);
        int32_t ap = -1;
        int64_t x = or_node_bound(n, m, p, child, a + (dir == 0), b + (dir == 1), kind, mask,
                                  out_argpair ? &ap : NULL);
        if (x > INT32_MAX) err = 1;
        lb[dir][q] = x;
        out_lb[o] = (int32_t)x;
        out_prune[o] = x >= ub;
        if (out_argpair) out_argpair[o] = ap;
      }
    if (out_dir) out_dir[i] = (uint8_t)or_minmin(r, lb[0], lb[1]);
  }
  return err ? -3 : 0;
}

/* Depth-first branch-and-bound (Sections 2.2-2.5) with dynamic branching and
 * MinMin.  A child is explored iff its LB < incumbent at the time it is
 * visited; the children of the chosen set are visited in list order; leaves
 * (no unscheduled job left) update the incumbent when strictly better.  With
 * kind OR_LB2_SUBSET every node is bounded over the same pair set `mask`
 * (Section 2.4: any number of pairs between m and m(m-1)/2).  lb1_r > 0
 * chooses the bound by depth: the children of a node with at most lb1_r
 * unscheduled jobs get LB1, the others `kind` (Section 2.4 ranks LB1 as the
 * cheaper, weaker bound; any valid bound keeps the search exact). */
typedef struct {
  int n, m, kind, cutoff, lb1_r;
  const int32_t *p;
  const uint32_t *mask;
  int64_t ub, budget, nodes, children;
  int found, aborted;
  uint8_t best[MAXN];
} search_t;

/* Bounds both children sets of a node and returns the MinMin direction. */
static int decompose(const search_t *s, const uint8_t *perm, int d1, int d2,
                     int64_t lb[2][MAXN]) {
  int n = s->n, r = n - d1 - d2;
  int kind = r <= s->lb1_r ? OR_LB1 : s->kind;
  uint8_t child[MAXN];
  for (int dir = 0; dir < 2; ++dir)
    for (int q = 0; q < r; ++q) {
      make_child(n, perm, d1, d2, q, dir, child);
      lb[dir][q] = or_node_bound(n, s->m, s->p, child, d1 + (dir == 0), d2 + (dir == 1),
                                 kind, s->mask, NULL);
    }
  return or_minmin(r, lb[0], lb[1]);
}

static void dfs(search_t *s, const uint8_t *perm, int d1, int d2) {
  if (s->budget > 0 && s->nodes >= s->budget) {
    s->aborted = 1;
    return;
  }
  int n = s->n, r = n - d1 - d2;
  s->nodes += 1;
  s->children += 2 * r;
  int64_t lb[2][MAXN];
  uint8_t child[MAXN];
  int dir = decompose(s, perm, d1, d2, lb);
  for (int q = 0; q < r; ++q) {
    int64_t x = lb[dir][q];
    if (x >= s->ub) continue;
    make_child(n, perm, d1, d2, q, dir, child);
    if (r == 1) {
      s->ub = x;
      s->found = 1;
      memcpy(s->best, child, (size_t)n);
    } else {
      uint8_t keep[MAXN];
      memcpy(keep, child, (size_t)n);
      dfs(s, keep, d1 + (dir == 0), d2 + (dir == 1));
      if (s->aborted) return;
    }
  }
}

/* The same search with the children of nodes shallower than s->cutoff run
 * as OpenMP tasks.  The incumbent, the counters and the best schedule are
 * shared: the incumbent is read atomically when a child is visited and
 * lowered under a critical section by a strictly better leaf.  When the
 * incumbent cannot improve (it starts at the optimum) the decomposed nodes
 * are exactly those of dfs(), in any order. */
static void dfs_task(search_t *s, const uint8_t *perm, int d1, int d2, int depth) {
  int n = s->n, r = n - d1 - d2;
#pragma omp atomic
  s->nodes += 1;
#pragma omp atomic
  s->children += 2 * r;
  int64_t lb[2][MAXN];
  int dir = decompose(s, perm, d1, d2, lb);
  for (int q = 0; q < r; ++q) {
    int64_t x = lb[dir][q], ub;
#pragma omp atomic read
    ub = s->ub;
    if (x >= ub) continue;
    uint8_t child[MAXN];
    make_child(n, perm, d1, d2, q, dir, child);
    if (r == 1) {
#pragma omp critical(or_incumbent)
      {
        if (x < s->ub) {
#pragma omp atomic write
          s->ub = x;
          s->found = 1;
          memcpy(s->best, child, (size_t)n);
        }
      }
    } else if (depth < s->cutoff) {
      int a = d1 + (dir == 0), b = d2 + (dir == 1);
#pragma omp task firstprivate(child, a, b) shared(s)
      dfs_task(s, child, a, b, depth + 1);
    } else {
      dfs_task(s, child, d1 + (dir == 0), d2 + (dir == 1), depth + 1);
    }
  }
}

/* Searches for a schedule with C_max < ub0.  found = 1 iff one was found
 * (best_cmax / best_perm set); proven = 1 iff the tree was exhausted within
 * the budget (0 = unlimited) of decomposed nodes.  nodes counts decomposed
 * nodes including the root; children counts bounded children (2(n-d) each).
 * kind OR_LB2_SUBSET bounds every node over the pairs of pair_mask (else
 * ignored).  threads > 1 runs the task-parallel search (budget must be 0).
 * lb1_r: nodes with at most this many unscheduled jobs bound their children
 * with LB1 (0: never). */
int or_search_ex(int n, int m, const int32_t *p, int64_t ub0, int kind,
                 const uint32_t *pair_mask, int64_t budget, int threads, int lb1_r,
                 int64_t *best_cmax, uint8_t *best_perm, int64_t *nodes, int64_t *children,
                 int *found, int *proven) {
  if (n < 2 || n > 255 || m < 1 || m > MAXM) return -1;
  if (lb1_r < 0) return -1;
  if (kind != OR_LB1 && kind != OR_LB2_FULL && kind != OR_LB2_SUBSET) return -1;
  if (kind != OR_LB1 && m < 2) return -1;
  if (kind == OR_LB2_SUBSET && !pair_mask) return -1;
  if (threads > 1 && budget > 0) return -1;
  search_t *s = (search_t *)calloc(1, sizeof(search_t));
  if (!s) return -4;
  s->n = n; s->m = m; s->kind = kind; s->p = p;
  s->mask = kind == OR_LB2_SUBSET ? pair_mask : NULL;
  s->ub = ub0; s->budget = budget;
  s->lb1_r = lb1_r;
  s->cutoff = n / 2;
  uint8_t root[MAXN];
  for (int j = 0; j < n; ++j) root[j] = (uint8_t)j;
  if (threads > 1) {
#pragma omp parallel num_threads(threads)
#pragma omp single
    dfs_task(s, root, 0, 0, 0);
  } else {
    dfs(s, root, 0, 0);
  }
  *best_cmax = s->found ? s->ub : ub0;
  if (s->found && best_perm) memcpy(best_perm, s->best, (size_t)n);
  *nodes = s->nodes;
  *children = s->children;
  *found = s->found;
  *proven = !s->aborted;
  free(s);
  return 0;
}

int or_search(int n, int m, const int32_t *p, int64_t ub0, int kind, int64_t budget,
              int64_t *best_cmax, uint8_t *best_perm, int64_t *nodes, int64_t *children,
              int *found, int *proven) {
  if (kind != OR_LB1 && kind != OR_LB2_FULL) return -1;
  return or_search_ex(n, m, p, ub0, kind, NULL, budget, 1, 0, best_cmax, best_perm, nodes,
                      children, found, proven);
}

/* Optimal makespan by enumerating all n! permutations (n <= 10 or so). */
int64_t or_bruteforce(int n, int m, const int32_t *p, uint8_t *best_perm) {
  uint8_t s[MAXN];
  for (int j = 0; j < n; ++j) s[j] = (uint8_t)j;
  int64_t best = INT64_MAX;
  do {
    int64_t c = or_makespan(m, p, s, n);
    if (c < best) {
      best = c;
      if (best_perm) memcpy(best_perm, s, (size_t)n);
    }
  } while (next_perm(s, n));
  return best;
}

/* Nawaz-Enscore-Ham insertion heuristic for the initial incumbent: jobs in
 * decreasing order of total processing time (equal totals: lower id first),
 * each inserted at the position of the partial sequence that minimises its
 * makespan (equal makespans: earliest position). */
int64_t or_neh(int n, int m, const int32_t *p, uint8_t *perm_out) {
  uint8_t order[MAXN], seq[MAXN], trial[MAXN];
  int64_t tot[MAXN];
  for (int j = 0; j < n; ++j) {
    order[j] = (uint8_t)j;
    tot[j] = 0;
    for (int k = 0; k < m; ++k) tot[j] += P_(p, m, j, k);
  }
  for (int i = 1; i < n; ++i) {
    uint8_t x = order[i];
    int k = i - 1;
    while (k >= 0 && tot[order[k]] < tot[x]) {
      order[k + 1] = order[k];
      --k;
    }
    order[k + 1] = x;
  }
  int len = 0;
  for (int i = 0; i < n; ++i) {
    int bestpos = 0;
    int64_t best = INT64_MAX;
    for (int pos = 0; pos <= len; ++pos) {
      memcpy(trial, seq, (size_t)pos);
      trial[pos] = order[i];
      memcpy(trial + pos + 1, seq + pos, (size_t)(len - pos));
      int64_t c = or_makespan(m, p, trial, len + 1);
      if (c < best) {
        best = c;
        bestpos = pos;
      }
    }
    memmove(seq + bestpos + 1, seq + bestpos, (size_t)(len - bestpos));
    seq[bestpos] = order[i];
    ++len;
  }
  memcpy(perm_out, seq, (size_t)n);
  return or_makespan(m, p, seq, n);
}
