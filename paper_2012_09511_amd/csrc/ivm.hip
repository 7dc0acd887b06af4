// Depth-first search with integer-vector-matrix (IVM) explorers, factoradic
// work units and work stealing on the device (Sections 2.5, 2.6, 3.1-3.4).
//
// Each of K explorers holds one IVM: a level I, a position vector V (the cell
// chosen in each row), a matrix M whose row L lists the jobs that can be
// scheduled at level L (row 0: all n jobs, row L + 1: row L without the job
// chosen at L, in the same order), a prune flag and the stored bound of every
// cell, and the direction D[L] in which row L's jobs are scheduled (the
// MinMin choice of the node that generated the row; level 0 schedules one
// job).  The node at level I schedules M[L][V[L]], L <= I: at the front of
// sigma1 in level order for D[L] = 0, at the front of sigma2 (so sigma2 reads
// the back-scheduled levels in reverse) for D[L] = 1; its unscheduled jobs
// are row I without the chosen cell.
//
// Read as digits (digit L in [0, n - L), weight (n - 1 - L)!), V numbers the
// n! complete schedules in the factorial number system, and a depth-first
// exploration moves V forward through [0, n!).  An explorer owns an interval
// [V, E) of that numbering (a work unit).  When fewer than 80 % of the
// explorers hold work, each empty explorer steals the right half of a busy
// neighbour's interval: the K = 4^d explorers are the vertices of a 4-ary
// d-cube, and in 3d rounds (digit i of the index lowered by j = 1, 2, 3,
// mod 4) an empty explorer takes a neighbour that nobody took in this phase
// and whose interval is longer than the average and than a minimum.  A thief
// starts at the midpoint: it decomposes the root and the midpoint's ancestors
// again (those decompositions belong to the explorer that owned them before
// and are not counted), then explores from there.  With the incumbent fixed,
// every node is therefore decomposed and counted exactly once, by the
// explorer whose interval holds its first position.
//
// One step: k_ivm_select (every explorer moves to its next node and writes it
// as a pool row) -> the bounding kernels of pfsp_bound_children on that
// pool -> k_ivm_branch (rows of the next level, prune flags, leaves) ->
// k_ivm_balance (the step's best leaf; a stealing phase, every poll_every
// steps when few explorers were busy, with the lengths from k_ivm_branch).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "internal.h"

namespace pfsp {

constexpr int kIvmMaxN = 64;

// ------------------------------------------------------ factoradic numbers
// A position in [0, n!]: digits d[0 .. n) (digit L in [0, n - L), weight
// (n - 1 - L)!) and a top digit in {0, 1} for n! itself.
__host__ __device__ inline int fact_cmp(int n, const uint8_t *a, int atop, const uint8_t *b,
                                        int btop) {
  if (atop != btop) return atop < btop ? -1 : 1;
  for (int L = 0; L < n; ++L)
    if (a[L] != b[L]) return a[L] < b[L] ? -1 : 1;
  return 0;
}

// c = a + b; returns the top digit of the sum (a + b <= n! assumed).
__host__ __device__ inline int fact_add(int n, const uint8_t *a, int atop, const uint8_t *b,
                                        int btop, uint8_t *c) {
  int carry = 0;
  for (int L = n - 1; L >= 0; --L) {  // digits below their radix: the carry is 0 or 1
    const int radix = n - L;
    int t = a[L] + b[L] + carry;
    carry = t >= radix;
    if (carry) t -= radix;
    c[L] = (uint8_t)t;
  }
  return atop + btop + carry;
}

// c = b - a (b >= a); returns the top digit of the difference.
__host__ __device__ inline int fact_sub(int n, const uint8_t *b, int btop, const uint8_t *a,
                                        int atop, uint8_t *c) {
  int borrow = 0;
  for (int L = n - 1; L >= 0; --L) {
    int t = (int)b[L] - (int)a[L] - borrow;
    borrow = t < 0;
    if (borrow) t += n - L;
    c[L] = (uint8_t)t;
  }
  return btop - atop - borrow;
}

// c = floor(c / 2) in place (top digit ctop on entry); the top of the result is 0.
__host__ __device__ inline void fact_half(int n, uint8_t *c, int ctop) {
  int rem = ctop;  // one unit of the digit above L is n - L units of digit L
  for (int L = 0; L < n; ++L) {
    const int t = c[L] + rem * (n - L);
    c[L] = (uint8_t)(t >> 1);
    rem = t & 1;
  }
}

// The value as a double (interval lengths for the stealing heuristics).
__host__ __device__ inline double fact_double(int n, const uint8_t *a, int atop) {
  double v = 0.0, w = 1.0;  // w = (n - 1 - L)!
  for (int L = n - 1; L >= 0; --L) {
    v += a[L] * w;
    w *= (double)(n - L);
  }
  return v + atop * w;
}

// ------------------------------------------------------------ IVM decoding
// Pool row (perm, d1, d2) of the node at level I (see the file comment).
// M rows have stride n.
__host__ __device__ inline void ivm_decode(int n, const uint8_t *M, const uint8_t *V,
                                           const uint8_t *D, int I, uint8_t *perm, int *d1,
                                           int *d2) {
  int a = 0, b = 0;
  for (int L = 0; L <= I; ++L) {
    const uint8_t j = M[L * n + V[L]];
    if (D[L] == 0)
      perm[a++] = j;
    else
      perm[n - 1 - b++] = j;
  }
  const uint8_t *row = M + I * n;
  int w = a;
  for (int x = 0; x < n - I; ++x)
    if (x != V[I]) perm[w++] = row[x];
  *d1 = a;
  *d2 = b;
}

enum : int { kIvmEmpty = 0, kIvmActive = 1, kIvmInit = 2, kIvmRoot = 3 };

struct IvmCtl {
  int batch;       // rows of this step's pool (explorers that hold a node)
  int pad0;
  int ub;          // incumbent (lowered by atomicMin)
  int ub_step;     // prune threshold of the step
  unsigned long long step_best;  // (makespan << 32) | pool row of the step's best leaf
  long long nodes, children, steps, steals;
  double len_sum;  // interval lengths of the busy explorers (stealing phases)
  int busy;        // busy explorers (stealing phases)
  int newbest;
  int last_batch;  // rows of the last finished step
  int pad1;
};

struct IvmState {
  int n = 0, K = 0, d = 0;
  hipStream_t stream = nullptr;
  int *st = nullptr, *lev = nullptr;  // [K] state, level
  uint8_t *V = nullptr, *E = nullptr, *D = nullptr;  // [K][n]
  uint8_t *Etop = nullptr;                           // [K]
  uint8_t *M = nullptr;                              // [K][n][n]
  unsigned long long *Pr = nullptr;                  // [K][n] prune bits per row
  int *LB = nullptr;                                 // [K][n][n] stored child bounds
  double *len = nullptr;                             // [K]
  int *taken = nullptr;                              // [K]
  // pool of the step
  uint8_t *b_perm = nullptr, *b_d1 = nullptr, *b_d2 = nullptr, *b_dir = nullptr;
  int *b_ivm = nullptr;
  uint8_t *b_counted = nullptr;
  int *out_lb = nullptr;
  uint8_t *out_prune = nullptr, *best_perm = nullptr;
  IvmCtl *ctl = nullptr, *ctl_host = nullptr;
};

static void ivm_free(IvmState *S) {
  if (!S) return;
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  void *bufs[] = {S->st,     S->lev,   S->V,     S->E,      S->D,     S->Etop,
                  S->M,      S->Pr,    S->LB,    S->len,    S->taken, S->b_perm,
                  S->b_d1,   S->b_d2,  S->b_dir, S->b_ivm,  S->b_counted, S->out_lb,
                  S->out_prune, S->best_perm, S->ctl};
  for (void *p : bufs) (void)hipFree(p);
  if (S->ctl_host) (void)hipHostFree(S->ctl_host);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

// -------------------------------------------------------------- kernels
__device__ __forceinline__ bool cell_pruned(const IvmState &S, int k, int L, int x, int ub) {
  const size_t cell = ((size_t)k * S.n + L) * S.n + x;
  return ((S.Pr[(size_t)k * S.n + L] >> x) & 1ull) || S.LB[cell] >= ub;
}

// Appends the rows of the wave's lanes with app set to a counter: one atomic
// per wave; returns this lane's slot.
__device__ __forceinline__ int wave_append(int *count, bool app) {
  const uint64_t bal = __ballot(app);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (bal) {
    if (lane == 0) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, 0, 64);
  }
  return base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
}

// Every explorer moves to its next node (depth-first, leftmost first) and
// writes it as a row of the step's pool.  The walk reads the explorer's
// position and interval end many times, so both are copied to LDS first
// (digit L of thread t at [L][t]) and the position is written back once.
__global__ void __launch_bounds__(256) k_ivm_select(IvmState S) {
  __shared__ uint8_t sV[kIvmMaxN * 256], sE[kIvmMaxN * 256], sP[kIvmMaxN * 256];
  const int t = threadIdx.x;
  const int k = blockIdx.x * blockDim.x + t;
  IvmCtl *c = S.ctl;
  const int n = S.n;
  bool emit = false, counted = true, root = false;
  int I = -1;
  if (k < S.K && S.st[k] != kIvmEmpty) {
    int st = S.st[k];
    uint8_t *Vg = S.V + (size_t)k * n;
    const uint8_t *Eg = S.E + (size_t)k * n;
    for (int L = 0; L < n; ++L) {
      sV[L * 256 + t] = Vg[L];
      sE[L * 256 + t] = Eg[L];
    }
    auto V = [&](int L) -> uint8_t & { return sV[L * 256 + t]; };
    // position >= interval end (the top digit of the position is 0)
    auto at_end = [&]() {
      const int etop = S.Etop[k];
      if (etop) return false;
      for (int L = 0; L < n; ++L) {
        const int a = sV[L * 256 + t], b = sE[L * 256 + t];
        if (a != b) return a > b;
      }
      return true;
    };
    const int ub = c->ub_step;
    I = S.lev[k];
    if (st == kIvmRoot) {
      // the root: decomposed again by a thief (not counted) unless the work
      // unit starts at position 0
      for (int L = 0; L < n; ++L) counted = counted && V(L) == 0;
      root = true;
      emit = true;
    } else {
      bool moved = false;
      if (st == kIvmInit) {
        if (cell_pruned(S, k, I, V(I), ub)) {
          // the path's subtree is pruned: continue after it
          for (int L = I + 1; L < n; ++L) V(L) = 0;
          V(I) += 1;
          moved = true;
          st = kIvmActive;
        } else {
          bool zero = true;
          for (int L = I + 1; L < n; ++L) zero = zero && V(L) == 0;
          if (zero) {
            st = kIvmActive;  // the work unit starts at this node: it is ours
          } else {
            counted = false;  // an ancestor of the work unit's start
            emit = true;
          }
        }
      }
      if (st == kIvmActive) {
        // the cells of row L that cannot be taken: pruned, bound at or above
        // the incumbent, or past the row's end (its bounds load together)
        auto row_mask = [&](int L) -> unsigned long long {
          unsigned long long msk = S.Pr[(size_t)k * n + L];
          const int *__restrict__ lbr = S.LB + ((size_t)k * n + L) * n;
          const int len = n - L;
          for (int x = 0; x < len; ++x)
            if (lbr[x] >= ub) msk |= 1ull << x;
          return len >= 64 ? msk : msk | (~0ull << len);
        };
        unsigned long long mI = I >= 0 ? row_mask(I) : 0ull;
        for (;;) {
          if (I < 0) {
            st = kIvmEmpty;
            break;
          }
          const int x0 = V(I);
          const unsigned long long open = x0 < 64 ? ~mI & (~0ull << x0) : 0ull;
          if (!open) {  // the rest of the row is closed: back to the parent's next sibling
            V(I) = 0;
            --I;
            if (I >= 0) {
              V(I) += 1;
              mI = row_mask(I);
            }
            moved = true;
            continue;
          }
          // the next open cell; the cells skipped are closed, and a position
          // past the end of the work unit stays past it as it grows
          const int x = __builtin_ctzll(open);
          if (x != x0) {
            V(I) = (uint8_t)x;
            moved = true;
          }
          if (at_end()) {
            st = kIvmEmpty;
            break;
          }
          emit = true;
          break;
        }
      }
      if (moved)
        for (int L = 0; L < n; ++L) Vg[L] = sV[L * 256 + t];
      S.st[k] = st;
      S.lev[k] = I;
    }
  }
  if (k < S.K) {  // for a stealing phase at the end of this step
    S.taken[k] = 0;
    if (!emit) S.len[k] = 0.0;
  }
  const int b = wave_append(&c->batch, emit);
  if (!emit) return;
  uint8_t *perm = S.b_perm + (size_t)b * n;
  int d1 = 0, d2 = 0;
  if (root) {
    for (int j = 0; j < n; ++j) perm[j] = (uint8_t)j;
  } else {
    // ivm_decode with the row built in LDS: the loads of M and D do not wait
    // for stores to the pool row
    const uint8_t *__restrict__ Mk = S.M + (size_t)k * n * n;
    const uint8_t *__restrict__ Dk = S.D + (size_t)k * n;
#pragma unroll 4
    for (int L = 0; L <= I; ++L) {
      const uint8_t j = Mk[L * n + sV[L * 256 + t]];
      if (Dk[L] == 0)
        sP[(d1++) * 256 + t] = j;
      else
        sP[(n - 1 - d2++) * 256 + t] = j;
    }
    const uint8_t *__restrict__ row = Mk + (size_t)I * n;
    const int vi = sV[I * 256 + t];
    int w = d1;
#pragma unroll 4
    for (int x = 0; x < n - I; ++x)
      if (x != vi) sP[(w++) * 256 + t] = row[x];
    for (int x = 0; x < n; ++x) perm[x] = sP[x * 256 + t];
  }
  S.b_d1[b] = (uint8_t)d1;
  S.b_d2[b] = (uint8_t)d2;
  S.b_ivm[b] = k;
  S.b_counted[b] = counted;
}

// Per pool row: node statistics, leaves, and the next row of the explorer.
__device__ void ivm_branch_row(const IvmState &S, IvmCtl *c, int b) {
  const int n = S.n;
  const int k = S.b_ivm[b];
  const int r = n - S.b_d1[b] - S.b_d2[b], dir = S.b_dir[b];
  const int ub = c->ub_step;
  const int *__restrict__ lb = S.out_lb + ((size_t)b * 2 + dir) * n;
  const uint8_t *__restrict__ pr = S.out_prune + ((size_t)b * 2 + dir) * n;
  const int st = S.st[k];
  int I = st == kIvmRoot ? -1 : S.lev[k];
  uint8_t *V = S.V + (size_t)k * n;
  if (r == 1) {  // the only child is a complete schedule: its bound is its makespan
    if (!pr[0] && lb[0] < ub) {
      atomicMin(&c->ub, lb[0]);
      atomicMin(&c->step_best, ((unsigned long long)(unsigned)lb[0] << 32) | (unsigned)b);
    }
    V[I] += 1;
    return;
  }
  // row I + 1: the unscheduled jobs in list order, their flags and bounds
  const int L = I + 1;
  const uint8_t *__restrict__ perm = S.b_perm + (size_t)b * n;
  const int a = S.b_d1[b];
  uint8_t *__restrict__ row = S.M + ((size_t)k * n + L) * n;
  int *__restrict__ lbrow = S.LB + ((size_t)k * n + L) * n;
  unsigned long long bits = 0ull;
#pragma unroll 4
  for (int q = 0; q < r; ++q) {
    row[q] = perm[a + q];
    lbrow[q] = lb[q];
    if (pr[q]) bits |= 1ull << q;
  }
  S.Pr[(size_t)k * n + L] = bits;
  S.D[(size_t)k * n + L] = (uint8_t)dir;
  S.lev[k] = L;
  if (st == kIvmRoot) {
    S.st[k] = kIvmInit;  // walk down to the start of the work unit
  } else if (st == kIvmActive) {
    V[L] = 0;
  }
  // an initializing explorer keeps V[L], the start's digit
}

// Length E - V of explorer k's interval as a double (the digits of the
// difference are produced from the least significant one up and summed with
// their weights, so no digit array is kept).
__device__ inline double ivm_len(const IvmState &S, int k) {
  const int n = S.n;
  const uint8_t *__restrict__ V = S.V + (size_t)k * n;
  const uint8_t *__restrict__ E = S.E + (size_t)k * n;
  double v = 0.0, w = 1.0;  // w = (n - 1 - L)!
  int borrow = 0;
#pragma unroll 8
  for (int L = n - 1; L >= 0; --L) {
    int t = (int)E[L] - (int)V[L] - borrow;
    borrow = t < 0;
    if (borrow) t += n - L;
    v += t * w;
    w *= (double)(n - L);
  }
  return v + (S.Etop[k] - borrow) * w;
}

// Whether this step ends with a stealing phase: every every-th step, when
// fewer than 80 % of the explorers held a node in it (uniform).
__device__ __forceinline__ bool ivm_balancing(const IvmState &S, int every) {
  const IvmCtl *c = S.ctl;
  return S.K > 1 && c->steps % every == 0 && c->batch * 5 < S.K * 4;
}

// Per pool row: node statistics, leaves, and the next row of the explorer;
// on a stealing step also the first part of the phase: the interval lengths
// of the busy explorers (those in the pool), their sum and count.  The
// empty explorers' lengths and every explorer's victim flag were cleared by
// k_ivm_select.
__global__ void __launch_bounds__(256) k_ivm_branch(IvmState S, int every) {
  IvmCtl *c = S.ctl;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int count = c->batch;
  const int n = S.n;
  {  // node statistics, one atomic per wave
    const bool cnt = b < count && S.b_counted[b];
    long long nodes = cnt, ch = cnt ? 2 * (n - S.b_d1[b] - S.b_d2[b]) : 0;
    for (int o = 32; o >= 1; o >>= 1) {
      nodes += __shfl_xor(nodes, o, 64);
      ch += __shfl_xor(ch, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && nodes) {
      atomicAdd((unsigned long long *)&c->nodes, (unsigned long long)nodes);
      atomicAdd((unsigned long long *)&c->children, (unsigned long long)ch);
    }
  }
  if (b < count) ivm_branch_row(S, c, b);
  if (!ivm_balancing(S, every)) return;  // uniform
  double l = 0.0;
  int busy = 0;
  if (b < count) {
    const int k = S.b_ivm[b];
    l = ivm_len(S, k);
    S.len[k] = l;
    busy = 1;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    l += __shfl_xor(l, o, 64);
    busy += __shfl_xor(busy, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && busy) {
    atomicAdd(&c->len_sum, l);
    atomicAdd(&c->busy, busy);
  }
}

// The step's best leaf, then the stealing phase's second part (one block):
// in 3d rounds (digit i of the index lowered by j = 1, 2, 3, mod 4) every
// empty explorer e tries the neighbour v and takes the right half of v's
// interval if v is busy, nobody took from v in this phase, and v's interval
// is longer than the mean and than min_len.  SH (K <= kIvmBalLds): the busy
// flags, lengths and victim flags of the phase sit in LDS.  Each thread
// stages its victim's digits in LDS for the midpoint.  Last, the control
// block is reset for the next step.
constexpr int kIvmBalThreads = 1024, kIvmBalLds = 4096;
template <bool SH>
__global__ void __launch_bounds__(kIvmBalThreads) k_ivm_balance(IvmState S, double min_len,
                                                                int every) {
  constexpr int T = kIvmBalThreads;
  __shared__ uint8_t sA[kIvmMaxN * T], sB[kIvmMaxN * T];
  __shared__ uint8_t sBusy[SH ? kIvmBalLds : 1];
  __shared__ float sLen[SH ? kIvmBalLds : 1];
  __shared__ uint32_t sTaken[SH ? kIvmBalLds / 32 : 1];
  IvmCtl *c = S.ctl;
  const int K = S.K, n = S.n, t = threadIdx.x;
  {  // the step's best leaf: its schedule (a one-job parent's only child is
     // its own row) and the flag for the host
    const unsigned long long sb = c->step_best;
    if (sb != ~0ull) {
      const int b = (int)(sb & 0xffffffffu);
      for (int x = t; x < n; x += T) S.best_perm[x] = S.b_perm[(size_t)b * n + x];
      if (t == 0) c->newbest = 1;
    }
  }
  const int busy = c->busy;
  const double avg = busy ? c->len_sum / busy : 0.0;
  long long steals = 0;
  // uniform: a stealing step with a busy explorer
  const int rounds = ivm_balancing(S, every) && busy > 0 ? S.d : 0;
  if (SH && rounds) {
    for (int k = t; k < K; k += T) {
      sBusy[k] = S.st[k] != kIvmEmpty;
      sLen[k] = (float)S.len[k];
    }
    for (int x = t; x < (K + 31) / 32; x += T) sTaken[x] = 0u;
    __syncthreads();
  }
  for (int i = 0; i < rounds; ++i) {
    for (int j = 1; j <= 3; ++j) {
      for (int e = t; e < K; e += T) {
        if (SH ? sBusy[e] != 0 : S.st[e] != kIvmEmpty) continue;
        const int dig = (e >> (2 * i)) & 3;
        const int v = e - (dig << (2 * i)) + (((dig - j) & 3) << (2 * i));
        if (v == e) continue;
        if (SH) {
          if (!sBusy[v] || sLen[v] <= avg || sLen[v] < min_len) continue;
          const uint32_t bit = 1u << (v & 31);
          if (atomicOr(&sTaken[v >> 5], bit) & bit) continue;
        } else {
          if (S.st[v] == kIvmEmpty || S.len[v] <= avg || S.len[v] < min_len) continue;
          if (atomicCAS(&S.taken[v], 0, 1) != 0) continue;
        }
        uint8_t *__restrict__ Vv = S.V + (size_t)v * n;
        uint8_t *__restrict__ Ev = S.E + (size_t)v * n;
        uint8_t *__restrict__ Ve = S.V + (size_t)e * n;
        uint8_t *__restrict__ Ee = S.E + (size_t)e * n;
        for (int L = 0; L < n; ++L) {
          sA[L * T + t] = Vv[L];
          sB[L * T + t] = Ev[L];
        }
        // mid = Vv + (Ev - Vv) / 2 < Ev, in sB: difference, half, sum
        int borrow = 0;
        for (int L = n - 1; L >= 0; --L) {
          int x = (int)sB[L * T + t] - (int)sA[L * T + t] - borrow;
          borrow = x < 0;
          if (borrow) x += n - L;
          Ee[L] = sB[L * T + t];  // the thief's end: the victim's old end
          sB[L * T + t] = (uint8_t)x;
        }
        int rem = S.Etop[v] - borrow;
        for (int L = 0; L < n; ++L) {
          const int x = sB[L * T + t] + rem * (n - L);
          sB[L * T + t] = (uint8_t)(x >> 1);
          rem = x & 1;
        }
        int carry = 0;
        for (int L = n - 1; L >= 0; --L) {
          int x = sA[L * T + t] + sB[L * T + t] + carry;
          carry = x >= n - L;
          if (carry) x -= n - L;
          Ve[L] = (uint8_t)x;
          Ev[L] = (uint8_t)x;
        }
        S.Etop[e] = S.Etop[v];
        S.Etop[v] = (uint8_t)carry;
        S.st[e] = kIvmRoot;
        S.lev[e] = -1;
        if (SH) sBusy[e] = 1;  // a thief is no victim in this phase (its length stays 0)
        ++steals;
      }
      __syncthreads();  // the next round sees this round's thieves and victims
    }
  }
  for (int o = 32; o >= 1; o >>= 1) steals += __shfl_xor(steals, o, 64);
  if ((t & 63) == 0 && steals)
    atomicAdd((unsigned long long *)&c->steals, (unsigned long long)steals);
  __syncthreads();  // every read of the control block above is done
  if (t == 0) {     // the next step's start
    c->last_batch = c->batch;
    c->batch = 0;
    c->ub_step = c->ub;
    c->step_best = ~0ull;
    c->steps += 1;
    c->len_sum = 0.0;
    c->busy = 0;
  }
}

static IvmState *ivm_alloc(Ctx *c, int K) {
  const int n = c->n;
  IvmState *S = new (std::nothrow) IvmState();
  if (!S) return nullptr;
  S->n = n;
  S->K = K;
  bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
  auto alloc = [&](void **p, size_t bytes) {
    if (ok && hipMalloc(p, bytes ? bytes : 1) != hipSuccess) ok = false;
  };
  const size_t Kn = (size_t)K * n, Knn = Kn * n;
  alloc((void **)&S->st, K * 4);
  alloc((void **)&S->lev, K * 4);
  alloc((void **)&S->V, Kn);
  alloc((void **)&S->E, Kn);
  alloc((void **)&S->D, Kn);
  alloc((void **)&S->Etop, K);
  alloc((void **)&S->M, Knn);
  alloc((void **)&S->Pr, Kn * 8);
  alloc((void **)&S->LB, Knn * 4);
  alloc((void **)&S->len, (size_t)K * 8);
  alloc((void **)&S->taken, (size_t)K * 4);
  alloc((void **)&S->b_perm, Kn);
  alloc((void **)&S->b_d1, K);
  alloc((void **)&S->b_d2, K);
  alloc((void **)&S->b_dir, K);
  alloc((void **)&S->b_ivm, (size_t)K * 4);
  alloc((void **)&S->b_counted, K);
  alloc((void **)&S->out_lb, Kn * 2 * 4);
  alloc((void **)&S->out_prune, Kn * 2);
  alloc((void **)&S->best_perm, n);
  alloc((void **)&S->ctl, sizeof(IvmCtl));
  if (ok && hipHostMalloc((void **)&S->ctl_host, sizeof(IvmCtl), hipHostMallocDefault) !=
                hipSuccess)
    ok = false;
  if (!ok) {
    ivm_free(S);
    return nullptr;
  }
  return S;
}

// Work units of the K explorers: [0, n!) halved recursively, each bound
// rounded down to the first position of its subtree at a shallow level (so
// that an explorer's start needs few initialising decompositions).
static void initial_units(int n, int K, std::vector<uint8_t> &V, std::vector<uint8_t> &E,
                          std::vector<uint8_t> &Etop) {
  std::vector<uint8_t> bnd((size_t)(K + 1) * n, 0);
  std::vector<int> top(K + 1, 0);
  top[K] = 1;  // n!
  for (int step = K; step > 1; step >>= 1)
    for (int lo = 0; lo < K; lo += step) {
      const int hi = lo + step, mid = lo + step / 2;
      uint8_t *m = &bnd[(size_t)mid * n];
      const int t = fact_sub(n, &bnd[(size_t)hi * n], top[hi], &bnd[(size_t)lo * n], top[lo], m);
      fact_half(n, m, t);
      top[mid] = fact_add(n, &bnd[(size_t)lo * n], top[lo], m, 0, m);
    }
  // keep the digits of the levels whose subtrees still outnumber 4K explorers
  int keep = 0;
  double leaves = 1.0;
  while (keep < n && leaves < 4.0 * K) leaves *= (double)(n - keep++);
  for (int x = 1; x < K; ++x)
    for (int L = keep; L < n; ++L) bnd[(size_t)x * n + L] = 0;
  V.assign((size_t)K * n, 0);
  E.assign((size_t)K * n, 0);
  Etop.assign(K, 0);
  for (int x = 0; x < K; ++x) {
    memcpy(&V[(size_t)x * n], &bnd[(size_t)x * n], n);
    memcpy(&E[(size_t)x * n], &bnd[(size_t)(x + 1) * n], n);
    Etop[x] = (uint8_t)top[x + 1];
  }
}

}  // namespace pfsp

using namespace pfsp;

namespace pfsp {
namespace {

// Checkpoint of an IVM search stopped on its budget (Section 4.1 saves the
// explorers' work units; here every explorer's whole state, so that a
// resumed search continues exactly and counts every node once): the header,
// the best schedule, then st, lev [K] int32, V, E, D [K][n], Etop [K], M
// [K][n][n], prune bits [K][n] u64 and stored bounds [K][n][n] int32.
struct IvmCkptHeader {
  char magic[8];  // "PFSPIVM1"
  int32_t n, m, kind, ub0, ub, K, d, pad;
  uint64_t inst_hash;
  int64_t nodes, children, steps, steals;
};

struct IvmPart {
  void *dev;
  size_t bytes;
};

static std::vector<IvmPart> ivm_parts(const IvmState *S) {
  const size_t K = S->K, n = S->n;
  return {{S->st, K * 4},         {S->lev, K * 4},      {S->V, K * n},
          {S->E, K * n},          {S->D, K * n},        {S->Etop, K},
          {S->M, K * n * n},      {S->Pr, K * n * 8},   {S->LB, K * n * n * 4}};
}

static size_t ivm_ckpt_bytes(int K, int n) {
  const size_t k = K, nn = n;
  return sizeof(IvmCkptHeader) + ((nn + 7) & ~size_t(7)) + k * 8 + 3 * k * nn + k +
         k * nn * nn + k * nn * 8 + k * nn * nn * 4;
}

// The search loop shared by pfsp_search_ivm and pfsp_search_ivm_resume.
// ck: the checkpoint to continue, or null for a fresh start from ub0.
static int ivm_search(Ctx *c, int32_t ub0, int64_t budget_nodes, int lb_kind, int K,
                      const unsigned char *ck, pfsp_result *res, int64_t *steals) {
  int d = 0;
  while ((1 << (2 * d)) < K) ++d;
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  const int n = c->n;
  int rc = ensure_costs(c, K);
  if (rc) return rc;
  IvmState *S = ivm_alloc(c, K);
  if (!S) return set_err(c, PFSP_ENOMEM, "IVM buffers do not fit in device memory");
  S->d = d;
  // pools of fewer than 32768 rows: one full-scan LB2 launch costs less than
  // the depth split's second one (the option is restored on return)
  struct DeepGuard {
    Ctx *c;
    int64_t v;
    ~DeepGuard() { c->deep_r = v; }
  } dguard{c, c->deep_r};
  if (K < 32768) c->deep_r = 0;
  struct Guard {
    IvmState *S;
    ~Guard() { ivm_free(S); }
  } guard{S};
  const auto t0 = std::chrono::steady_clock::now();
  IvmCtl ctl0;
  memset(&ctl0, 0, sizeof ctl0);
  ctl0.ub = ctl0.ub_step = ub0;
  ctl0.step_best = ~0ull;
  ctl0.steps = 1;  // the number of the step under way
  if (ck) {
    IvmCkptHeader hd;
    memcpy(&hd, ck, sizeof hd);
    const unsigned char *q = ck + sizeof hd;
    PFSP_HIP(c, hipMemcpy(S->best_perm, q, n, hipMemcpyHostToDevice));
    q += (n + 7) & ~7;
    for (const IvmPart &pt : ivm_parts(S)) {
      PFSP_HIP(c, hipMemcpy(pt.dev, q, pt.bytes, hipMemcpyHostToDevice));
      q += pt.bytes;
    }
    ctl0.ub = ctl0.ub_step = hd.ub;
    ctl0.steps = hd.steps;
    ctl0.nodes = hd.nodes;
    ctl0.children = hd.children;
    ctl0.steals = hd.steals;
  } else {
    std::vector<uint8_t> V, E, Et;
    initial_units(n, K, V, E, Et);
    std::vector<int> st(K, kIvmRoot), lev(K, -1);
    PFSP_HIP(c, hipMemcpy(S->V, V.data(), V.size(), hipMemcpyHostToDevice));
    PFSP_HIP(c, hipMemcpy(S->E, E.data(), E.size(), hipMemcpyHostToDevice));
    PFSP_HIP(c, hipMemcpy(S->Etop, Et.data(), Et.size(), hipMemcpyHostToDevice));
    PFSP_HIP(c, hipMemcpy(S->st, st.data(), K * 4, hipMemcpyHostToDevice));
    PFSP_HIP(c, hipMemcpy(S->lev, lev.data(), K * 4, hipMemcpyHostToDevice));
    PFSP_HIP(c, hipMemset(S->Pr, 0, (size_t)K * n * 8));
    PFSP_HIP(c, hipMemset(S->D, 0, (size_t)K * n));
  }
  PFSP_HIP(c, hipMemcpy(S->ctl, &ctl0, sizeof ctl0, hipMemcpyHostToDevice));
  DevPool pool;
  pool.count = K;
  pool.n = n;
  pool.count_dev = &S->ctl->batch;
  pool.ub_dev = &S->ctl->ub_step;
  pool.perm = S->b_perm;
  pool.d1 = S->b_d1;
  pool.d2 = S->b_d2;
  pool.mask = nullptr;
  pool.mask_words = 0;
  pool.dir = S->b_dir;
  pool.argpair = nullptr;
  const int g = (K + 255) / 256;
  const double min_len = std::min(40320.0, 2.0 * (double)K);  // 8! or 2K positions
  const int every = (int)c->poll_every;  // steps between polls and between stealing phases
  // one step as a HIP graph (all sizes come from the control block), replayed
  // poll_every times between reads of the control block
  auto enqueue = [&]() -> int {
    hipLaunchKernelGGL(k_ivm_select, dim3(g), dim3(256), 0, S->stream, *S);
    const int r = launch_bound(c, pool, lb_kind, 0, S->out_lb, S->out_prune, S->stream);
    if (r) return r;
    hipLaunchKernelGGL(k_ivm_branch, dim3(g), dim3(256), 0, S->stream, *S, every);
    if (K <= kIvmBalLds)
      hipLaunchKernelGGL(k_ivm_balance<true>, dim3(1), dim3(kIvmBalThreads), 0, S->stream, *S,
                         min_len, every);
    else
      hipLaunchKernelGGL(k_ivm_balance<false>, dim3(1), dim3(kIvmBalThreads), 0, S->stream, *S,
                         min_len, every);
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraph_t &g;
    hipGraphExec_t &e;
    ~GraphGuard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } gguard{graph, gexec};
  if (c->use_graph) {
    PFSP_HIP(c, hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = 1;
    rc = enqueue();
    c->capturing = 0;
    const hipError_t e = hipStreamEndCapture(S->stream, &graph);
    if (rc) return rc;
    if (e != hipSuccess) return hip_err(c, e, "hipStreamEndCapture");
    PFSP_HIP(c, hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }
  int status = PFSP_OK;
  for (;;) {
    for (int t = 0; t < every; ++t) {
      if (gexec) {
        PFSP_HIP(c, hipGraphLaunch(gexec, S->stream));
      } else {
        rc = enqueue();
        if (rc) return rc;
      }
    }
    PFSP_HIP(c, hipMemcpyAsync(S->ctl_host, S->ctl, sizeof(IvmCtl), hipMemcpyDeviceToHost,
                               S->stream));
    PFSP_HIP(c, hipStreamSynchronize(S->stream));
    const IvmCtl hc = *S->ctl_host;
    if (hc.last_batch == 0) break;  // every explorer is empty: the tree is exhausted
    if (budget_nodes > 0 && hc.nodes >= budget_nodes) {
      status = PFSP_BUDGET;
      break;
    }
  }
  const IvmCtl hc = *S->ctl_host;
  c->ivm_ckpt.clear();
  if (status == PFSP_BUDGET) {  // keep the state for pfsp_search_ivm_dump
    c->ivm_ckpt.resize(ivm_ckpt_bytes(K, n));
    IvmCkptHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, "PFSPIVM1", 8);
    hd.n = n;
    hd.m = c->m;
    hd.kind = lb_kind;
    hd.ub0 = ub0;
    hd.ub = hc.ub;
    hd.K = K;
    hd.d = d;
    hd.inst_hash = instance_hash(c);
    hd.nodes = hc.nodes;
    hd.children = hc.children;
    hd.steps = hc.steps;
    hd.steals = hc.steals;
    unsigned char *q = c->ivm_ckpt.data();
    memcpy(q, &hd, sizeof hd);
    q += sizeof hd;
    PFSP_HIP(c, hipMemcpy(q, S->best_perm, n, hipMemcpyDeviceToHost));
    q += (n + 7) & ~7;
    for (const IvmPart &pt : ivm_parts(S)) {
      PFSP_HIP(c, hipMemcpy(q, pt.dev, pt.bytes, hipMemcpyDeviceToHost));
      q += pt.bytes;
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  res->found = hc.ub < ub0;
  res->best_cmax = res->found ? hc.ub : ub0;
  res->proven = status == PFSP_OK;
  res->steps = (int)hc.steps - 1;
  res->nodes_decomposed = hc.nodes;
  res->children_bounded = hc.children;
  res->max_pool = K;
  res->seconds = std::chrono::duration<double>(t1 - t0).count();
  if (steals) *steals = hc.steals;
  if (res->found && res->best_perm) {
    uint8_t tmp[kMaxN];
    PFSP_HIP(c, hipMemcpy(tmp, S->best_perm, n, hipMemcpyDeviceToHost));
    for (int j = 0; j < n; ++j) res->best_perm[j] = tmp[j];
  }
  return status;
}


}  // namespace
}  // namespace pfsp

extern "C" int pfsp_search_ivm(pfsp_ctx *h, int32_t ub0, int64_t budget_nodes, int lb_kind,
                               int32_t explorers, pfsp_result *res, int64_t *steals) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!res) return set_err(c, PFSP_EINVAL, "res is NULL");
  if (lb_kind != PFSP_LB1 && lb_kind != PFSP_LB2_FULL)
    return set_err(c, PFSP_EINVAL, "IVM search takes PFSP_LB1 or PFSP_LB2_FULL");
  if (lb_kind != PFSP_LB1 && c->m < 2) return set_err(c, PFSP_ERANGE, "LB2 kinds need m >= 2");
  if (c->n > kIvmMaxN) return set_err(c, PFSP_ERANGE, "IVM search covers n <= 64");
  if (budget_nodes < 0) return set_err(c, PFSP_EINVAL, "negative budget");
  int d = 0;
  while ((1 << (2 * d)) < explorers) ++d;
  if (explorers < 1 || (1 << (2 * d)) != explorers || explorers > (1 << 20))
    return set_err(c, PFSP_ERANGE, "explorers must be a power of 4 in [1, 4^10]");
  return ivm_search(c, ub0, budget_nodes, lb_kind, explorers, nullptr, res, steals);
}

extern "C" int pfsp_search_ivm_dump(pfsp_ctx *h, void *buf, int64_t cap, int64_t *size) {
  if (!h || !size) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->ivm_ckpt.empty())
    return set_err(c, PFSP_EINVAL, "no IVM search stopped on its budget to dump");
  *size = (int64_t)c->ivm_ckpt.size();
  if (!buf) return PFSP_OK;
  if (cap < *size) return set_err(c, PFSP_ERANGE, "checkpoint buffer too small");
  memcpy(buf, c->ivm_ckpt.data(), c->ivm_ckpt.size());
  return PFSP_OK;
}

extern "C" int pfsp_search_ivm_resume(pfsp_ctx *h, const void *buf, int64_t size,
                                      int64_t budget_nodes, pfsp_result *res, int64_t *steals) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (!buf || !res || budget_nodes < 0) return set_err(c, PFSP_EINVAL, "bad arguments");
  IvmCkptHeader hd;
  if (size < (int64_t)sizeof hd) return set_err(c, PFSP_EINVAL, "not an IVM checkpoint");
  memcpy(&hd, buf, sizeof hd);
  if (memcmp(hd.magic, "PFSPIVM1", 8) != 0) return set_err(c, PFSP_EINVAL, "not an IVM checkpoint");
  if (hd.n != c->n || hd.m != c->m || hd.inst_hash != instance_hash(c))
    return set_err(c, PFSP_EINVAL, "checkpoint of another instance");
  if (hd.K < 1 || hd.K > (1 << 20) || (hd.K & (hd.K - 1)) != 0 ||
      (hd.kind != PFSP_LB1 && hd.kind != PFSP_LB2_FULL) ||
      size != (int64_t)ivm_ckpt_bytes(hd.K, hd.n))
    return set_err(c, PFSP_EINVAL, "malformed IVM checkpoint");
  // copy first: a budget stop of this run replaces the context's checkpoint
  std::vector<unsigned char> ck((const unsigned char *)buf, (const unsigned char *)buf + size);
  return ivm_search(c, hd.ub0, budget_nodes, hd.kind, hd.K, ck.data(), res, steals);
}

// Host checks of the work-unit arithmetic and the decoding.
extern "C" int pfsp_factoradic(int op, int32_t n, const uint8_t *a, int32_t atop,
                               const uint8_t *b, int32_t btop, uint8_t *out, int32_t *out_top) {
  if (n < 1 || n > kIvmMaxN || !a || !out || !out_top) return PFSP_EINVAL;
  for (int L = 0; L < n; ++L)
    if (a[L] >= n - L || (b && b[L] >= n - L)) return PFSP_ERANGE;
  uint8_t t[kIvmMaxN];
  switch (op) {
    case 0:  // a + b
      if (!b) return PFSP_EINVAL;
      *out_top = fact_add(n, a, atop, b, btop, t);
      break;
    case 1:  // b - a
      if (!b || fact_cmp(n, b, btop, a, atop) < 0) return PFSP_EINVAL;
      *out_top = fact_sub(n, b, btop, a, atop, t);
      break;
    case 2:  // floor(a / 2)
      memcpy(t, a, n);
      fact_half(n, t, atop);
      *out_top = 0;
      break;
    case 3:  // a + (b - a) / 2, the midpoint of a work unit [a, b)
      if (!b || fact_cmp(n, b, btop, a, atop) < 0) return PFSP_EINVAL;
      {
        const int top = fact_sub(n, b, btop, a, atop, t);
        fact_half(n, t, top);
        *out_top = fact_add(n, a, atop, t, 0, t);
      }
      break;
    default:
      return PFSP_EINVAL;
  }
  memcpy(out, t, n);
  return PFSP_OK;
}

extern "C" int pfsp_ivm_decode(int32_t n, const uint8_t *M, const uint8_t *V, const uint8_t *D,
                               int32_t level, uint8_t *perm_out, int32_t *d1, int32_t *d2) {
  if (n < 2 || n > kIvmMaxN || !M || !V || !D || !perm_out || !d1 || !d2) return PFSP_EINVAL;
  if (level < 0 || level >= n) return PFSP_ERANGE;
  for (int L = 0; L <= level; ++L)
    if (V[L] >= n - L) return PFSP_ERANGE;
  int a, b;
  ivm_decode(n, M, V, D, level, perm_out, &a, &b);
  *d1 = a;
  *d2 = b;
  return PFSP_OK;
}
