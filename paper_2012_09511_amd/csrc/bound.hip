// Bounding, MinMin branching and pruning of a batch of parents (Sections
// 2.3-2.4 and the decomposition step of Section 3.3).
//
// k_lb1: one lane per parent.  Computes the parent's front C1 (completion
//   times of sigma1 on every machine, Eq. (1)), back C2 (sigma2 scheduled in
//   reverse on reversed machines) and remaining work R = T - scheduled work.
//   In LB1 mode it then derives every child's LB1 in O(m) (Section 2.4:
//   the incremental evaluation of the 2(n-d) children):
//     forward child j:  C1'[k] = max(C1'[k-1], C1[k]) + p[j][k],
//                       LB = max_k C1'[k] + R[k] - p[j][k] + C2[k]
//     backward child j: C2'[k] = max(C2'[k+1], C2[k]) + p[j][k],
//                       LB = max_k C1[k] + R[k] - p[j][k] + C2'[k]
//   followed by MinMin and the prune flags.  In LB2 mode it only writes
//   (C1, C2, R) to the workspace for k_lb2.
//
// k_lb2: one wave per parent, lanes = machine pairs (64 per pass).  For a
//   pair (u, v) the two-machine value of a child whose unscheduled set is
//   U \ {j}, with heads h and tails t, is
//     t_u = h_u + A(U\j),  t_v = max(h_v + B(U\j), h_u + max_i term_i(U\j)),
//     value = max(t_u + t_u', t_v + t_v'),
//   where A, B sum a = p[.][u], b = p[.][v] and term_i = A(<= i) + lag_i + B(>= i)
//   along the pair's Johnson order.  Removing j lowers the terms before j by
//   b_j and those after j by a_j, so with the parent's exclusive prefix and
//   suffix maxima PM, SM of term over U:
//     max_i term_i(U\j) = max(PM(j) - b_j, SM(j) - a_j).
//   Two scans per (parent, pair) produce X(j) = that maximum for every j in
//   U; each child then costs O(1) per pair.  The result is exactly the value
//   of running the Johnson recurrence over the child's jobs (proof: the
//   recurrence unrolls to max(h_v + B, h_u + max_i term_i)).  The maxima over
//   pairs are kept per child in registers and reduced across lanes by a
//   transposing exchange at the end.
#include <type_traits>

#include "internal.h"
#include "wave.h"

namespace pfsp {

namespace {

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct Narrow {
  using T = uint2;
  __device__ __forceinline__ static void get(const uint2 e, int &a, int &b, int &l, int &k) {
    a = (int)(e.x & 0xffffu);
    b = (int)(e.x >> 16);
    l = (int)(e.y & 0xffffffu);
    k = (int)(e.y >> 24);
  }
};
struct Wide {
  using T = uint4;
  __device__ __forceinline__ static void get(const uint4 e, int &a, int &b, int &l, int &k) {
    a = (int)e.x;
    b = (int)e.y;
    l = (int)e.z;
    k = (int)e.w;
  }
};

// Slots q >= from of both directions of a row of 2 * n entries: INT32_MAX,
// pruned, no argmax pair.
// The pair-mask row of pool row par (a shared row when mask_stride is 0).
__device__ __forceinline__ const uint32_t *mask_row(const DevPool &pool, int par) {
  return pool.mask +
         (size_t)par * (size_t)(pool.mask_stride >= 0 ? pool.mask_stride : pool.mask_words);
}

__device__ __forceinline__ void fill_invalid(int *lbrow, uint8_t *prow, int16_t *arow, int n,
                                             int from, int lane, int step) {
  for (int x = lane; x < 2 * n; x += step) {
    const int q = x < n ? x : x - n;
    if (q >= from) {
      lbrow[x] = kInt32Max;
      prow[x] = 1;
      if (arow) arow[x] = -1;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- LB1 / costs
// One parent (one lane): validity check, front/back/remaining, and in LB1 mode
// every child's LB1 plus MinMin and prune flags.  pmat: p[n][m] (LDS or
// global); C1/C2/R: per-lane scratch with stride B; rows of the pool and the
// outputs have stride ns >= n.
__device__ __forceinline__ void lb1_row(const DevInst &I, const int *__restrict__ pmat, int *C1,
                                        int *C2, int *R, int B, const uint8_t *__restrict__ row,
                                        int a, int b, int ns, int ub, int *__restrict__ lbrow,
                                        uint8_t *__restrict__ prow, int16_t *__restrict__ arow,
                                        uint8_t *__restrict__ dirp, int *__restrict__ cs,
                                        int write_out, int *__restrict__ flag) {
  const int n = I.n, m = I.m;
  const int r = n - a - b;
  // a row must be a permutation of 0..n-1 with d1 + d2 < n
  bool bad = r < 1;
  uint32_t seen[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int x = 0; x < n && !bad; ++x) {
    const int j = row[x];
    const uint32_t bit = 1u << (j & 31);
    if (j >= n || (seen[j >> 5] & bit)) bad = true;
    seen[j >> 5] |= bit;
  }
  if (bad) {
    flag[0] = 1;
    if (write_out) {  // in costs mode the LB2 kernel fills the outputs of this row
      fill_invalid(lbrow, prow, arow, ns, 0, 0, 1);
      if (dirp) *dirp = 0;
    }
    if (cs) {
      for (int k = 0; k < 3 * m; ++k) cs[k] = 0;
      cs[0] = -1;  // marks the row invalid for the LB2 kernels
    }
    return;
  }
  for (int k = 0; k < m; ++k) {
    C1[k * B] = 0;
    C2[k * B] = 0;
    R[k * B] = I.T[k];
  }
  for (int x = 0; x < a; ++x) {  // front of sigma1, Eq. (1)
    const int *pj = pmat + row[x] * m;
    int c = 0;
    for (int k = 0; k < m; ++k) {
      c = max(c, C1[k * B]) + pj[k];
      C1[k * B] = c;
      R[k * B] -= pj[k];
    }
  }
  for (int x = n - 1; x >= n - b; --x) {  // back of sigma2: reverse jobs, reverse machines
    const int *pj = pmat + row[x] * m;
    int c = 0;
    for (int k = m - 1; k >= 0; --k) {
      c = max(c, C2[k * B]) + pj[k];
      C2[k * B] = c;
      R[k * B] -= pj[k];
    }
  }
  if (cs) {
    for (int k = 0; k < m; ++k) {
      cs[k] = C1[k * B];
      cs[m + k] = C2[k * B];
      cs[2 * m + k] = R[k * B];
    }
  }
  if (!write_out) return;
  MinMin mm;
  mm.init();
  for (int q = 0; q < r; ++q) {
    const int *pj = pmat + row[a + q] * m;
    int c = 0, lbf = 0;
    for (int k = 0; k < m; ++k) {
      c = max(c, C1[k * B]) + pj[k];
      lbf = max(lbf, c + R[k * B] - pj[k] + C2[k * B]);
    }
    c = 0;
    int lbb = 0;
    for (int k = m - 1; k >= 0; --k) {
      c = max(c, C2[k * B]) + pj[k];
      lbb = max(lbb, C1[k * B] + R[k * B] - pj[k] + c);
    }
    lbrow[q] = lbf;
    lbrow[ns + q] = lbb;
    prow[q] = lbf >= ub;
    prow[ns + q] = lbb >= ub;
    mm.add(lbf, false);
    mm.add(lbb, true);
  }
  for (int q = r; q < ns; ++q) {
    lbrow[q] = kInt32Max;
    lbrow[ns + q] = kInt32Max;
    prow[q] = 1;
    prow[ns + q] = 1;
  }
  if (dirp) *dirp = (uint8_t)mm.dir();
}

// Filter outcome of pool row i (see CostFilter): closed rows get their prune
// row and direction here, open rows are appended to the list (one atomic per
// wave).  Whole waves call it.
__device__ __forceinline__ void list_append(int *rows, int *count, bool app, int i, int lane) {
  const uint64_t bal = __ballot(app);
  int base = 0;
  if (bal) {
    if (lane == 0) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, 0, kWave);
  }
  if (app) {
    const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
    rows[base + pos] = i;
  }
}

// r: the row's jobs left (deep: 1 <= r <= f.deep_r; the LB1 band: 1 <= r <=
// f.lb1_r, which takes precedence).
__device__ __forceinline__ void filter_row(const CostFilter &f, int i, bool live, bool open,
                                           int r, int ns, int lane) {
  const bool app = live && open;
  const bool to_lb1 = app && f.rows_lb1 != nullptr && r >= 1 && r <= f.lb1_r;
  const bool to_deep = app && !to_lb1 && f.rows_deep != nullptr && r >= 1 && r <= f.deep_r;
  list_append(f.rows, f.open, app && !to_deep && !to_lb1, i, lane);
  if (f.rows_deep) list_append(f.rows_deep, f.open_deep, to_deep, i, lane);
  if (f.rows_lb1) list_append(f.rows_lb1, f.open_lb1, to_lb1, i, lane);
  if (!app && live) {
    uint8_t *pr = f.out_prune + (size_t)i * 2 * ns;
    for (int x = 0; x < 2 * ns; ++x) pr[x] = 1;
    if (f.dir) f.dir[i] = 0;
  }
}

__global__ void __launch_bounds__(128)
k_lb1(DevInst I, DevPool pool, int ub, int *__restrict__ out_lb, uint8_t *__restrict__ out_prune,
      int *__restrict__ costs, int write_out, int *__restrict__ flag, CostFilter f) {
  extern __shared__ int sh[];
  const int n = I.n, m = I.m, B = blockDim.x, t = threadIdx.x;
  int *sp = sh;  // p[n][m]
  for (int x = t; x < n * m; x += B) sp[x] = I.p[x];
  __syncthreads();
  const int it = blockIdx.x * B + t;
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const bool filt = f.rows != nullptr;  // costs mode only (every row, no index)
  if (it >= count && !filt) return;
  // launch row it bounds pool row i
  const int i = !filt && pool.index && it < count ? pool.index[it] : it;
  if (pool.ub_dev) ub = *pool.ub_dev;
  int *C1 = sh + n * m + t;  // per-lane arrays, stride B (bank-conflict free)
  const int ns = pool.n;     // row stride of the pool and the outputs (>= n)
  bool live = false, open = false;
  int rj = 0;  // jobs left
  if (it < count) {
    live = !filt || !f.alive || f.alive[i];
    const uint8_t *row = pool.perm + (size_t)i * ns;
    const int a = pool.d1[i], b = pool.d2[i];
    rj = n - a - b;
    int *cs = costs ? costs + (size_t)i * 3 * m : nullptr;
    lb1_row(I, sp, C1, C1 + m * B, C1 + 2 * m * B, B, row, a, b, ns, ub,
            write_out ? out_lb + (size_t)i * 2 * ns : nullptr,
            write_out ? out_prune + (size_t)i * 2 * ns : nullptr,
            write_out && pool.argpair ? pool.argpair + (size_t)i * 2 * ns : nullptr,
            write_out && pool.dir ? pool.dir + i : nullptr, cs, write_out, flag);
    if (filt && live && cs[0] >= 0) {
      // children's LB1 from the state lb1_row left in the lane's arrays
      const int fub = *f.ub_dev;
      const int *C2 = C1 + m * B, *R = C1 + 2 * m * B;
      for (int x = a; x < n - b && !open; ++x) {
        const int *pj = sp + row[x] * m;
        int c = 0, lf = 0;
        for (int k = 0; k < m; ++k) {
          c = max(c, C1[k * B]) + pj[k];
          lf = max(lf, c + R[k * B] - pj[k] + C2[k * B]);
        }
        int d = 0, lb = 0;
        for (int k = m - 1; k >= 0; --k) {
          d = max(d, C2[k * B]) + pj[k];
          lb = max(lb, C1[k * B] + R[k * B] - pj[k] + d);
        }
        open = lf < fub || lb < fub;
      }
    }
  }
  if (filt) filter_row(f, i, live, open, rj, ns, t & 63);
}

// One parent's costs (front C1, back C2, remaining R; Eq. (1)) for n <= NJ
// (32 or 64) and m <= MMAX, written to cs[0 .. 3m); an invalid row (not a
// permutation of 0..n-1, or d1 + d2 >= n) sets *flag and gets cs = {-1, 0,
// ...}.  The row and the per-machine state stay in registers; sp holds p
// zero-padded to MMAX machines (row stride MS) so that the machine loops need
// no bounds.  *valid reports whether the row is a valid node.  With check,
// returns whether some child (either direction) has LB1 < ub (the children's
// LB1 of Section 2.4 from the same state; padded machines add nothing);
// without check, returns whether the row is valid.
template <int MMAX, int MS, int NJ = 32>
__device__ __forceinline__ bool costs_row(int n, int m, const int *__restrict__ sp,
                                          const int *__restrict__ sT,
                                          const uint8_t *__restrict__ row, int a, int b,
                                          int *__restrict__ cs, int *__restrict__ flag,
                                          bool check, int ub, bool *valid) {
  constexpr int NWD = NJ / 4;
  uint32_t rw[NWD];
#pragma unroll
  for (int w = 0; w < NWD; ++w) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * w + q < n) v |= (uint32_t)row[4 * w + q] << (8 * q);
    rw[w] = v;
  }
  uint64_t seen = 0;
  bool bad = a + b >= n;
#pragma unroll
  for (int x = 0; x < NJ; ++x) {
    if (x < n) {
      const uint32_t j = (rw[x >> 2] >> (8 * (x & 3))) & 0xffu;
      seen |= 1ull << (j & 63u);
      bad |= j >= (uint32_t)n;
    }
  }
  bad |= seen != (n == 64 ? ~0ull : (1ull << n) - 1ull);
  *valid = !bad;
  if (bad) {
    flag[0] = 1;
    for (int k = 0; k < 3 * m; ++k) cs[k] = 0;
    cs[0] = -1;  // marks the row invalid for the LB2 kernels
    return false;
  }
  int C1[MMAX], C2[MMAX], R[MMAX];
#pragma unroll
  for (int k = 0; k < MMAX; ++k) {
    C1[k] = 0;
    C2[k] = 0;
    R[k] = sT[k];
  }
#pragma unroll
  for (int x = 0; x < NJ; ++x) {  // front of sigma1
    if (x < a) {
      const int *pj = sp + (int)((rw[x >> 2] >> (8 * (x & 3))) & 0xffu) * MS;
      int c = 0;
#pragma unroll
      for (int k = 0; k < MMAX; ++k) {
        const int q = pj[k];
        c = max(c, C1[k]) + q;
        C1[k] = c;
        R[k] -= q;
      }
    }
  }
#pragma unroll
  for (int x = NJ - 1; x >= 0; --x) {  // back of sigma2: jobs and machines reversed
    if (x < n && x >= n - b) {
      const int *pj = sp + (int)((rw[x >> 2] >> (8 * (x & 3))) & 0xffu) * MS;
      int c = 0;
#pragma unroll
      for (int k = MMAX - 1; k >= 0; --k) {
        const int q = pj[k];
        c = max(c, C2[k]) + q;
        C2[k] = c;
        R[k] -= q;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MMAX; ++k) {
    if (k < m) {
      cs[k] = C1[k];
      cs[m + k] = C2[k];
      cs[2 * m + k] = R[k];
    }
  }
  if (!check) return true;
  bool open = false;
#pragma unroll
  for (int x = 0; x < NJ; ++x) {
    if (x >= a && x < n - b && !open) {
      const int *pj = sp + (int)((rw[x >> 2] >> (8 * (x & 3))) & 0xffu) * MS;
      int c = 0, lf = 0;
#pragma unroll
      for (int k = 0; k < MMAX; ++k) {  // child with the job appended to sigma1
        c = max(c, C1[k]) + pj[k];
        lf = max(lf, c + R[k] - pj[k] + C2[k]);
      }
      int d = 0, lb = 0;
#pragma unroll
      for (int k = MMAX - 1; k >= 0; --k) {  // child with the job prepended to sigma2
        d = max(d, C2[k]) + pj[k];
        lb = max(lb, C1[k] + R[k] - pj[k] + d);
      }
      open = lf < ub || lb < ub;
    }
  }
  return open;
}

// Parent costs for n <= 32 and m <= MMAX (the values of k_lb1 in costs mode),
// one lane per parent.  p is staged in LDS with an odd row stride, so that
// lanes reading different jobs hit different banks.  The 64 rows of a wave
// are contiguous in the workspace: each lane writes its row into the wave's
// LDS tile and the wave then stores the tile with consecutive lanes on
// consecutive words (whole cache lines rather than scattered words).
template <int MMAX, int NJ = 32>
__global__ void __launch_bounds__(256)
k_costs(DevInst I, DevPool pool, int *__restrict__ costs, int *__restrict__ flag, CostFilter f) {
  extern __shared__ int sh[];
  constexpr int MS = MMAX | 1;
  const int n = I.n, m = I.m, cm = 3 * m;
  const int RS = cm + 1;   // tile row stride (odd: the lanes' row writes spread over banks)
  int *sp = sh;            // [n][MS]
  int *sT = sh + n * MS;   // [MMAX] per-machine totals
  const int lane = threadIdx.x & 63;
  int *tile = sT + MMAX + (threadIdx.x >> 6) * 64 * RS;  // this wave's [64][RS]
  for (int x = threadIdx.x; x < n * MS; x += blockDim.x) {
    const int j = x / MS, k = x - j * MS;
    sp[x] = k < m ? I.p[j * m + k] : 0;
  }
  for (int x = threadIdx.x; x < MMAX; x += blockDim.x) sT[x] = x < m ? I.T[x] : 0;
  __syncthreads();
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int ns = pool.n;
  const bool filt = f.rows != nullptr;
  const int ub = filt ? *f.ub_dev : 0;
  // whole waves step together: the tile store is a wave-wide operation
  for (int i0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63); i0 < count;
       i0 += gridDim.x * blockDim.x) {
    const int i = i0 + lane;
    bool live = false, open = false, valid = false;
    int rj = 0;  // jobs left
    if (i < count) {
      live = !filt || !f.alive || f.alive[i];
      const int a = pool.d1[i], b = pool.d2[i];
      open = costs_row<MMAX, MS, NJ>(n, m, sp, sT, pool.perm + (size_t)i * ns, a, b,
                                 tile + lane * RS, flag, filt && live, ub, &valid);
      open = open && valid;
      rj = n - a - b;
    }
    if (filt) filter_row(f, i, live, open, rj, ns, lane);
    wave_sync();
    const int rows = min(64, count - i0);
    int *dst = costs + (size_t)i0 * cm;
    for (int x = lane; x < rows * cm; x += 64) {
      const int r = x / cm;
      dst[x] = tile[r * RS + (x - r * cm)];
    }
    wave_sync();
  }
}

// Several instances: parent i belongs to the instance k with
// seg[k] <= i < seg[k + 1]; p is read from global memory (cached); costs rows
// have stride 3 * mmax.
__global__ void __launch_bounds__(128)
k_lb1m(const DevInst *__restrict__ insts, const long long *__restrict__ seg, int ninst,
       const uint8_t *__restrict__ perm, const uint8_t *__restrict__ d1,
       const uint8_t *__restrict__ d2, int stride, int mmax, const int *__restrict__ ubs,
       int *__restrict__ out_lb, uint8_t *__restrict__ out_prune, uint8_t *__restrict__ dir,
       int *__restrict__ costs, int write_out, int *__restrict__ flag) {
  extern __shared__ int sh[];
  const int B = blockDim.x, t = threadIdx.x;
  const long long i = (long long)blockIdx.x * B + t;
  if (i >= seg[ninst]) return;
  int lo = 0, hi = ninst;  // seg[lo] <= i < seg[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid;
  }
  const DevInst I = insts[lo];
  int *C1 = sh + t;
  lb1_row(I, I.p, C1, C1 + mmax * B, C1 + 2 * mmax * B, B, perm + (size_t)i * stride, d1[i],
          d2[i], stride, ubs[lo], write_out ? out_lb + (size_t)i * 2 * stride : nullptr,
          write_out ? out_prune + (size_t)i * 2 * stride : nullptr, nullptr,
          write_out ? dir + i : nullptr, costs ? costs + (size_t)i * 3 * mmax : nullptr,
          write_out, flag);
}

// Costs only (the LB2 kinds of the multi-instance launch) for n <= 128 and
// m <= MMAX: k_lb1m's values with the block's pool rows (one contiguous
// range) copied to LDS by whole words, the block's instance's p staged in
// LDS (odd row stride) when all its parents belong to one instance, which the
// grouping by instance makes the common case, and the three cost vectors in
// registers.  A block that straddles two instances reads p from global
// memory.
template <int MMAX>
__global__ void __launch_bounds__(128)
k_costsm(const DevInst *__restrict__ insts, const long long *__restrict__ seg, int ninst,
         const uint8_t *__restrict__ perm, const uint8_t *__restrict__ d1,
         const uint8_t *__restrict__ d2, int stride, int mmax, int *__restrict__ costs,
         int *__restrict__ flag) {
  extern __shared__ int sh[];
  constexpr int MS = MMAX | 1, B = 128;
  const int t = threadIdx.x;
  const long long total = seg[ninst];
  const long long b0 = (long long)blockIdx.x * B;
  const int rows = (int)min((long long)B, total - b0);
  auto inst_of = [&](long long x) {  // seg[k] <= x < seg[k + 1]
    int lo = 0, hi = ninst;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (seg[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
  };
  const int k0 = inst_of(b0);
  const bool staged = inst_of(b0 + rows - 1) == k0;  // uniform
  int *sp = sh;                                       // [128][MS] p of instance k0
  uint8_t *srow = (uint8_t *)(sh + 128 * MS);         // [B][stride] the block's rows
  if (staged) {
    const DevInst I0 = insts[k0];
    for (int x = t; x < I0.n * MS; x += B) {
      const int j = x / MS, k = x - j * MS;
      sp[x] = k < I0.m ? I0.p[j * I0.m + k] : 0;
    }
  }
  {  // rows b0 .. b0 + rows: whole words (the range starts 4-byte aligned), then the tail
    const size_t bytes = (size_t)rows * stride;
    const uint8_t *src = perm + (size_t)b0 * stride;
    const size_t words = ((uintptr_t)src & 3u) ? 0 : bytes >> 2;
    for (size_t x = t; x < words; x += B) ((uint32_t *)srow)[x] = ((const uint32_t *)src)[x];
    for (size_t x = words * 4 + t; x < bytes; x += B) srow[x] = src[x];
  }
  __syncthreads();
  if (t >= rows) return;
  const long long i = b0 + t;
  const int k = staged ? k0 : inst_of(i);
  const DevInst I = insts[k];
  const int n = I.n, m = I.m;
  const int *pm = staged ? sp : I.p;
  const int ps = staged ? MS : m;
  const uint8_t *row = srow + (size_t)t * stride;
  const int a = d1[i], b = d2[i];
  int *cs = costs + (size_t)i * 3 * mmax;
  // a row must be a permutation of 0..n-1 with d1 + d2 < n
  uint64_t s0 = 0, s1 = 0;
  bool bad = a + b >= n;
  for (int x = 0; x < n; ++x) {
    const unsigned j = row[x];
    bad |= j >= (unsigned)n;
    const uint64_t bit = 1ull << (j & 63u);
    s0 |= j < 64 ? bit : 0ull;
    s1 |= j >= 64 ? bit : 0ull;
  }
  bad |= s0 != (n >= 64 ? ~0ull : (1ull << n) - 1ull) ||
         s1 != (n > 64 ? (n == 128 ? ~0ull : (1ull << (n - 64)) - 1ull) : 0ull);
  if (bad) {
    flag[0] = 1;
    for (int q = 0; q < 3 * m; ++q) cs[q] = 0;
    cs[0] = -1;  // marks the row invalid for the LB2 kernels
    return;
  }
  int C1[MMAX], C2[MMAX], R[MMAX];
#pragma unroll
  for (int q = 0; q < MMAX; ++q) {
    C1[q] = 0;
    C2[q] = 0;
    R[q] = q < m ? I.T[q] : 0;
  }
  for (int x = 0; x < a; ++x) {  // front of sigma1, Eq. (1)
    const int *pj = pm + row[x] * ps;
    int c = 0;
#pragma unroll
    for (int q = 0; q < MMAX; ++q) {
      if (q < m) {
        const int v = pj[q];
        c = max(c, C1[q]) + v;
        C1[q] = c;
        R[q] -= v;
      }
    }
  }
  for (int x = n - 1; x >= n - b; --x) {  // back of sigma2: jobs and machines reversed
    const int *pj = pm + row[x] * ps;
    int c = 0;
#pragma unroll
    for (int q = MMAX - 1; q >= 0; --q) {
      if (q < m) {
        const int v = pj[q];
        c = max(c, C2[q]) + v;
        C2[q] = c;
        R[q] -= v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < MMAX; ++q) {
    if (q < m) {
      cs[q] = C1[q];
      cs[m + q] = C2[q];
      cs[2 * m + q] = R[q];
    }
  }
}

// ------------------------------------------------------------------------ LB2
template <class E, bool ENT_LDS, bool SUBSET, bool LOG>
__global__ void __launch_bounds__(512)
k_lb2(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
      uint8_t *__restrict__ out_prune, int xrows) {
  extern __shared__ __align__(16) unsigned char sm[];
  using ET = typename E::T;
  const int n = I.n, m = I.m, P = I.P;
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  if ((int)blockIdx.x * nw >= (pool.count_dev ? *pool.count_dev : pool.count)) return;
  const ET *ent_g = (const ET *)(I.narrow ? (const void *)I.ent : (const void *)I.entw);
  size_t off = 0;
  ET *ent_s = (ET *)sm;
  if (ENT_LDS) off += align16((size_t)n * P * sizeof(ET));
  int *sp = (int *)(sm + off);
  off += align16((size_t)n * m * 4);
  const size_t per_wave = align16((size_t)xrows * 64 * 8) + align16((size_t)xrows * m * 8) +
                          align16((size_t)3 * m * 4) + align16((size_t)2 * n * 4);
  unsigned char *wb = sm + off + w * per_wave;
  int2 *X = (int2 *)wb;  // [xrows][64]: per child slot, per lane (pair)
  wb += align16((size_t)xrows * 64 * 8);
  int2 *FB = (int2 *)wb;  // [xrows][m]: (fwd child front - p, bwd child back - p)
  wb += align16((size_t)xrows * m * 8);
  int *c1 = (int *)wb, *c2 = c1 + m, *rr = c2 + m;
  wb += align16((size_t)3 * m * 4);
  int *slot = (int *)wb, *jobs = slot + n;

  if (ENT_LDS)
    for (int x = threadIdx.x; x < n * P; x += blockDim.x) ent_s[x] = ent_g[x];
  for (int x = threadIdx.x; x < n * m; x += blockDim.x) sp[x] = I.p[x];
  __syncthreads();
  const ET *ent = ENT_LDS ? ent_s : ent_g;
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if (pool.ub_dev) ub = *pool.ub_dev;

  const int ns = pool.n;  // row stride of the pool and the outputs (>= n)
  for (int it = blockIdx.x * nw + w; it < count; it += gridDim.x * nw) {
    const int par = pool.index ? pool.index[it] : it;
    const int a = pool.d1[par], b = pool.d2[par], r = n - a - b;
    int *lbrow = out_lb + (size_t)par * 2 * ns;
    uint8_t *prow = out_prune + (size_t)par * 2 * ns;
    int16_t *arow = LOG ? pool.argpair + (size_t)par * 2 * ns : nullptr;
    // rows that are not valid nodes were flagged by k_lb1 (a front value is
    // never negative otherwise): every slot gets INT32_MAX / prune 1
    if (r < 1 || costs[(size_t)par * 3 * m] < 0) {
      fill_invalid(lbrow, prow, arow, ns, 0, lane, 64);
      if (pool.dir && lane == 0) pool.dir[par] = 0;
      continue;
    }
    for (int x = lane; x < n; x += 64) {
      jobs[x] = pool.perm[(size_t)par * ns + x];
      slot[x] = -1;
    }
    for (int x = lane; x < m; x += 64) {
      const int *cs = costs + (size_t)par * 3 * m;
      c1[x] = cs[x];
      c2[x] = cs[m + x];
      rr[x] = cs[2 * m + x];
    }
    wave_sync();
    for (int x = lane; x < r; x += 64) slot[jobs[a + x]] = x;
    wave_sync();
    MinMin mm;
    mm.init();
    for (int cb = 0; cb < r; cb += 32) {
      const int nq = min(32, r - cb);
      // children fronts/backs of this chunk: lanes [0,32) forward, [32,64) backward
      int lb1 = kNeg;
      const int ql = lane & 31;
      if (ql < nq) {
        const int *pj = sp + jobs[a + cb + ql] * m;
        int c = 0, l = 0;
        if (lane < 32) {
          for (int k = 0; k < m; ++k) {
            c = max(c, c1[k]) + pj[k];
            FB[ql * m + k].x = c - pj[k];
            l = max(l, c + rr[k] - pj[k] + c2[k]);
          }
        } else {
          for (int k = m - 1; k >= 0; --k) {
            c = max(c, c2[k]) + pj[k];
            FB[ql * m + k].y = c - pj[k];
            l = max(l, c1[k] + rr[k] - pj[k] + c);
          }
        }
        lb1 = l;
      }
      wave_sync();
      int acc[64];
      int arg[LOG ? 64 : 1];
#pragma unroll
      for (int q = 0; q < 64; ++q) acc[q] = kNeg;
      if (LOG) {
#pragma unroll
        for (int q = 0; q < 64; ++q) arg[LOG ? q : 0] = 0x7fffffff;
      }
      for (int pc = 0; pc < P; pc += 64) {
        const int pi = pc + lane;
        bool act = pi < P;
        if (SUBSET && act)
          act = (mask_row(pool, par)[pi >> 5] >> (pi & 31)) & 1u;
        if (act) {
          const int u = I.pu[pi], v = I.pv[pi];
          const int RU = rr[u], RV = rr[v], C1u = c1[u], C1v = c1[v], C2u = c2[u], C2v = c2[v];
          // forward scan: exclusive prefix maximum of term (minus B(U)), minus b_j
          int Y = 0, Pm = kNeg;
          for (int i = 0; i < n; ++i) {
            int ea, eb, el, ek;
            E::get(ent[(size_t)i * P + pi], ea, eb, el, ek);
            const int s = slot[ek];
            if (s >= 0) {
              Y += ea;
              const int tt = Y + el;
              const int sq = s - cb;
              if ((unsigned)sq < (unsigned)nq) X[sq * 64 + lane].x = Pm - eb;
              Pm = max(Pm, tt);
              Y -= eb;
            }
          }
          // backward scan: exclusive suffix maximum, combined into X(j)
          const int c0 = RU - RV;
          int Wb = 0, Sm = kNeg;
          for (int i = n - 1; i >= 0; --i) {
            int ea, eb, el, ek;
            E::get(ent[(size_t)i * P + pi], ea, eb, el, ek);
            const int s = slot[ek];
            if (s >= 0) {
              Wb += eb;
              const int tp = Wb + el + c0;
              const int sq = s - cb;
              if ((unsigned)sq < (unsigned)nq) {
                const int x = max(X[sq * 64 + lane].x, Sm - ea);
                X[sq * 64 + lane] = make_int2(x + ea, x + eb);
              }
              Sm = max(Sm, tp);
              Wb -= ea;
            }
          }
          const int K1 = RU + C2u, K2 = C1u + RU, K3 = C1v + RV;
#pragma unroll
          for (int q = 0; q < 32; ++q) {
            if (q < nq) {
              const int2 xab = X[q * 64 + lane];
              const int2 fu = FB[q * m + u], fv = FB[q * m + v];
              const int xa = xab.x + RV, xb = xab.y + RV;
              const int lbf = max(fu.x + K1, max(fv.x + RV, fu.x + xa) + C2v);
              const int lbb = max(fu.y + K2, max(K3, C1u + xb) + fv.y);
              if (LOG) {
                if (lbf > acc[q]) { acc[q] = lbf; arg[LOG ? q : 0] = pi; }
                if (lbb > acc[32 + q]) { acc[32 + q] = lbb; arg[LOG ? 32 + q : 0] = pi; }
              } else {
                acc[q] = max(acc[q], lbf);
                acc[32 + q] = max(acc[32 + q], lbb);
              }
            }
          }
        }
      }
      if (LOG) {
        int (&argr)[64] = *reinterpret_cast<int (*)[64]>(&arg[0]);
        transpose_argmax64(acc, argr, lane);
      } else {
        transpose_max64(acc, lane);
      }
      // lane q < 32 now holds forward child cb+q, lane 32+q backward child cb+q
      const bool mine = ql < nq;
      const bool bwd = lane >= 32;
      const int val = mine ? max(lb1, acc[0]) : kInt32Max;
      if (mine) {
        const int o = (bwd ? ns : 0) + cb + ql;
        lbrow[o] = val;
        prow[o] = val >= ub;
        if (LOG) arow[o] = (int16_t)(acc[0] > lb1 ? arg[0] : -1);  // -1: LB1 suffices
      }
      // MinMin over this chunk
      const int cmn = wave_min(val);
      const int ccf = wave_popc(mine && !bwd && val == cmn);
      const int ccb = wave_popc(mine && bwd && val == cmn);
      const long long csf = wave_sum64(mine && !bwd ? (long long)val : 0);
      const long long csb = wave_sum64(mine && bwd ? (long long)val : 0);
      mm.merge(cmn, ccf, ccb, csf, csb);
      wave_sync();
    }
    fill_invalid(lbrow, prow, arow, ns, r, lane, 64);
    if (pool.dir && lane == 0) pool.dir[par] = (uint8_t)mm.dir();
  }
}

// ------------------------------------------------------------- LB2, fast path
// Same computation as k_lb2 for instances with n <= NMAX <= 64 and packed
// (narrow) pair entries.  The pair table is staged in LDS padded to NMAX rows
// and to whole waves of pairs, so the two scans are fully unrolled and free
// of branches: membership of each job in the parent's unscheduled set comes
// from a wave-uniform bit mask, non-members contribute zeros, and the prefix
// maxima of the forward scan stay in registers.  X(j) is kept per lane in an
// LDS column indexed by job id.
template <int NMAX>
struct MaskT {
  using T = typename std::conditional<(NMAX <= 32), uint32_t, uint64_t>::type;
  __device__ __forceinline__ static int neg(T mask, int k) {  // -1 if k is a member, else 0
    if constexpr (NMAX <= 32)
      return __builtin_amdgcn_sbfe((int)mask, k, 1);
    else
      return -(int)((mask >> k) & 1u);
  }
};

// LDS layout of the fast LB2 kernels for a class of instances with at most
// NMAX jobs, mmax machines and ppad padded pairs.
struct FastLayout {
  int ppad, nmax_jobs, mmax;
  __host__ __device__ size_t block_bytes(int nmax) const {
    return align16((size_t)nmax * ppad * 8) + align16((size_t)ppad * 4) +
           align16((size_t)nmax_jobs * mmax * 4);
  }
  __host__ __device__ size_t wave_bytes(int nmax) const {
    const int xr = nmax < 32 ? nmax : 32;
    return align16((size_t)nmax * 64 * 8) + align16((size_t)xr * mmax * 8) +
           align16((size_t)3 * mmax * 4) + align16((size_t)nmax * 4);
  }
};

template <int NMAX>
struct FastLds {
  uint2 *ent;  // [NMAX][Ppad] padded pair entries
  int *uv;     // [Ppad] u | v << 8
  int *sp;     // p[n][m]
  int2 *X;     // per wave [NMAX][64]: per job, per lane
  int2 *FB;    // per wave [32][m]: (forward child front - p, backward child back - p)
  int *c1, *c2, *rr, *jobs;
  __device__ FastLds(unsigned char *sm, const FastLayout &L, int w) {
    ent = (uint2 *)sm;
    size_t off = align16((size_t)NMAX * L.ppad * 8);
    uv = (int *)(sm + off);
    off += align16((size_t)L.ppad * 4);
    sp = (int *)(sm + off);
    off += align16((size_t)L.nmax_jobs * L.mmax * 4);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(NMAX);
    const int xr = NMAX < 32 ? NMAX : 32;
    X = (int2 *)wb;
    wb += align16((size_t)NMAX * 64 * 8);
    FB = (int2 *)wb;
    wb += align16((size_t)xr * L.mmax * 8);
    c1 = (int *)wb;
    c2 = c1 + L.mmax;
    rr = c2 + L.mmax;
    wb += align16((size_t)3 * L.mmax * 4);
    jobs = (int *)wb;
  }
};

// Block-cooperative staging of one instance: rows >= n and pairs >= P of the
// padded table hold a job id that is never a member (NMAX - 1 >= n whenever
// such rows exist) and zero times.  No barrier inside.
template <int NMAX>
__device__ void lb2f_stage(const DevInst &I, int Ppad, const FastLds<NMAX> &S) {
  const int n = I.n, m = I.m, P = I.P;
  // NMAX <= 32: entries are restaged as (a | b << 16, job | lag << 16) (the
  // launcher only takes this path when every lag is below 2^16), so that the
  // job id is the low field used by the membership bit test and the lag a
  // 16-bit field; NMAX = 64 keeps (a | b << 16, lag | job << 24).
  constexpr bool L16 = NMAX <= 32;
  const unsigned kpad = L16 ? (unsigned)(NMAX - 1) : (unsigned)(NMAX - 1) << 24;
  for (int x = threadIdx.x; x < NMAX * Ppad; x += blockDim.x) {
    const int i = x / Ppad, pi = x - i * Ppad;
    uint2 e = make_uint2(0u, kpad);
    if (i < n && pi < P) {
      e = I.ent[(size_t)i * P + pi];
      if (L16) e.y = (e.y >> 24) | ((e.y & 0xffffu) << 16);
    }
    S.ent[x] = e;
  }
  for (int x = threadIdx.x; x < Ppad; x += blockDim.x)
    S.uv[x] = x < P ? ((int)I.pu[x] | ((int)I.pv[x] << 8)) : 0;
  for (int x = threadIdx.x; x < n * m; x += blockDim.x) S.sp[x] = I.p[x];
}

// One wave decomposes one parent (see k_lb2 for the method).  row: the
// parent's perm; cs: its (C1, C2, R); outputs lbrow/prow/arow hold 2 * stride
// slots (stride >= n; slots q >= n - d1 - d2 get INT32_MAX / prune 1).
template <int NMAX, bool SUBSET, bool LOG>
__device__ void lb2f_parent(const DevInst &I, int Ppad, const FastLds<NMAX> &S,
                            const uint8_t *__restrict__ row, int a, int b,
                            const int *__restrict__ cs, const uint32_t *__restrict__ mw,
                            int stride, int ub, int *__restrict__ lbrow,
                            uint8_t *__restrict__ prow, int16_t *__restrict__ arow,
                            uint8_t *__restrict__ dirp, int lane) {
  using M = MaskT<NMAX>;
  using MT = typename M::T;
  // pair entries stay in registers between the two scans when they fit
  constexpr bool KEEP = NMAX <= 20 && !LOG && !SUBSET;
  constexpr bool PMB_REG = NMAX <= 20 && !LOG;
  constexpr bool L16 = NMAX <= 32;  // staged entry layout, see lb2f_stage
  const int n = I.n, m = I.m, P = I.P;
  const int r = n - a - b;
  if (r < 1 || cs[0] < 0) {  // flagged by k_lb1: not a valid node
    fill_invalid(lbrow, prow, arow, stride, 0, lane, 64);
    if (dirp && lane == 0) *dirp = 0;
    return;
  }
  const uint2 *ent = S.ent;
  int2 *X = S.X, *FB = S.FB;
  int *c1 = S.c1, *c2 = S.c2, *rr = S.rr, *jobs = S.jobs;
  const int *sp = S.sp;
  const int *uv = S.uv;
  MT bits = 0;
  for (int x = lane; x < n; x += 64) {
    const int j = row[x];
    jobs[x] = j;
    if (x >= a && x < a + r) bits |= (MT)1 << j;
  }
  for (int x = lane; x < m; x += 64) {
    c1[x] = cs[x];
    c2[x] = cs[m + x];
    rr[x] = cs[2 * m + x];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) bits |= __shfl_xor(bits, o, kWave);
  MT umask;
  if constexpr (NMAX <= 32) {
    umask = (MT)__builtin_amdgcn_readfirstlane((int)bits);
  } else {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)bits);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(bits >> 32));
    umask = ((MT)hi << 32) | lo;
  }
  wave_sync();
  // number of selected pairs of this parent (subset bounds)
  int nsel = 0;
  if constexpr (SUBSET) {
    const int words = (P + 31) >> 5;
    for (int w = lane; w < words; w += 64)
      nsel += __popc(mw[w] & (w == words - 1 && (P & 31) ? (1u << (P & 31)) - 1u : 0xffffffffu));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nsel += __shfl_xor(nsel, o, kWave);
    nsel = __builtin_amdgcn_readfirstlane(nsel);
  }
  MinMin mm;
  mm.init();
  for (int cb = 0; cb < r; cb += 32) {
    const int nq = min(32, r - cb);
    int lb1 = kNeg;
    const int ql = lane & 31;
    const int myjob = ql < nq ? jobs[a + cb + ql] : 0;
    if (ql < nq) {
      const int *pj = sp + myjob * m;
      int c = 0, l = 0;
      if (lane < 32) {
        for (int k = 0; k < m; ++k) {
          c = max(c, c1[k]) + pj[k];
          FB[ql * m + k].x = c - pj[k];
          l = max(l, c + rr[k] - pj[k] + c2[k]);
        }
      } else {
        for (int k = m - 1; k >= 0; --k) {
          c = max(c, c2[k]) + pj[k];
          FB[ql * m + k].y = c - pj[k];
          l = max(l, c1[k] + rr[k] - pj[k] + c);
        }
      }
      lb1 = l;
    }
    wave_sync();
    int acc[64];
    int arg[LOG ? 64 : 1];
#pragma unroll
    for (int q = 0; q < 64; ++q) acc[q] = kNeg;
    if constexpr (LOG) {
#pragma unroll
      for (int q = 0; q < 64; ++q) arg[q] = 0x7fffffff;
    }
    // subset bounds: lane l of pass pc takes the (pc + l)-th selected pair, so
    // k selected pairs need ceil(k / 64) passes instead of ceil(P / 64)
    const int npass = SUBSET ? nsel : Ppad;
    for (int pc = 0; pc < npass; pc += 64) {
      int pi = pc + lane;
      bool act = pi < P;
      if constexpr (SUBSET) {
        act = pi < nsel;
        int sidx = pi;
        pi = Ppad - 1;  // a padded pair for idle lanes
        if (act) {
          const int words = (P + 31) >> 5;
          for (int w = 0; w < words; ++w) {
            uint32_t wbits = mw[w];
            if (w == words - 1 && (P & 31)) wbits &= (1u << (P & 31)) - 1u;  // pairs >= P
            const int cnt = __popc(wbits);
            if (sidx < cnt) {
              for (int t = 0; t < sidx; ++t) wbits &= wbits - 1u;
              pi = w * 32 + __ffs(wbits) - 1;
              break;
            }
            sidx -= cnt;
          }
        }
      }
      const int uvp = uv[pi];
      const int u = uvp & 0xff, v = uvp >> 8;
      const int RU = rr[u], RV = rr[v], C1u = c1[u], C1v = c1[v], C2u = c2[u], C2v = c2[v];
      uint2 e[KEEP ? NMAX : 1];
      if constexpr (KEEP) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i) e[i] = ent[i * Ppad + pi];
      }
      if constexpr (L16) {
        // forward scan: running A - B over members and, per entry, the exclusive
        // prefix maximum minus b and the member's term (-inf for non-members),
        // all relative to B(U); the backward scan then only combines the stored
        // terms into suffix maxima.
        int pmb[PMB_REG ? NMAX : 1], tmv[PMB_REG ? NMAX : 1];
        int Y = 0, Pm = kNeg;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          const uint2 ei = KEEP ? e[KEEP ? i : 0] : ent[i * Ppad + pi];
          const int ng = M::neg(umask, (int)(ei.y & 31u));
          const int ea = (int)(ei.x & 0xffffu), eb = (int)(ei.x >> 16);
          const int t0 = Y + (ea & ng);
          const int tt = t0 + (int)(ei.y >> 16);
          const int tm = (tt & ng) | (kNeg & ~ng);
          if constexpr (PMB_REG) {
            pmb[PMB_REG ? i : 0] = Pm - eb;
            tmv[PMB_REG ? i : 0] = tm;
          } else {
            X[(int)(ei.y & 0xffu) * 64 + lane] = make_int2(Pm - eb, tm);
          }
          Pm = max(Pm, tm);
          Y = t0 - (eb & ng);
        }
        // backward scan: X(j) = max(PM - b, SM - a), stored as (X + a, X + b)
        int Sm = kNeg;
#pragma unroll
        for (int i = NMAX - 1; i >= 0; --i) {
          const uint2 ei = KEEP ? e[KEEP ? i : 0] : ent[i * Ppad + pi];
          const int ea = (int)(ei.x & 0xffffu), eb = (int)(ei.x >> 16);
          const int ek = (int)(ei.y & 0xffu);
          int pm, tm;
          if constexpr (PMB_REG) {
            pm = pmb[PMB_REG ? i : 0];
            tm = tmv[PMB_REG ? i : 0];
          } else {
            // padding rows share one job id, so their stored values may have
            // been overwritten: only members may feed the suffix maximum
            const int2 st = X[ek * 64 + lane];
            pm = st.x;
            tm = M::neg(umask, (int)(ei.y & 31u)) ? st.y : kNeg;
          }
          const int x = max(pm, Sm - ea);
          X[ek * 64 + lane] = make_int2(x + ea, x + eb);
          Sm = max(Sm, tm);
        }
      } else {
        // forward scan: exclusive prefix maxima of term - B(U), minus b (kept in
        // registers when they fit, else in the lane's X column)
        int pmb[PMB_REG ? NMAX : 1];
        int Y = 0, Pm = kNeg;
  #pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          const uint2 ei = KEEP ? e[KEEP ? i : 0] : ent[i * Ppad + pi];
          const int ea = (int)(ei.x & 0xffffu), eb = (int)(ei.x >> 16);
          const int el = (int)(ei.y & 0xffffffu), ek = (int)(ei.y >> 24);
          const int ng = M::neg(umask, ek);
          Y += ea & ng;
          const int tt = Y + el;
          if constexpr (PMB_REG)
            pmb[PMB_REG ? i : 0] = Pm - eb;
          else
            X[ek * 64 + lane].x = Pm - eb;
          Pm = max(Pm, ng ? tt : kNeg);
          Y -= eb & ng;
        }
        // backward scan: exclusive suffix maxima; X(j) = max(PM - b, SM - a)
        const int c0 = RU - RV;
        int Wb = 0, Sm = kNeg;
  #pragma unroll
        for (int i = NMAX - 1; i >= 0; --i) {
          const uint2 ei = KEEP ? e[KEEP ? i : 0] : ent[i * Ppad + pi];
          const int ea = (int)(ei.x & 0xffffu), eb = (int)(ei.x >> 16);
          const int el = (int)(ei.y & 0xffffffu), ek = (int)(ei.y >> 24);
          const int ng = M::neg(umask, ek);
          Wb += eb & ng;
          const int tp = Wb + el + c0;
          const int pm = PMB_REG ? pmb[PMB_REG ? i : 0] : X[ek * 64 + lane].x;
          const int x = max(pm, Sm - ea);
          X[ek * 64 + lane] = make_int2(x + ea, x + eb);
          Sm = max(Sm, ng ? tp : kNeg);
          Wb -= ea & ng;
        }
      }
      const int K1 = RU + C2u, K2 = C1u + RU, K3 = C1v + RV;
#pragma unroll
      for (int q = 0; q < 32; ++q) {
        if (q < nq) {
          const int kq = __builtin_amdgcn_readlane(myjob, q);
          const int2 xab = X[kq * 64 + lane];
          const int2 fu = FB[q * m + u], fv = FB[q * m + v];
          const int xa = xab.x + RV, xb = xab.y + RV;
          int lbf = max(fu.x + K1, max(fv.x + RV, fu.x + xa) + C2v);
          int lbb = max(fu.y + K2, max(K3, C1u + xb) + fv.y);
          lbf = act ? lbf : kNeg;
          lbb = act ? lbb : kNeg;
          if constexpr (LOG) {
            if (lbf > acc[q]) { acc[q] = lbf; arg[q] = pi; }
            if (lbb > acc[32 + q]) { acc[32 + q] = lbb; arg[32 + q] = pi; }
          } else {
            acc[q] = max(acc[q], lbf);
            acc[32 + q] = max(acc[32 + q], lbb);
          }
        }
      }
    }
    if constexpr (LOG) {
      transpose_argmax64(acc, arg, lane);
    } else {
      transpose_max64_xl(acc, lane);
    }
    const bool mine = ql < nq;
    const bool bwd = lane >= 32;
    const int val = mine ? max(lb1, acc[0]) : kInt32Max;
    if (mine) {
      const int o = (bwd ? stride : 0) + cb + ql;
      lbrow[o] = val;
      prow[o] = val >= ub;
      if constexpr (LOG) arow[o] = (int16_t)(acc[0] > lb1 ? arg[0] : -1);  // -1: LB1 suffices
    }
    const int cmn = wave_min(val);
    const int ccf = wave_popc(mine && !bwd && val == cmn);
    const int ccb = wave_popc(mine && bwd && val == cmn);
    const long long csf = wave_sum64(mine && !bwd ? (long long)val : 0);
    const long long csb = wave_sum64(mine && bwd ? (long long)val : 0);
    mm.merge(cmn, ccf, ccb, csf, csb);
    wave_sync();
  }
  fill_invalid(lbrow, prow, arow, stride, r, lane, 64);
  if (dirp && lane == 0) *dirp = (uint8_t)mm.dir();
}

// ---------------------------------------------------------------- quick LB2
// LB2 for instances with n <= NMAX <= 32 and every a_j + l_j below 2^16.
//
// For a pair (u, v) and a child whose unscheduled set is U' (the parent's U
// without the child's job j), the two-machine value is the maximum of three
// terms: h_u + A(U') + t_u, h_v + B(U') + t_v, and h_u + T(U') + t_v, where
// h and t are the child's heads and tails and T(U') is the longest
// first-to-second machine path of the Johnson schedule of U' (Section 2.4).
// The first two are one-machine bounds of machines u and v, never above LB1,
// so LB2 = max(LB1, max over pairs of h_u + T(U') + t_v) and only the third
// term is evaluated per child and pair.  With terms relative to B(U),
// term_i = Y(<i) + a_i + l_i, Y(<i) = sum over members before i of a - b,
// and the exclusive prefix/suffix maxima PM(i), SM(i) over the members of U
// in Johnson order, removing member j gives
//   T(U') - B(U) + a_j = max(PM(j) + a_j - b_j, SM(j))  =: Xa(j)
//   T(U') - B(U) + b_j = Xa(j) + b_j - a_j               =: Xb(j)
// so that, with f_u the start of j on machine u in the forward child and g_v
// its start on machine v in the backward child,
//   forward child:  f_u + Xa(j) + R_v + C2_v
//   backward child: g_v + Xb(j) + C1_u + R_v.
// One wave decomposes one parent; lane L takes pair 64 * pass + L, and the
// per-child maxima over pairs are folded across lanes at the end.
//
// Block-shared LDS: ent [npass][NMAX][64] entries {b - a, k | (a + l) << 16}
// in Johnson order (pairs >= P repeat pair 0, rows >= n hold job NMAX - 1
// with zero times), uv [Ppad] (u | v << 8), and p transposed [m][32] plus a
// copy with the machines reversed.  Per wave: X [NMAX][64] (Xa, Xb) by job
// (two 16-bit halves when X16, see below),
// child starts FBf [m][ROW] (forward, by machine) and FBb [m][ROW] (backward,
// machines reversed), HTf/HTb [m] (head, tail + remaining work per machine
// in scan order), C1, C2, R [m], and the inverse permutation inv [32].
struct QuickLayout {
  int ppad, mmax, x16, subset;  // X16 needs one start-time table, subset bounds the sel list
  __host__ __device__ static constexpr int row(int nmax) { return nmax | 1; }
  __host__ __device__ size_t block_bytes(int nmax) const {
    return align16((size_t)nmax * ppad * 8) + align16((size_t)ppad * 4) +
           align16((size_t)2 * mmax * 32 * 4);
  }
  __host__ __device__ size_t wave_bytes(int nmax) const {
    return align16((size_t)nmax * 64 * (x16 ? 4 : 8)) +
           align16((size_t)(x16 ? 1 : 2) * mmax * row(nmax) * 4) + align16((size_t)2 * mmax * 8) +
           align16((size_t)3 * mmax * 4) + align16(32 * 4) + (subset ? align16((size_t)ppad * 2) : 0);
  }
};

template <int NMAX>
struct QuickLds {
  uint2 *ent;
  int *uv, *pt, *pr;
  void *X;
  int *FBf, *FBb;
  int2 *HTf, *HTb;
  int *c1, *c2, *rr, *inv;
  short *sel;  // subset bounds: the selected pair indices in order
  __device__ QuickLds(unsigned char *sm, const QuickLayout &L, int w) {
    constexpr int ROW = QuickLayout::row(NMAX);
    ent = (uint2 *)sm;
    size_t off = align16((size_t)NMAX * L.ppad * 8);
    uv = (int *)(sm + off);
    off += align16((size_t)L.ppad * 4);
    pt = (int *)(sm + off);
    pr = pt + L.mmax * 32;
    off += align16((size_t)2 * L.mmax * 32 * 4);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(NMAX);
    X = wb;
    wb += align16((size_t)NMAX * 64 * (L.x16 ? 4 : 8));
    FBf = (int *)wb;
    FBb = FBf + (L.x16 ? 0 : L.mmax * ROW);  // X16: one table of int16 pairs
    wb += align16((size_t)(L.x16 ? 1 : 2) * L.mmax * ROW * 4);
    HTf = (int2 *)wb;
    HTb = HTf + L.mmax;
    wb += align16((size_t)2 * L.mmax * 8);
    c1 = (int *)wb;
    c2 = c1 + L.mmax;
    rr = c2 + L.mmax;
    wb += align16((size_t)3 * L.mmax * 4);
    inv = (int *)wb;
    wb += align16(32 * 4);
    sel = (short *)wb;
  }
};

// Block-cooperative staging of one instance for the quick kernels (no
// barrier inside).  The staged narrow entries hold x = a | b << 16 and
// y = l | k << 24; the quick entries are {E, k | (a + l) << 16} with
// E = b - a: the scans take a + l from the high half of y, and k < 32 sits
// in the low bits that a bit-field extract takes as its offset.  KE (the
// kernels with 16-bit X): x = E in its low 16 bits | k << 24, which is the
// scan's stored word (E, row of X) as it stands, and the running sums add E
// with a 16-bit multiply-add; else x = E as a full word.
template <int NMAX, bool KE, class Lds>
__device__ void lb2q_stage(const DevInst &I, int Ppad, const Lds &S) {
  const int n = I.n, m = I.m, P = I.P;
  for (int x = threadIdx.x; x < NMAX * Ppad; x += blockDim.x) {
    const int pass = x / (NMAX * 64), rem = x - pass * NMAX * 64;
    const int i = rem >> 6, pi = pass * 64 + (rem & 63);
    uint2 e = make_uint2(KE ? (unsigned)(NMAX - 1) << 24 : 0u, (unsigned)(NMAX - 1));
    if (i < n && P > 0) {
      const uint2 s = I.ent[(size_t)i * P + (pi < P ? pi : 0)];
      const unsigned a = s.x & 0xffffu, b = s.x >> 16, l = s.y & 0xffffffu, k = s.y >> 24;
      e = make_uint2(KE ? ((b - a) & 0xffffu) | (k << 24) : b - a, k | ((a + l) << 16));
    }
    S.ent[x] = e;
  }
  for (int x = threadIdx.x; x < Ppad; x += blockDim.x) {
    const int q = x < P ? x : 0;
    S.uv[x] = P > 0 ? ((int)I.pu[q] | ((int)I.pv[q] << 8)) : 0;
  }
  for (int x = threadIdx.x; x < m * 32; x += blockDim.x) {
    const int s = x >> 5, k = x & 31;
    S.pt[x] = k < n ? I.p[k * m + s] : 0;
    S.pr[x] = k < n ? I.p[k * m + (m - 1 - s)] : 0;
  }
}

// Global inputs of one parent as the lanes hold them: row byte `lane` (lane
// < n), costs C1, C2, R of machine `lane` (lane < m), mask word `lane`
// (lane < words), and d1, d2 (c1 = -1 on every lane: no parent).  The
// kernels load them one parent (or batch) ahead so that their latency
// overlaps the previous one's work.
struct PackFetch {
  int rb, c1, c2, rr, d1, d2;
  uint32_t mw;
};

__device__ __forceinline__ PackFetch row_fetch(const uint8_t *__restrict__ row,
                                               const int *__restrict__ cs, int d1, int d2, int n,
                                               int m, int lane) {
  PackFetch F{0, -1, 0, 0, d1, d2, 0u};
  if (lane < n) F.rb = row[lane];
  if (lane < m) {
    F.c1 = cs[lane];
    F.c2 = cs[m + lane];
    F.rr = cs[2 * m + lane];
  }
  return F;
}

__device__ __forceinline__ PackFetch pack_fetch(const DevPool &pool, int par, int n, int m,
                                                const int *__restrict__ costs, int lane) {
  PackFetch F{0, -1, 0, 0, 0, 0, 0u};
  if (par >= 0) {
    const int *cs = costs + (size_t)par * 3 * m;
    F.d1 = pool.d1[par];
    F.d2 = pool.d2[par];
    if (lane < n) F.rb = pool.perm[(size_t)par * pool.n + lane];
    if (lane < m) {
      F.c1 = cs[lane];
      F.c2 = cs[m + lane];
      F.rr = cs[2 * m + lane];
    }
    if (lane < pool.mask_words) F.mw = mask_row(pool, par)[lane];
  }
  return F;
}

// Static LDS of the depth-bin row lists (one chunk of a block's rows plus a
// count per wave).
constexpr int kBinListCap = 1024;
constexpr size_t kBinListLds = (kBinListCap + 16) * 4;

// Runs body(par, F) for the parents a wave bounds, with the next parent's
// inputs loaded while the current one is bounded.  Without a depth bin the
// waves take launch rows blockIdx.x * nw + w + k * gridDim.x * nw.  With one,
// the block takes chunks of CH consecutive launch rows (chunk c = blockIdx.x +
// k * gridDim.x; CH = the rows per block of an even split, between nw and
// blockDim.x, so that small launches still reach every block), lists the
// rows of its bin in LDS (wave ballots, one count per wave) and its waves
// take list entries w, w + nw, ...  Every wave of the block runs the chunk
// loop (it holds barriers).
template <class Body>
__device__ __forceinline__ void parent_loop(const DevPool &pool, int count, int n, int m,
                                            const int *__restrict__ costs, int lane, int w,
                                            int nw, int *blist, Body body) {
  if (!pool.bin) {
    const int step = gridDim.x * nw;
    auto row_of = [&](int x) { return x < count ? (pool.index ? pool.index[x] : x) : -1; };
    int it = blockIdx.x * nw + w;
    int par = row_of(it);
    PackFetch F = pack_fetch(pool, par, n, m, costs, lane);
    for (; it < count; it += step) {
      const int nxt = row_of(it + step);  // the next parent's inputs are loaded meanwhile
      const PackFetch Fn = pack_fetch(pool, nxt, n, m, costs, lane);
      body(par, F);
      par = nxt;
      F = Fn;
    }
    return;
  }
  const int T = blockDim.x;
  const int CH = min(T, max(nw, (count + (int)gridDim.x - 1) / (int)gridDim.x));
  int *wcnt = blist + kBinListCap;
  for (int c0 = blockIdx.x * CH; c0 < count; c0 += gridDim.x * CH) {
    const int x = c0 + (int)threadIdx.x;
    bool in = false;
    int row = -1;
    if ((int)threadIdx.x < CH && x < count) {
      row = pool.index ? pool.index[x] : x;
      const int r = n - pool.d1[row] - pool.d2[row];
      const bool deep = r >= 1 && r <= pool.bin_r;
      in = pool.bin == 2 ? deep : !deep;
    }
    const uint64_t bal = __ballot(in);
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = 0, total = 0;
    for (int v = 0; v < nw; ++v) {
      const int cv = wcnt[v];
      off += v < w ? cv : 0;
      total += cv;
    }
    if (in)
      blist[off + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0))] =
          row;
    __syncthreads();
    int j = w;
    int par = j < total ? blist[j] : -1;
    PackFetch F = pack_fetch(pool, par, n, m, costs, lane);
    for (; j < total; j += nw) {
      const int nxt = j + nw < total ? blist[j + nw] : -1;
      const PackFetch Fn = pack_fetch(pool, nxt, n, m, costs, lane);
      body(par, F);
      par = nxt;
      F = Fn;
    }
    __syncthreads();  // the next chunk rewrites the list
  }
}

// X16: the scan starts from Y = R_v + C2_v instead of 0.  For a member j
// with at least one other member (U' not empty) the stored Xa(j) + R_v +
// C2_v equals T(U') + a_j + C2_v and the high half Xb(j) + C1_u + R_v equals
// T(U') + b_j + C1_u: sums of processing times over disjoint cells, in
// [0, (n + m) max p], so with (n + m) max p < 2^15 both fit int16.  A parent
// with one job left needs no pair (its children are leaves and LB1 is their
// makespan), so the only NEG-derived value, that of a sole member, never
// reaches a bound.
template <int NMAX, bool SUBSET, bool X16>
__device__ void lb2q_parent(const DevInst &I, int Ppad, const QuickLds<NMAX> &S,
                            const PackFetch &F, int stride, int ub, int *__restrict__ lbrow,
                            uint8_t *__restrict__ prow, uint8_t *__restrict__ dirp, int lane,
                            int tsrc) {
  constexpr int ROW = QuickLayout::row(NMAX);
  const int n = I.n, m = I.m, P = I.P;
  const int a = __builtin_amdgcn_readfirstlane(F.d1), b = __builtin_amdgcn_readfirstlane(F.d2);
  const int r = n - a - b;
  if (r < 1 || __builtin_amdgcn_readfirstlane(F.c1) < 0) {  // flagged by the costs kernel
    fill_invalid(lbrow, prow, nullptr, stride, 0, lane, 64);
    if (dirp && lane == 0) *dirp = 0;
    return;
  }
  // inverse permutation, parent costs, per-direction head/tail tables
  if (lane < n) S.inv[F.rb] = lane;
  if (lane < m) {
    S.c1[lane] = F.c1;
    S.c2[lane] = F.c2;
    S.rr[lane] = F.rr;
    S.HTf[lane] = make_int2(F.c1, F.rr + F.c2);
    S.HTb[m - 1 - lane] = make_int2(F.c2, F.c1 + F.rr);
  }
  wave_sync();
  const int k = lane & 31;  // job of this lane; lanes >= 32 take its backward child
  const bool bwd = lane >= 32;
  const int slot = k < n ? S.inv[k] - a : -1;
  const bool member = slot >= 0 && slot < r;
  const uint32_t umask =
      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)__ballot(member && !bwd));
  // LB1 of both children of job k, and the start times f (forward child,
  // machines in order) or g (backward child, machines reversed).  X16: one
  // table of int16 pairs in scan order, f of machine s in the low half of
  // [s][k] and g of machine m - 1 - s in the high half (both below 2^15), so
  // that both directions write with one constant stride
  int lb1 = 0;
  if (k < NMAX) {
    const int2 *HT = bwd ? S.HTb : S.HTf;
    const int *PT = (bwd ? S.pr : S.pt) + k;
    int *FB = (bwd ? S.FBb : S.FBf) + k;
    unsigned short *fb16 = (unsigned short *)S.FBf + 2 * k + (bwd ? 1 : 0);
    int c = 0;
#pragma unroll 4
    for (int s = 0; s < m; ++s) {
      const int2 ht = HT[s];
      const int f = max(c, ht.x);
      c = f + PT[s * 32];
      if constexpr (X16)
        fb16[s * 2 * ROW] = (unsigned short)f;
      else
        FB[s * ROW] = f;
      lb1 = max(lb1, f + ht.y);
    }
  }
  wave_sync();
  int nsel = 0;
  if constexpr (SUBSET) {  // selected pairs in index order, compacted by ballot
    for (int base = 0; base < P; base += 64) {
      const int q = base + lane;
      const uint32_t wq = (uint32_t)__shfl((int)F.mw, (q >> 5) & 63, kWave);
      const bool on = q < P && ((wq >> (q & 31)) & 1u);
      const uint64_t bal = __ballot(on);
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (on) S.sel[nsel + pos] = (short)q;
      nsel += __popcll(bal);
    }
    wave_sync();
  }
  // pair maxima per job: X16 keeps both directions in one register as int16
  // halves (every pair term of a child is at most (n + m - 1) max p < 2^15)
  constexpr int NA = X16 ? 1 : NMAX;
  int accf[NA], accb[NA], acc[X16 ? NMAX : 1];
#pragma unroll
  for (int q = 0; q < NA; ++q) accf[q] = accb[q] = kNeg;
  // (set once here: left to itself the compiler repeats these moves on the
  // path into the pair loop)
#pragma unroll
  for (int q = 0; q < (X16 ? NMAX : 1); ++q) {
    acc[q] = (int)0x80008000u;
    asm volatile("" : "+v"(acc[q]));
  }
  const int npass = r < 2 ? 0 : SUBSET ? nsel : (P > 0 ? Ppad : 0);  // leaves: LB2 = LB1
  constexpr int NEGX = X16 ? -(1 << 14) : kNeg;
  int2 *__restrict__ Xl = (int2 *)S.X + lane;
  int *__restrict__ Xh = (int *)S.X + lane;
  for (int pc = 0; pc < npass; pc += 64) {
    int pi = pc + lane;
    // subset bounds: lanes past the selection repeat the first selected pair
    if constexpr (SUBSET) pi = S.sel[pi < nsel ? pi : 0];
    const int uvp = S.uv[pi];
    const int u = uvp & 0xff, v = uvp >> 8;
    const int K4 = S.rr[v] + S.c2[v], K5 = S.c1[u] + S.rr[v];
    const int *Fu = lds_opaque(S.FBf + u * ROW);
    const int *Gv = lds_opaque((X16 ? S.FBf : S.FBb) + (m - 1 - v) * ROW);
    const uint2 *__restrict__ eb = S.ent + (pi >> 6) * (NMAX * 64) + (pi & 63);
    // forward scan: terms of members (NEG for the others) and exclusive prefix
    // maxima.  X16 keeps per position one int16 pair, the prefix maximum less
    // b - a (low) and the term (high), and E | job << 24
    constexpr int NS = X16 ? 1 : NMAX, NP = X16 ? NMAX : 1;
    int pm[NS], tm[NS], pt[NP];
    unsigned ke[NP];
    int Y = X16 ? K4 : 0, Pm = NEGX;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      const uint2 e = eb[i * 64];
      const int ng = __builtin_amdgcn_sbfe((int)umask, (int)e.y, 1);  // -1 if member
      const int tt = Y + (int)(e.y >> 16);
      const int term = (tt & ng) | (NEGX & ~ng);
      if constexpr (X16) {
        pt[i] = (int)__builtin_amdgcn_perm((unsigned)term, (unsigned)(Pm - (int)e.x), 0x05040100u);
        ke[i] = e.x;
        Y = mad_i16(ng, (int)e.x, Y);  // Y += a - b for members
      } else {
        tm[i] = term;
        pm[i] = Pm;
        Y = __mul24(ng, (int)e.x) + Y;
      }
      Pm = max(Pm, term);
    }
    // backward scan: Xa, Xb by job (the 32-bit entries are read again rather
    // than held in registers; X16 keeps a packed copy from the forward scan)
    const int K5x = K5 - K4;  // X16: the high half is Xb + K5 (K4 is already inside)
    if constexpr (X16) {
      // one packed maximum per position: against the suffix maximum Sm of the
      // terms after it (held in both halves) the low half becomes Xa and the
      // high half the suffix maximum that includes this term.  Xa - b + a
      // fits int16 wherever the value is used (a member with another member
      // left), and Xb + K5 = Xa + E + K5x in the high half of the stored word
      // needs only the low 16 bits of each addend
      int R = (int)0xC000C000u;  // NEGX in both halves
#pragma unroll
      for (int i = NMAX - 1; i >= 0; --i) {
        R = pk_max_hi(pt[i], R);
        *(int *)((char *)Xh + (ke[i] >> 16)) = (int)__builtin_amdgcn_perm(
            (unsigned)(R + (int)ke[i] + K5x), (unsigned)R, 0x05040100u);
      }
    } else {
      int Sm = NEGX;
#pragma unroll
      for (int i = NMAX - 1; i >= 0; --i) {
        const uint2 e = eb[i * 64];
        const int E = (int)e.x;
        const int xa = max(pm[i] - E, Sm);
        Xl[(e.y & 31u) * 64] = make_int2(xa, xa + E);
        Sm = max(Sm, tm[i]);
      }
    }
    // children, four jobs at a time so that their loads are issued together
    // (each lane reads back only its own column of X; jobs that are not
    // members accumulate values that are never used)
#pragma unroll
    for (int g = 0; g < NMAX; g += 4) {
      if (umask & (0xfu << g)) {
        if constexpr (X16) {  // f_u + xa | g_v + xb in int16 halves
          int h[4], fw[4], gw[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (g + j < NMAX) {
              h[j] = Xh[(g + j) * 64];
              fw[j] = Fu[g + j];
              gw[j] = Gv[g + j];
            }
          }
          // all four sums before the maxima: a packed result read by the
          // next instruction costs a wait state
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (g + j < NMAX)
              h[j] = pk_add((int)__builtin_amdgcn_perm((unsigned)gw[j], (unsigned)fw[j],
                                                       0x07060100u),
                            h[j]);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (g + j < NMAX) acc[g + j] = pk_max(acc[g + j], h[j]);
          }
        } else {
          int xa[4], xb[4], fu[4], gv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (g + j < NMAX) {
              const int2 x = Xl[(g + j) * 64];
              xa[j] = x.x + K4;
              xb[j] = x.y + K5;
              fu[j] = Fu[g + j];
              gv[j] = Gv[g + j];
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (g + j < NMAX) {
              accf[g + j] = max(accf[g + j], fu[j] + xa[j]);
              accb[g + j] = max(accb[g + j], gv[j] + xb[j]);
            }
          }
        }
      }
    }
  }
  int t;
  if constexpr (X16) {
    t = transpose_pkmax<NMAX>(acc, lane, tsrc);
  } else {
    t = transpose_max_fb<NMAX>(accf, accb, lane, kNeg);
  }
  const int val = member ? max(lb1, t) : kInt32Max;
  if (member) {
    const int o = (bwd ? stride : 0) + slot;
    lbrow[o] = val;
    prow[o] = val >= ub;
  }
  fill_invalid(lbrow, prow, nullptr, stride, r, lane, 64);
  if (dirp) {
    // MinMin over both children sets
    const int cmn = wave_min_xl(val);
    const uint64_t at = __ballot(member && val == cmn);
    const int cf = __popc((uint32_t)at), cb = __popc((uint32_t)(at >> 32));
    const int sv = member ? val : 0;
    long long sf, sb;
    if constexpr (X16) {  // bounds below 2^15: the 32 of a half sum below 2^20
      const int s = half_sum(sv);
      sf = __builtin_amdgcn_readlane(s, 0);
      sb = __builtin_amdgcn_readlane(s, 32);
    } else {
      const int slo = half_sum(sv & 0xffff), shi = half_sum(sv >> 16);
      sf = ((long long)__builtin_amdgcn_readlane(shi, 0) << 16) + __builtin_amdgcn_readlane(slo, 0);
      sb = ((long long)__builtin_amdgcn_readlane(shi, 32) << 16) +
           __builtin_amdgcn_readlane(slo, 32);
    }
    MinMin mm;
    mm.init();
    mm.merge(cmn, cf, cb, sf, sb);
    if (lane == 0) *dirp = (uint8_t)mm.dir();
  }
  wave_sync();  // the next parent rewrites this wave's tables
}

// Up to 16 waves per block (four per SIMD, which the registers of up to 20
// jobs with 16-bit X allow), else 12 (three per SIMD, up to 24 jobs); 8 for
// 32 jobs, whose registers need two per SIMD.
template <int NMAX, bool SUBSET, bool X16>
__global__ void __launch_bounds__(X16 && NMAX <= 20 ? 1024 : NMAX <= 24 ? 768 : 512)
k_lb2q(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
       uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  // the wave index as a uniform value: parent indices, and the loads of their
  // depths and pool rows, stay scalar
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  __shared__ int blist[kBinListCap + 16];
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw >= count) return;  // no parent for this block: skip the staging
  const QuickLayout L{Ppad, I.m, X16, SUBSET};
  const QuickLds<NMAX> S(sm, L, w);
  lb2q_stage<NMAX, X16>(I, Ppad, S);
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int n = I.n, m = I.m, ns = pool.n;  // ns: row stride (>= n)
  const int tsrc = tp_source<NMAX>(lane);
  parent_loop(pool, count, n, m, costs, lane, w, nw, blist, [&](int par, const PackFetch &F) {
    lb2q_parent<NMAX, SUBSET, X16>(I, Ppad, S, F, ns, ub, out_lb + (size_t)par * 2 * ns,
                                   out_prune + (size_t)par * 2 * ns,
                                   pool.dir ? pool.dir + par : nullptr, lane, tsrc);
  });
}

// ------------------------------------------------------------ deep LB2
// Full LB2 for parents with few unscheduled jobs (r <= RMAX; n <= 32 with
// 16-bit X).  The quick kernel scans all n Johnson positions of every pair,
// members or not, so its cost hardly falls with depth; here each lane visits
// only the r member positions of its pair, in Johnson order, by taking the
// set bits of a per-parent position mask from the lowest.  A block-level
// table gives the position of every job in every pair's order.  The values
// are those of the quick kernel (same terms, same packed scans); the
// children are indexed by list slot q (job perm[d1 + q]) instead of job id,
// so the per-child registers, the LB1 lanes and the fold cover RMAX slots.
struct DeepLayout {
  int ppad, mmax, rmax;
  __host__ __device__ size_t block_bytes(int nmax) const {
    return align16((size_t)nmax * ppad * 8) + align16((size_t)ppad * 4) +
           align16((size_t)2 * mmax * 32 * 4) + align16((size_t)ppad * 32);
  }
  __host__ __device__ size_t wave_bytes(int nmax) const {
    return align16((size_t)rmax * 64 * 4) + align16((size_t)mmax * QuickLayout::row(nmax) * 4) +
           align16((size_t)2 * mmax * 8) + align16((size_t)3 * mmax * 4) + align16(32 * 4);
  }
};

// The quick kernel's tables (X with one row per slot, the single X16
// start-time table) plus the block's position table pos[pass][job][lane].
template <int NMAX>
struct DeepLds {
  uint2 *ent;
  int *uv, *pt, *pr;
  uint8_t *pos;
  int *X;
  int *FBf;
  int2 *HTf, *HTb;
  int *c1, *c2, *rr, *inv;
  __device__ DeepLds(unsigned char *sm, const DeepLayout &L, int w) {
    ent = (uint2 *)sm;
    size_t off = align16((size_t)NMAX * L.ppad * 8);
    uv = (int *)(sm + off);
    off += align16((size_t)L.ppad * 4);
    pt = (int *)(sm + off);
    pr = pt + L.mmax * 32;
    off += align16((size_t)2 * L.mmax * 32 * 4);
    pos = sm + off;
    off += align16((size_t)L.ppad * 32);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(NMAX);
    X = (int *)wb;
    wb += align16((size_t)L.rmax * 64 * 4);
    FBf = (int *)wb;
    wb += align16((size_t)L.mmax * QuickLayout::row(NMAX) * 4);
    HTf = (int2 *)wb;
    HTb = HTf + L.mmax;
    wb += align16((size_t)2 * L.mmax * 8);
    c1 = (int *)wb;
    c2 = c1 + L.mmax;
    rr = c2 + L.mmax;
    wb += align16((size_t)3 * L.mmax * 4);
    inv = (int *)wb;
  }
};

// Block-cooperative: pos[pass][job][lane] = Johnson position of job in the
// order of pair pass * 64 + lane (u8).  No barrier inside.
template <int NMAX>
__device__ void lb2d_stage_pos(const DevInst &I, int Ppad, uint8_t *__restrict__ pos) {
  const int n = I.n, P = I.P;
  for (int x = threadIdx.x; x < n * Ppad; x += blockDim.x) {
    const int pass = x / (n * 64), rem = x - pass * n * 64;
    const int i = rem >> 6, l = rem & 63, pi = pass * 64 + l;
    const unsigned k = I.ent[(size_t)i * P + (pi < P ? pi : 0)].y >> 24;
    pos[(pass * 32 + (int)k) * 64 + l] = (uint8_t)i;
  }
}

template <int NMAX, int RMAX>
__device__ void lb2d_parent(const DevInst &I, int Ppad, const DeepLds<NMAX> &S,
                            const PackFetch &F, int stride,
                            int ub, int *__restrict__ lbrow, uint8_t *__restrict__ prow,
                            uint8_t *__restrict__ dirp, int lane, int tsrc) {
  constexpr int ROW = QuickLayout::row(NMAX);
  const int n = I.n, m = I.m, P = I.P;
  const int a = __builtin_amdgcn_readfirstlane(F.d1), b = __builtin_amdgcn_readfirstlane(F.d2);
  const int r = n - a - b;
  if (r < 1 || r > RMAX || __builtin_amdgcn_readfirstlane(F.c1) < 0) {
    // an invalid row (flagged by the costs kernel); the launcher gives this
    // kernel only rows with 1 <= r <= RMAX
    fill_invalid(lbrow, prow, nullptr, stride, 0, lane, 64);
    if (dirp && lane == 0) *dirp = 0;
    return;
  }
  if (lane < m) {
    S.c1[lane] = F.c1;
    S.c2[lane] = F.c2;
    S.rr[lane] = F.rr;
    S.HTf[lane] = make_int2(F.c1, F.rr + F.c2);
    S.HTb[m - 1 - lane] = make_int2(F.c2, F.c1 + F.rr);
  }
  // slot q: the q-th unscheduled job of the list; lanes >= 32 its backward child
  const int q = lane & 31;
  const bool bwd = lane >= 32;
  const bool member = q < r;
  const int jq = __shfl(F.rb, a + (member ? q : 0), kWave);
  // slot of every job, for the X rows (only members are read)
  if (lane < r) S.inv[jq] = lane;
  wave_sync();
  // LB1 of both children of slot q, and their start times: f of machine s in
  // the low half of [s][job], g of machine m - 1 - s in the high half
  int lb1 = 0;
  if (r == 2) {
    // Two jobs left: each child has one, and its LB2 is the makespan of its
    // only completion.  That makespan is a longest path that enters the last
    // job's operations on some machine k1 and leaves on some k2 >= k1; LB1
    // covers k1 = k2 and the pair (k1, k2) the others, and every term is a
    // lower bound.  So the bound is the makespan itself, from the walk of the
    // child's job and then the other one over the machines (reversed for the
    // backward child), closed by the other side's costs; no pair pass.
    if (member) {
      const int j0 = __builtin_amdgcn_readlane(jq, 0), j1 = __builtin_amdgcn_readlane(jq, 1);
      const int jo = q == 0 ? j1 : j0;  // the job left after this child's
      const int2 *HT = bwd ? S.HTb : S.HTf;
      const int *PT = (bwd ? S.pr : S.pt) + jq;
      const int *PO = (bwd ? S.pr : S.pt) + jo;
      const int *OT = bwd ? S.c1 + (m - 1) : S.c2;  // the far side, in walk order
      const int ostep = bwd ? -1 : 1;
      int c = 0, g = 0;
#pragma unroll 4
      for (int s = 0; s < m; ++s) {
        c = max(c, HT[s].x) + PT[s * 32];
        g = max(g, c) + PO[s * 32];
        lb1 = max(lb1, g + OT[s * ostep]);
      }
    }
  } else if (member) {
    const int2 *HT = bwd ? S.HTb : S.HTf;
    const int *PT = (bwd ? S.pr : S.pt) + jq;
    unsigned short *fb16 = (unsigned short *)S.FBf + 2 * jq + (bwd ? 1 : 0);
    int c = 0;
#pragma unroll 4
    for (int s = 0; s < m; ++s) {
      const int2 ht = HT[s];
      const int f = max(c, ht.x);
      c = f + PT[s * 32];
      fb16[s * 2 * ROW] = (unsigned short)f;
      lb1 = max(lb1, f + ht.y);
    }
  }
  wave_sync();
  int acc[RMAX];
#pragma unroll
  for (int x = 0; x < RMAX; ++x) {
    acc[x] = (int)0x80008000u;
    asm volatile("" : "+v"(acc[x]));
  }
  const int npass = r <= 2 || P == 0 ? 0 : Ppad;  // one job left: LB2 = LB1
  constexpr int NEGX = -(1 << 14);
  int *__restrict__ Xh = S.X + lane;
  for (int pc = 0; pc < npass; pc += 64) {
    const int pi = pc + lane;
    const int uvp = S.uv[pi];
    const int u = uvp & 0xff, v = uvp >> 8;
    const int K4 = S.rr[v] + S.c2[v], K5 = S.c1[u] + S.rr[v];
    const int *Fu = lds_opaque(S.FBf + u * ROW);
    const int *Gv = lds_opaque(S.FBf + (m - 1 - v) * ROW);
    const uint2 *__restrict__ eb = S.ent + (pi >> 6) * (NMAX * 64) + (pi & 63);
    const uint8_t *__restrict__ pb = S.pos + (pi >> 6) * (32 * 64) + (pi & 63);
    // positions of the members in this pair's Johnson order
    uint32_t pm = 0u;
#pragma unroll
    for (int x = 0; x < RMAX; ++x) {
      if (x < r) {
        const int j = __builtin_amdgcn_readlane(jq, x);
        pm |= 1u << pb[j * 64];
      }
    }
    // forward scan over the members: per member one int16 pair (prefix
    // maximum less b - a, term) and b - a with the member's X row offset
    int pt[RMAX];
    unsigned ke[RMAX];
    int Y = K4, Pm = NEGX;
#pragma unroll
    for (int x = 0; x < RMAX; ++x) {
      if (x < r) {
        const int p = __builtin_ctz(pm);
        pm &= pm - 1u;
        const uint2 e = eb[p * 64];
        const int term = Y + (int)(e.y >> 16);
        pt[x] = (int)__builtin_amdgcn_perm((unsigned)term, (unsigned)(Pm - (int)e.x), 0x05040100u);
        const int slot = S.inv[e.y & 31u];
        ke[x] = (e.x & 0xffffu) | ((unsigned)slot << 24);
        Pm = max(Pm, term);
        Y = mad_i16(-1, (int)e.x, Y);  // Y += a - b
      }
    }
    // backward scan: Xa (low) and Xb + K5 (high) per member, into its X row
    const int K5x = K5 - K4;
    int R = (int)0xC000C000u;
#pragma unroll
    for (int x = RMAX - 1; x >= 0; --x) {
      if (x < r) {
        R = pk_max_hi(pt[x], R);
        *(int *)((char *)Xh + (ke[x] >> 16)) = (int)__builtin_amdgcn_perm(
            (unsigned)(R + (int)ke[x] + K5x), (unsigned)R, 0x05040100u);
      }
    }
    // children of every slot: f_u + Xa | g_v + Xb in int16 halves
#pragma unroll
    for (int x = 0; x < RMAX; ++x) {
      if (x < r) {
        const int j = __builtin_amdgcn_readlane(jq, x);
        const int h = Xh[x * 64];
        const int fw = Fu[j], gw = Gv[j];
        acc[x] = pk_max(acc[x], pk_add((int)__builtin_amdgcn_perm((unsigned)gw, (unsigned)fw,
                                                                  0x07060100u),
                                       h));
      }
    }
  }
  const int t = transpose_pkmax<RMAX>(acc, lane, tsrc);
  const int val = member ? max(lb1, t) : kInt32Max;
  if (member) {
    const int o = (bwd ? stride : 0) + q;
    lbrow[o] = val;
    prow[o] = val >= ub;
  }
  fill_invalid(lbrow, prow, nullptr, stride, r, lane, 64);
  if (dirp) {
    const int cmn = wave_min_xl(val);
    const uint64_t at = __ballot(member && val == cmn);
    const int cf = __popc((uint32_t)at), cb = __popc((uint32_t)(at >> 32));
    const int s = half_sum(member ? val : 0);  // bounds below 2^15: sums below 2^20
    MinMin mm;
    mm.init();
    mm.merge(cmn, cf, cb, __builtin_amdgcn_readlane(s, 0), __builtin_amdgcn_readlane(s, 32));
    if (lane == 0) *dirp = (uint8_t)mm.dir();
  }
  wave_sync();  // the next parent rewrites this wave's tables
}

template <int NMAX, int RMAX>
__global__ void __launch_bounds__(1024)
k_lb2d(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
       uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  __shared__ int blist[kBinListCap + 16];
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw >= count) return;
  const DeepLayout L{Ppad, I.m, RMAX};
  const DeepLds<NMAX> S(sm, L, w);
  lb2q_stage<NMAX, true>(I, Ppad, S);
  lb2d_stage_pos<NMAX>(I, Ppad, S.pos);
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int n = I.n, m = I.m, ns = pool.n;
  const int tsrc = tp_source<RMAX>(lane);
  parent_loop(pool, count, n, m, costs, lane, w, nw, blist, [&](int par, const PackFetch &F) {
    lb2d_parent<NMAX, RMAX>(I, Ppad, S, F, ns, ub, out_lb + (size_t)par * 2 * ns,
                            out_prune + (size_t)par * 2 * ns,
                            pool.dir ? pool.dir + par : nullptr, lane, tsrc);
  });
}

// ------------------------------------------------------------ wide LB2
// Full LB2 for 32 < n <= NMAX (64 or 128) with 16-bit X, one wave per
// parent and lanes = pairs as in k_lb2q.  The per-pair scan runs over the n
// Johnson positions in chunks of CH: a first sweep keeps only the running Y
// and prefix maximum at each chunk start; the second sweep takes the chunks
// from last to first, repeats each chunk's forward steps in registers and
// then its backward steps, so the suffix maximum carries across chunks.  The
// quick-format entries stream from the instance's global table
// [pass][position][64 lanes] (L2-resident, coalesced).  The children's
// pair maxima of both directions live in one register per job as two int16
// halves (forward low, backward high): every pair term of a child is a
// lower bound of one of its completions, hence at most (n + m - 1) max p,
// below 2^15 when 16-bit X applies.
// Tables are sized by the largest n and m they serve (nj, mmax), so that a
// 100-job, 20-machine class fits four waves per CU.
struct WideLayout {
  int ppad, nj, mmax;  // padded pairs, rows of X (largest n), machines
  int subset = 0;      // subset bounds: a list of the selected pairs per wave
  // start-time rows: odd, and long enough for reads up to job n + 2
  __host__ __device__ int row() const { return (nj + 3) | 1; }
  // scan chunk length: the 128-job variant keeps fewer positions in registers
  __host__ __device__ static constexpr int chunk_len(int nmax) { return nmax >= 128 ? 8 : 16; }
  __host__ __device__ int chunks(int nmax) const {
    return (nj + chunk_len(nmax) - 1) / chunk_len(nmax);
  }
  __host__ __device__ size_t block_bytes(int nmax) const {
    return align16((size_t)ppad * 4) + align16((size_t)mmax * nmax * 2);
  }
  __host__ __device__ size_t wave_bytes(int nmax) const {
    return align16((size_t)(nj + 3) * 64 * 4) + align16((size_t)mmax * row() * 4) +
           align16((size_t)chunks(nmax) * 64 * 4) + align16((size_t)2 * mmax * 8) +
           align16((size_t)3 * mmax * 4) + align16((size_t)nj * 4) +
           (subset ? align16((size_t)ppad * 2) : 0);
  }
};

template <int NMAX>
struct WideLds {
  int *uv;         // block: pair -> u | v << 8
  unsigned short *pt;  // block: p by [machine][job] (below 2^15 with 16-bit X)
  int ROW;         // row length of FB
  int *X;          // [nj + 3][64]: xa | xb << 16 by job (row n: padding sink; rows
                   // n + 1, n + 2: read, never used, by the last group of four jobs)
  int *FB;         // [m][ROW]: f (forward, low half) | g (backward, high half) by machine
  int *ST;         // [chunks][64]: Y | prefix max << 16 at each chunk start (both int16)
  int2 *HTf, *HTb;
  int *c1, *c2, *rr, *inv;
  short *sel;  // subset bounds: the selected pair indices in order
  __device__ WideLds(unsigned char *sm, const WideLayout &L, int w) {
    ROW = L.row();
    uv = (int *)sm;
    size_t off = align16((size_t)L.ppad * 4);
    pt = (unsigned short *)(sm + off);
    off += align16((size_t)L.mmax * NMAX * 2);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(NMAX);
    X = (int *)wb;
    wb += align16((size_t)(L.nj + 3) * 64 * 4);
    FB = (int *)wb;
    wb += align16((size_t)L.mmax * ROW * 4);
    ST = (int *)wb;
    wb += align16((size_t)L.chunks(NMAX) * 64 * 4);
    HTf = (int2 *)wb;
    HTb = HTf + L.mmax;
    wb += align16((size_t)2 * L.mmax * 8);
    c1 = (int *)wb;
    c2 = c1 + L.mmax;
    rr = c2 + L.mmax;
    wb += align16((size_t)3 * L.mmax * 4);
    inv = (int *)wb;
    wb += align16((size_t)L.nj * 4);
    sel = (short *)wb;
  }
};

// Block-cooperative staging of one instance for the wide kernels (no
// barrier inside): pair machines and the processing times by machine.
template <int NMAX>
__device__ void lb2w_stage(const DevInst &I, int Ppad, const WideLds<NMAX> &S) {
  const int n = I.n, m = I.m, P = I.P;
  for (int x = threadIdx.x; x < Ppad; x += blockDim.x) {
    const int q = x < P ? x : 0;
    S.uv[x] = P > 0 ? ((int)I.pu[q] | ((int)I.pv[q] << 8)) : 0;
  }
  for (int x = threadIdx.x; x < m * NMAX; x += blockDim.x) {
    const int s = x / NMAX, k = x - s * NMAX;
    S.pt[x] = (unsigned short)(k < n ? I.p[k * m + s] : 0);
  }
}

// -1 if job k is a member (bit k of the mask words), else 0.
template <int NW>
__device__ __forceinline__ int member_ng(const uint64_t (&um)[NW], unsigned k) {
  if constexpr (NW == 1) {
    return __builtin_amdgcn_sbfe((int)(uint32_t)(um[0] >> (k & 63u)), 0, 1);
  } else {  // both words shifted, then a bitwise select (no indexed register array)
    const uint32_t b0 = (uint32_t)(um[0] >> (k & 63u)), b1 = (uint32_t)(um[1] >> (k & 63u));
    const uint32_t hi = (uint32_t)__builtin_amdgcn_sbfe((int)k, 6, 1);
    return __builtin_amdgcn_sbfe((int)((b1 & hi) | (b0 & ~hi)), 0, 1);
  }
}

// One chunk of the second sweep: the forward steps from the chunk-start
// state (Y, Pm), then the backward steps with the suffix maximum Sm, storing
// xa | xb << 16 in the job's row of X.  RAGGED: positions from rem on lie
// past n (they count as non-members and write the padding sink, row n).
template <int NW, int CH, bool RAGGED>
__device__ __forceinline__ void lb2w_chunk(const uint2 *__restrict__ ec, int rem,
                                           const uint64_t (&um)[NW], int n, int K5x, int Y,
                                           int Pm, int &Sm, int *__restrict__ Xh) {
  constexpr int NEGX = -(1 << 14);
  int pt[CH];       // (prefix maximum - E) | term << 16, int16 halves (as in the quick kernel)
  unsigned ke[CH];  // E in bits 0-15, job << 24: (ke >> 16) is the byte offset of its row of X
  uint2 ev[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) ev[i] = ec[(!RAGGED || i < rem ? i : rem - 1) * 64];
  __builtin_amdgcn_sched_barrier(0);  // all CH loads in flight before the first use
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    const bool in = !RAGGED || i < rem;
    const uint2 e = ev[i];
    int ng = member_ng<NW>(um, e.y);
    if (RAGGED) ng &= in ? -1 : 0;
    const int tt = Y + (int)(e.y >> 16);
    const int term = (tt & ng) | (NEGX & ~ng);
    pt[i] = (int)__builtin_amdgcn_perm((unsigned)term, (unsigned)(Pm - (int)e.x), 0x05040100u);
    Pm = max(Pm, term);
    Y = mad_i16(ng, (int)e.x, Y);
    ke[i] = in ? e.x : (e.x & 0xffffu) | ((unsigned)n << 24);
  }
  // the suffix maximum in both halves; each step leaves Xa low and the
  // suffix maximum with this term high
  int R = (int)__builtin_amdgcn_perm((unsigned)Sm, (unsigned)Sm, 0x05040100u);
#pragma unroll
  for (int i = CH - 1; i >= 0; --i) {
    R = pk_max_hi(pt[i], R);
    *(int *)((char *)Xh + (ke[i] >> 16)) =
        (int)__builtin_amdgcn_perm((unsigned)(R + (int)ke[i] + K5x), (unsigned)R, 0x05040100u);
  }
  Sm = R >> 16;
}

// SUBSET: only the pairs whose bit is set in mw[0 .. words) (compacted into
// S.sel in index order; lanes past the selection repeat its first pair), their
// entries gathered from the instance table by pair index.
template <int NMAX, bool SUBSET = false>
__device__ void lb2w_parent(const DevInst &I, int Ppad, const WideLds<NMAX> &S,
                            const uint8_t *__restrict__ row, int a, int b,
                            const int *__restrict__ cs, int stride, int ub,
                            int *__restrict__ lbrow, uint8_t *__restrict__ prow,
                            uint8_t *__restrict__ dirp, int lane,
                            const uint32_t *__restrict__ mw = nullptr, int words = 0) {
  const int ROW = S.ROW;
  constexpr int CH = WideLayout::chunk_len(NMAX);
  constexpr int NC = NMAX / 32;  // 32-job chunks of the lane-per-job steps
  constexpr int NW = NMAX / 64;  // 64-bit membership words
  constexpr int NEGX = -(1 << 14);
  const int n = I.n, m = I.m, P = I.P;
  const int r = n - a - b;
  if (r < 1 || cs[0] < 0) {  // flagged by the costs kernel: not a valid node
    fill_invalid(lbrow, prow, nullptr, stride, 0, lane, 64);
    if (dirp && lane == 0) *dirp = 0;
    return;
  }
  for (int x = lane; x < n; x += 64) S.inv[row[x]] = x;
  for (int x = lane; x < m; x += 64) {
    const int C1 = cs[x], C2 = cs[m + x], R = cs[2 * m + x];
    S.c1[x] = C1;
    S.c2[x] = C2;
    S.rr[x] = R;
    S.HTf[x] = make_int2(C1, R + C2);
    S.HTb[m - 1 - x] = make_int2(C2, C1 + R);
  }
  wave_sync();
  uint64_t um[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int k = 64 * w + lane;
    const int slot = k < n ? S.inv[k] - a : -1;
    um[w] = __ballot(slot >= 0 && slot < r);
  }
  // LB1 of both children of each member job and their start times: lane
  // q < 32 takes the forward child of job 32c + q, lane 32 + q its backward
  // child (machines reversed; g is stored under the machine's own index)
  const bool bwd = lane >= 32;
  int lb1[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    lb1[c] = 0;
    if (!((um[c >> 1] >> (32 * (c & 1))) & 0xffffffffull)) continue;
    const int k = 32 * c + (lane & 31);
    if (!((um[c >> 1] >> (k & 63)) & 1ull)) continue;
    const int2 *HT = bwd ? S.HTb : S.HTf;
    unsigned short *fb = (unsigned short *)S.FB + 2 * k + (bwd ? 1 + 2 * (m - 1) * ROW : 0);
    const int fstep = bwd ? -2 * ROW : 2 * ROW;
    const unsigned short *PT = S.pt + k + (bwd ? (m - 1) * NMAX : 0);
    const int pstep = bwd ? -NMAX : NMAX;
    int cc = 0, l = 0;
#pragma unroll 4
    for (int s = 0; s < m; ++s) {
      const int2 ht = HT[s];
      const int f = max(cc, ht.x);
      cc = f + PT[s * pstep];
      fb[s * fstep] = (unsigned short)f;
      l = max(l, f + ht.y);
    }
    lb1[c] = l;
  }
  wave_sync();
  int acc[NMAX];  // two int16 maxima per job: forward | backward << 16
#pragma unroll
  for (int q = 0; q < NMAX; ++q) {  // set once (not repeated on the path into the loop)
    acc[q] = (int)0x80008000u;
    asm volatile("" : "+v"(acc[q]));
  }
  int nsel = 0;
  if constexpr (SUBSET) {  // selected pairs in index order, compacted by ballot
    for (int base = 0; base < P; base += 64) {
      const int q = base + lane;
      const bool on = q < P && ((mw[q >> 5] >> (q & 31)) & 1u);
      const uint64_t bal = __ballot(on);
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (on) S.sel[nsel + pos] = (short)q;
      nsel += __popcll(bal);
    }
    wave_sync();
  }
  // leaves: LB2 = LB1
  const int npass = r < 2 ? 0 : SUBSET ? nsel : (P > 0 ? Ppad : 0);
  const int nch = (n + CH - 1) / CH;
  int *__restrict__ Xh = S.X + lane;
  int *__restrict__ st = S.ST + lane;
  for (int pc = 0; pc < npass; pc += 64) {
    // the masks are opaque per pass, so that the per-group branch conditions
    // below are recomputed (two scalar ops) rather than held in registers
#pragma unroll
    for (int w = 0; w < NW; ++w) asm volatile("" : "+s"(um[w]));
    int pi = pc + lane;
    if constexpr (SUBSET) pi = S.sel[pi < nsel ? pi : 0];
    const int uvp = S.uv[pi];
    const int u = uvp & 0xff, v = uvp >> 8;
    const int K4 = S.rr[v] + S.c2[v], K5 = S.c1[u] + S.rr[v];
    const int K5x = K5 - K4;  // the high half is Xb + K5 (K4 is already inside)
    const uint2 *__restrict__ eb = I.entq + (size_t)(pi >> 6) * n * 64 + (pi & 63);
    // first sweep: Y and the prefix maximum at each chunk start
    int Y = K4, Pm = NEGX;
    for (int ch = 0; ch < nch - 1; ++ch) {
      // Y lies in [0, (n + m) max p) and Pm in it or NEGX: both fit int16
      st[ch * 64] = (int)__builtin_amdgcn_perm((unsigned)Pm, (unsigned)Y, 0x05040100u);
      const uint2 *ec = eb + ch * CH * 64;
      uint2 ev[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) ev[i] = ec[i * 64];
      __builtin_amdgcn_sched_barrier(0);  // all CH loads in flight before the first use
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const uint2 e = ev[i];
        const int ng = member_ng<NW>(um, e.y);
        const int tt = Y + (int)(e.y >> 16);
        Pm = max(Pm, (tt & ng) | (NEGX & ~ng));
        Y = mad_i16(ng, (int)e.x, Y);
      }
    }
    // second sweep, chunks from last to first (only the last can be ragged)
    int Sm = NEGX;
    {
      const int ch = nch - 1, rem = n - ch * CH;
      if (rem < CH)
        lb2w_chunk<NW, CH, true>(eb + ch * CH * 64, rem, um, n, K5x, Y, Pm, Sm, Xh);
      else
        lb2w_chunk<NW, CH, false>(eb + ch * CH * 64, rem, um, n, K5x, Y, Pm, Sm, Xh);
    }
    for (int ch = nch - 2; ch >= 0; --ch) {
      const int s2 = st[ch * 64];
      lb2w_chunk<NW, CH, false>(eb + ch * CH * 64, CH, um, n, K5x, s2 & 0xffff, s2 >> 16, Sm,
                                Xh);
    }
    // children of the member jobs, four at a time: f_u + xa | g_v + xb
    const int *Fu = S.FB + u * ROW;
    const int *Gv = S.FB + v * ROW;
#pragma unroll
    for (int g = 0; g < NMAX; g += 4) {
      if ((um[g >> 6] >> (g & 63)) & 0xfull) {
        int h[4], fw[4], gw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // a group holding a member ends before row n + 3
          h[j] = Xh[(g + j) * 64];
          fw[j] = Fu[g + j];
          gw[j] = Gv[g + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)  // sums first: no wait state before each maximum
          h[j] = pk_add((int)__builtin_amdgcn_perm((unsigned)gw[j], (unsigned)fw[j], 0x07060100u),
                        h[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[g + j] = pk_max(acc[g + j], h[j]);
      }
    }
  }
  // per-job maxima over the pairs, 32 jobs at a time; outputs; MinMin
  int vmin = kInt32Max, slo = 0, shi = 0;
  int val[NC];
  bool mem[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int k = 32 * c + (lane & 31);
    const bool member = (um[c >> 1] >> (k & 63)) & 1ull;
    mem[c] = member;
    val[c] = kInt32Max;
    if (!((um[c >> 1] >> (32 * (c & 1))) & 0xffffffffull)) continue;
    int t;
    if (c == 0) t = transpose_pkmax32<0>(acc, lane);
    else if (c == 1) t = transpose_pkmax32<(NC > 1 ? 32 : 0)>(acc, lane);
    else if (c == 2) t = transpose_pkmax32<(NC > 2 ? 64 : 0)>(acc, lane);
    else t = transpose_pkmax32<(NC > 3 ? 96 : 0)>(acc, lane);
    const int v = member ? max(lb1[c], t) : kInt32Max;
    if (member) {
      const int o = (bwd ? stride : 0) + S.inv[k] - a;
      lbrow[o] = v;
      prow[o] = v >= ub;
      slo += v & 0xffff;
      shi += v >> 16;
    }
    val[c] = v;
    vmin = min(vmin, v);
  }
  fill_invalid(lbrow, prow, nullptr, stride, r, lane, 64);
  if (dirp) {
    const int cmn = wave_min_xl(vmin);
    int cf = 0, cb = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint64_t at = __ballot(mem[c] && val[c] == cmn);
      cf += __popc((uint32_t)at);
      cb += __popc((uint32_t)(at >> 32));
    }
    const int hlo = half_sum(slo), hhi = half_sum(shi);
    const long long sf = ((long long)__builtin_amdgcn_readlane(hhi, 0) << 16) +
                         __builtin_amdgcn_readlane(hlo, 0);
    const long long sb = ((long long)__builtin_amdgcn_readlane(hhi, 32) << 16) +
                         __builtin_amdgcn_readlane(hlo, 32);
    MinMin mm;
    mm.init();
    mm.merge(cmn, cf, cb, sf, sb);
    if (lane == 0) *dirp = (uint8_t)mm.dir();
  }
  wave_sync();  // the next parent rewrites this wave's tables
}

// Single instance: each block stages the pair machines and processing
// times, then its waves take parents in a grid-stride loop.  The 128-job
// variant runs one wave per SIMD (its LDS tables allow about three waves per
// CU anyway), which leaves it the accumulation registers beyond 256.
template <int NMAX, bool SUBSET>
__global__ void __launch_bounds__(NMAX >= 128 ? 256 : 512)
k_lb2w(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
       uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw >= count) return;  // no parent for this block: skip the staging
  WideLayout L{Ppad, I.n, I.m};
  L.subset = SUBSET;
  const WideLds<NMAX> S(sm, L, w);
  lb2w_stage<NMAX>(I, Ppad, S);
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int m = I.m;
  for (int it = blockIdx.x * nw + w; it < count; it += gridDim.x * nw) {
    const int par = pool.index ? pool.index[it] : it;
    const int ns = pool.n;  // row stride (>= n)
    lb2w_parent<NMAX, SUBSET>(I, Ppad, S, pool.perm + (size_t)par * ns, pool.d1[par],
                              pool.d2[par], costs + (size_t)par * 3 * m, ns, ub,
                              out_lb + (size_t)par * 2 * ns, out_prune + (size_t)par * 2 * ns,
                              pool.dir ? pool.dir + par : nullptr, lane,
                              SUBSET ? mask_row(pool, par) : nullptr, pool.mask_words);
  }
}

// ------------------------------------------------------- packed subset LB2
// Subset LB2 with G parents per wave for n <= NMAX <= 32 and 16-bit X (the
// method of k_lb2q): group g of L = 64 / G consecutive lanes takes parent g,
// lane l the l-th pair of the parent's selection (lanes past it repeat the
// first), so a selection of at most L pairs costs one scan pass for G
// parents.  Per-child maxima are folded within each group; MinMin reduces
// within each group.  Per parent and wave: start times FB [m][ROW] with f
// (forward child, by machine) in the low and g (backward child, by machine)
// in the high 16 bits (both below 2^15 when 16-bit X applies), C1, C2, R,
// the inverse permutation, the children's LB1 and the compacted selection.
struct PackLayout {
  int ppad, mmax;
  __host__ __device__ static constexpr int row(int nmax) { return nmax | 1; }
  __host__ __device__ size_t block_bytes(int nmax) const {
    return align16((size_t)nmax * ppad * 8) + align16((size_t)ppad * 4) +
           align16((size_t)2 * mmax * 32 * 4);
  }
  __host__ __device__ size_t parent_bytes(int nmax) const {
    return align16((size_t)mmax * row(nmax) * 4) + align16((size_t)3 * mmax * 4) + 32 * 4 +
           64 * 4 + align16((size_t)ppad * 2) + align16((size_t)2 * mmax * 8);
  }
  __host__ __device__ size_t wave_bytes(int nmax, int g) const {
    return align16((size_t)nmax * 64 * 4) + (size_t)g * parent_bytes(nmax);
  }
};

template <int NMAX>
struct PackParent {
  uint32_t *fb;  // [m][ROW]: f | g << 16
  int *c1, *c2, *rr, *inv, *lb1;
  int16_t *sel;
  int2 *htf, *htb;  // per scan step: (head, tail + remaining) forward, backward
};

template <int NMAX, int G>
struct PackLds {
  uint2 *ent;
  int *uv, *pt, *pr;
  int *X;
  unsigned char *pb;  // parent 0's block; parent g's starts g * pstride later
  int pstride, mmax, o_c, o_inv, o_lb1, o_sel, o_ht;
  __device__ PackLds(unsigned char *sm, const PackLayout &L, int w) {
    constexpr int ROW = PackLayout::row(NMAX);
    ent = (uint2 *)sm;
    size_t off = align16((size_t)NMAX * L.ppad * 8);
    uv = (int *)(sm + off);
    off += align16((size_t)L.ppad * 4);
    pt = (int *)(sm + off);
    pr = pt + L.mmax * 32;
    off += align16((size_t)2 * L.mmax * 32 * 4);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(NMAX, G);
    X = (int *)wb;
    pb = wb + align16((size_t)NMAX * 64 * 4);
    pstride = (int)L.parent_bytes(NMAX);
    mmax = L.mmax;
    o_c = (int)align16((size_t)L.mmax * ROW * 4);
    o_inv = o_c + (int)align16((size_t)3 * L.mmax * 4);
    o_lb1 = o_inv + 32 * 4;
    o_sel = o_lb1 + 64 * 4;
    o_ht = o_sel + (int)align16((size_t)L.ppad * 2);
  }
  // tables of parent g of this wave (g may differ between lanes)
  __device__ PackParent<NMAX> parent(int g) const {
    unsigned char *b = pb + (size_t)g * pstride;
    PackParent<NMAX> P;
    P.fb = (uint32_t *)b;
    P.c1 = (int *)(b + o_c);
    P.c2 = P.c1 + mmax;
    P.rr = P.c2 + mmax;
    P.inv = (int *)(b + o_inv);
    P.lb1 = (int *)(b + o_lb1);
    P.sel = (int16_t *)(b + o_sel);
    P.htf = (int2 *)(b + o_ht);
    P.htb = P.htf + mmax;
    return P;
  }
};

// Reductions within groups of L consecutive lanes (L = 16 or 32).
template <int L>
__device__ __forceinline__ int group_min(int x) {
  if constexpr (L == 32) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = min((int)r[0], (int)r[1]);
  }
  x = min(x, dpp_partner<8>(x));
  x = min(x, dpp_partner<4>(x));
  x = min(x, dpp_partner<2>(x));
  return min(x, dpp_partner<1>(x));
}

template <int L>
__device__ __forceinline__ int group_sum(int x) {
  if constexpr (L == 32) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = (int)r[0] + (int)r[1];
  }
  x += dpp_partner<8>(x);
  x += dpp_partner<4>(x);
  x += dpp_partner<2>(x);
  return x + dpp_partner<1>(x);
}

// acc[0..L) per lane -> lane p of each group holds the group maximum of acc[p].
template <int L>
__device__ __forceinline__ int group_transpose_max(int (&acc)[L], int lane) {
  if constexpr (L == 32) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const auto r = __builtin_amdgcn_permlane16_swap(acc[j], acc[16 + j], false, false);
      acc[j] = max((int)r[0], (int)r[1]);
    }
  }
  transpose_max_dpp<8>(acc, lane);
  return acc[0];
}

// Per group of L lanes (32 or 16): lane l ends with the group maximum of
// blk[l], the NJ <= L jobs combined without padding and gathered back to
// their own lanes from src = tp_group_source<L, NJ>(lane) (a full block
// already ends in place).
template <int L, int NJ>
__device__ __forceinline__ int group_transpose_pkmax(int (&blk)[L], int lane, int src) {
  constexpr int TOP = L == 32 ? 4 : 3;
  static_assert(L == 32 || L == 16, "two or four parents per wave");
  tp_steps<NJ, TOP>(blk, lane);
  if constexpr (NJ == L) return blk[0];
  return __shfl(blk[0], src, kWave);
}

// The gather lanes of the blocks of L jobs that cover NMAX jobs.
template <int NMAX, int L>
struct GroupSrc {
  static constexpr int NB = (NMAX + L - 1) / L;
  int s[NB];
  __device__ explicit GroupSrc(int lane) { fill<0>(lane); }
  template <int B>
  __device__ void fill(int lane) {
    if constexpr (B < NB) {
      s[B] = tp_group_source<L, (NMAX - B * L < L ? NMAX - B * L : L)>(lane);
      fill<B + 1>(lane);
    }
  }
};

// Block B of L jobs: job B * L + l ends in lane l of each group.
template <int B, int L, int NMAX, int NB>
__device__ __forceinline__ void group_blocks(const int (&acc)[NMAX], int (&t)[NB],
                                             const GroupSrc<NMAX, L> &src, int lane) {
  if constexpr (B < NB) {
    constexpr int NJ = NMAX - B * L < L ? NMAX - B * L : L;
    int blk[L];
#pragma unroll
    for (int j = 0; j < NJ; ++j) blk[j] = acc[B * L + j];
    t[B] = group_transpose_pkmax<L, NJ>(blk, lane, src.s[B]);
    group_blocks<B + 1, L, NMAX, NB>(acc, t, src, lane);
  }
}

// One wave bounds the pool rows rows[0 .. G) (-1: none) from their prefetched
// inputs F.
template <int NMAX, int G>
__device__ void lb2s_wave(const DevInst &I, int Ppad, const PackLds<NMAX, G> &S,
                          const DevPool &pool, const int (&rows)[G], const PackFetch (&F)[G],
                          int ub, int *__restrict__ out_lb, uint8_t *__restrict__ out_prune,
                          int lane, const GroupSrc<NMAX, 64 / G> &tsrc) {
  constexpr int L = 64 / G;
  constexpr int ROW = PackLayout::row(NMAX);
  constexpr int NB = (NMAX + L - 1) / L;  // blocks of L jobs (both directions per job)
  constexpr int NEGX = -(1 << 14);
  const int n = I.n, m = I.m, P = I.P, ns = pool.n;
  const int gl = lane / L, l = lane % L;  // this lane's group and position in it
  // per parent: validity, tables in LDS
  int a_[G], r_[G];
  bool ok_[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int a = __builtin_amdgcn_readfirstlane(F[g].d1);
    const int b = __builtin_amdgcn_readfirstlane(F[g].d2);
    a_[g] = a;
    r_[g] = n - a - b;
    // cs[0] < 0 flags a row that the costs kernel found invalid
    ok_[g] = rows[g] >= 0 && r_[g] >= 1 && __builtin_amdgcn_readfirstlane(F[g].c1) >= 0;
    if (ok_[g]) {
      const PackParent<NMAX> Q = S.parent(g);
      if (lane < n) Q.inv[F[g].rb] = lane;
      if (lane < m) {
        Q.c1[lane] = F[g].c1;
        Q.c2[lane] = F[g].c2;
        Q.rr[lane] = F[g].rr;
        Q.htf[lane] = make_int2(F[g].c1, F[g].rr + F[g].c2);
        Q.htb[m - 1 - lane] = make_int2(F[g].c2, F[g].c1 + F[g].rr);
      }
    }
  }
  wave_sync();
  // membership masks (uniform per parent), the children's LB1 and start times
  uint32_t um[G];
  uint32_t uany = 0;
  const int k = lane & 31;
  const bool bwd = lane >= 32;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    um[g] = 0;
    if (!ok_[g]) continue;
    const PackParent<NMAX> Q = S.parent(g);
    const int slot = k < n ? Q.inv[k] - a_[g] : -1;
    um[g] = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(uint32_t)__ballot(!bwd && slot >= 0 && slot < r_[g]));
    uany |= um[g];
    int lb1 = 0;
    if (k < NMAX) {
      const int2 *HT = bwd ? Q.htb : Q.htf;
      const int *PT = (bwd ? S.pr : S.pt) + k;
      // in scan order: f of machine s into the low half of [s][k], g of
      // machine m - 1 - s into the high half (one constant stride)
      unsigned short *fb = (unsigned short *)Q.fb + 2 * k + (bwd ? 1 : 0);
      int c = 0;
#pragma unroll 4
      for (int s = 0; s < m; ++s) {
        const int2 ht = HT[s];
        const int f = max(c, ht.x);
        c = f + PT[s * 32];
        fb[s * 2 * ROW] = (unsigned short)f;
        lb1 = max(lb1, f + ht.y);
      }
    }
    Q.lb1[lane] = lb1;
  }
  // compacted selections: pair indices whose bit is set, in index order
  int nsel[G];
  int nmax_sel = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    nsel[g] = 0;
    if (!ok_[g] || r_[g] < 2) continue;  // leaves: LB2 = LB1, no pair needed
    for (int base = 0; base < P; base += 64) {
      const int pi = base + lane;
      const uint32_t w = (uint32_t)__shfl((int)F[g].mw, (pi >> 5) & 63, kWave);
      const bool on = pi < P && ((w >> (pi & 31)) & 1u);
      const uint64_t bal = __ballot(on);
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (on) S.parent(g).sel[nsel[g] + pos] = (int16_t)pi;
      nsel[g] += __popcll(bal);
    }
    nmax_sel = max(nmax_sel, nsel[g]);
  }
  wave_sync();
  // this lane's parent
  uint32_t umask = 0;
  int nsg = 0;
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (gl == g) {
      umask = um[g];
      nsg = nsel[g];
    }
  const PackParent<NMAX> Q = S.parent(gl);  // this lane's parent
  int acc[NMAX];  // pair maxima per job: forward | backward << 16 (int16 halves)
#pragma unroll
  for (int q = 0; q < NMAX; ++q) {  // set once (not repeated on the path into the loop)
    acc[q] = (int)0x80008000u;
    asm volatile("" : "+v"(acc[q]));
  }
  int *__restrict__ Xh = S.X + lane;
  for (int pc = 0; pc < nmax_sel; pc += L) {
    const int idx = pc + l;
    const int pi = nsg > 0 ? Q.sel[idx < nsg ? idx : 0] : 0;
    const int uvp = S.uv[pi];
    const int u = uvp & 0xff, v = uvp >> 8;
    const int K4 = Q.rr[v] + Q.c2[v], K5 = Q.c1[u] + Q.rr[v];
    const int *Fu = lds_opaque((const int *)Q.fb + u * ROW);  // f_u in the low halves
    const int *Gv = lds_opaque((const int *)Q.fb + (m - 1 - v) * ROW);  // g_v, high halves
    const uint2 *__restrict__ eb = S.ent + (pi >> 6) * (NMAX * 64) + (pi & 63);
    // the scans of the quick kernel with 16-bit X: per position the pair
    // (prefix maximum - E, term) and E | job << 24, then one packed maximum
    // per position against the suffix maximum
    int pt[NMAX];
    unsigned ke[NMAX];
    int Y = K4, Pm = NEGX;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      const uint2 e = eb[i * 64];
      const int ng = __builtin_amdgcn_sbfe((int)umask, (int)e.y, 1);
      const int tt = Y + (int)(e.y >> 16);
      const int term = (tt & ng) | (NEGX & ~ng);
      pt[i] = (int)__builtin_amdgcn_perm((unsigned)term, (unsigned)(Pm - (int)e.x), 0x05040100u);
      Pm = max(Pm, term);
      Y = mad_i16(ng, (int)e.x, Y);
      ke[i] = e.x;
    }
    const int K5x = K5 - K4;
    int R = (int)0xC000C000u;  // NEGX in both halves
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
      R = pk_max_hi(pt[i], R);
      *(int *)((char *)Xh + (ke[i] >> 16)) =
          (int)__builtin_amdgcn_perm((unsigned)(R + (int)ke[i] + K5x), (unsigned)R, 0x05040100u);
    }
#pragma unroll
    for (int g0 = 0; g0 < NMAX; g0 += 4) {
      if (uany & (0xfu << g0)) {
        int h[4], fw[4], gw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (g0 + j < NMAX) {
            h[j] = Xh[(g0 + j) * 64];
            fw[j] = Fu[g0 + j];
            gw[j] = Gv[g0 + j];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (g0 + j < NMAX)
            h[j] = pk_add(
                (int)__builtin_amdgcn_perm((unsigned)gw[j], (unsigned)fw[j], 0x07060100u), h[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (g0 + j < NMAX) acc[g0 + j] = pk_max(acc[g0 + j], h[j]);
        }
      }
    }
  }
  // fold over each group's lanes: job b * L + j of block b
  int t[NB];
  group_blocks<0, L, NMAX, NB>(acc, t, tsrc, lane);
  // outputs and MinMin, per group: lane l of block b takes job b * L + l in
  // both directions
  int vmin = kInt32Max;
  int valf[NB], valb[NB];
  bool mem[NB];
  const bool okg = [&] {
    bool o = false;
#pragma unroll
    for (int g = 0; g < G; ++g) o = gl == g ? ok_[g] : o;
    return o;
  }();
  int ag = 0, rg = 0;
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (gl == g) {
      ag = a_[g];
      rg = r_[g];
    }
  int par = -1;
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (gl == g) par = rows[g];
  int *lbrow = out_lb + (size_t)(par >= 0 ? par : 0) * 2 * ns;
  uint8_t *prow = out_prune + (size_t)(par >= 0 ? par : 0) * 2 * ns;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int q = b * L + l;
    const bool member = okg && q < NMAX && q < n && ((umask >> (q & 31)) & 1u);
    const int sl = member ? Q.inv[q] - ag : 0;
    const int pf = nsg > 0 ? (int)(short)(t[b] & 0xffff) : kNeg;
    const int pb = nsg > 0 ? t[b] >> 16 : kNeg;
    const int vf = member ? max(Q.lb1[q & 31], pf) : kInt32Max;
    const int vb = member ? max(Q.lb1[32 + (q & 31)], pb) : kInt32Max;
    if (member) {
      lbrow[sl] = vf;
      prow[sl] = vf >= ub;
      lbrow[ns + sl] = vb;
      prow[ns + sl] = vb >= ub;
    }
    valf[b] = vf;
    valb[b] = vb;
    mem[b] = member;
    vmin = min(vmin, min(vf, vb));
  }
  const int cmn = group_min<L>(vmin);
  int cf = 0, cb = 0, flo = 0, fhi = 0, blo = 0, bhi = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (mem[b]) {
      cf += valf[b] == cmn;
      flo += valf[b] & 0xffff;
      fhi += valf[b] >> 16;
      cb += valb[b] == cmn;
      blo += valb[b] & 0xffff;
      bhi += valb[b] >> 16;
    }
  }
  cf = group_sum<L>(cf);
  cb = group_sum<L>(cb);
  flo = group_sum<L>(flo);
  fhi = group_sum<L>(fhi);
  blo = group_sum<L>(blo);
  bhi = group_sum<L>(bhi);
  if (par >= 0) {
    if (okg) {
      for (int x = l; x < 2 * ns; x += L) {  // slots >= r of both directions
        const int q = x < ns ? x : x - ns;
        if (q >= rg) {
          lbrow[x] = kInt32Max;
          prow[x] = 1;
        }
      }
      if (l == 0 && pool.dir) {
        MinMin mm;
        mm.init();
        mm.merge(cmn, cf, cb, ((long long)fhi << 16) + flo, ((long long)bhi << 16) + blo);
        pool.dir[par] = (uint8_t)mm.dir();
      }
    } else {
      for (int x = l; x < 2 * ns; x += L) {
        lbrow[x] = kInt32Max;
        prow[x] = 1;
      }
      if (l == 0 && pool.dir) pool.dir[par] = 0;
    }
  }
  wave_sync();  // the next parents rewrite this wave's tables
}

// Blocks of up to 8 waves (two per SIMD, the register budget that keeps the
// G parents' state out of scratch); two parents of at most 20 jobs fit three
// waves per SIMD, and their blocks take up to 12 waves.
template <int NMAX, int G>
__global__ void __launch_bounds__(G == 2 && NMAX <= 20 ? 768 : 512)
    __attribute__((amdgpu_waves_per_eu(G == 2 && NMAX <= 20 ? 3 : 1)))
k_lb2s(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
       uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  // the wave index as a uniform value: parent indices, and the loads of their
  // depths and pool rows, stay scalar
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw * G >= count) return;  // no parent for this block
  const PackLayout L{Ppad, I.m};
  const PackLds<NMAX, G> S(sm, L, w);
  lb2q_stage<NMAX, true>(I, Ppad, S);
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int step = gridDim.x * nw * G;
  int it0 = (blockIdx.x * nw + w) * G;
  auto row_of = [&](int it) { return it < count ? (pool.index ? pool.index[it] : it) : -1; };
  const GroupSrc<NMAX, 64 / G> tsrc(lane);
  int rows[G];
  PackFetch F[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    rows[g] = row_of(it0 + g);
    F[g] = pack_fetch(pool, rows[g], I.n, I.m, costs, lane);
  }
  for (; it0 < count; it0 += step) {
    PackFetch C[G];
    int cur[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      C[g] = F[g];
      cur[g] = rows[g];
      rows[g] = row_of(it0 + step + g);
      F[g] = pack_fetch(pool, rows[g], I.n, I.m, costs, lane);
    }
    lb2s_wave<NMAX, G>(I, Ppad, S, pool, cur, C, ub, out_lb, out_prune, lane, tsrc);
  }
}

// -------------------------------------------------- packed wide subset LB2
// Subset LB2 for 32 < n <= 64 with 16-bit X and G = 2 or 4 parents per wave:
// the grouping of k_lb2s (group g of L = 64 / G lanes takes parent g, lane l
// the l-th pair of its selection, lanes past it repeating the first) over
// the entries of k_lb2w (each lane gathers its pair's quick-format entries
// from the instance table).  A selection of at most L pairs thus costs one
// scan pass for G parents instead of one pass per parent with 64 - L idle
// lanes.  The G parents' start-time tables take most of a CU's LDS, so blocks
// hold up to four waves (one per SIMD) and the scan keeps twice as many
// positions in registers as k_lb2w's: a first sweep over the first 32
// positions for the running sum and prefix maximum there, then the last
// positions and the first ones with their backward steps.
struct WsLayout {
  int ppad, nj, mmax;  // padded pairs, jobs, machines
  __host__ __device__ int row() const { return (nj + 3) | 1; }
  __host__ __device__ size_t block_bytes() const {  // pair machines, p by [machine][job]
    return align16((size_t)ppad * 4) + align16((size_t)mmax * 64 * 2);
  }
  __host__ __device__ size_t parent_bytes() const {
    return align16((size_t)mmax * row() * 4) + align16((size_t)3 * mmax * 4) +
           align16((size_t)2 * mmax * 8) + 64 * 4 + 128 * 4 + align16((size_t)ppad * 2);
  }
  __host__ __device__ size_t wave_bytes(int g) const {
    return align16((size_t)(nj + 3) * 64 * 4) + (size_t)g * parent_bytes();
  }
};

struct WsParent {
  uint32_t *fb;  // [m][ROW]: f (forward child, low half) | g (backward child, high half) by job
  int *c1, *c2, *rr;
  int2 *htf, *htb;  // per scan step: (head, tail + remaining) forward, backward
  int *inv;         // [64] position of each job in the parent's row
  int *lb1;         // [2][64]: LB1 of job 32 c + q, forward in lane q, backward in 32 + q
  int16_t *sel;     // the selected pairs in index order
};

struct WsLds {
  int *uv;             // block: pair -> u | v << 8
  unsigned short *pt;  // block: p by [machine][job] (below 2^15 with 16-bit X)
  int *X;              // wave: [nj + 3][64] xa | xb << 16 by job (row n: padding sink)
  unsigned char *pb;   // wave: parent 0's tables; parent g's start g * pstride later
  int pstride, mmax, ROW, o_c, o_ht, o_inv, o_lb1, o_sel;
  __device__ WsLds(unsigned char *sm, const WsLayout &L, int w, int G) {
    ROW = L.row();
    mmax = L.mmax;
    uv = (int *)sm;
    size_t off = align16((size_t)L.ppad * 4);
    pt = (unsigned short *)(sm + off);
    off += align16((size_t)L.mmax * 64 * 2);
    unsigned char *wb = sm + off + (size_t)w * L.wave_bytes(G);
    X = (int *)wb;
    pb = wb + align16((size_t)(L.nj + 3) * 64 * 4);
    pstride = (int)L.parent_bytes();
    o_c = (int)align16((size_t)L.mmax * ROW * 4);
    o_ht = o_c + (int)align16((size_t)3 * L.mmax * 4);
    o_inv = o_ht + (int)align16((size_t)2 * L.mmax * 8);
    o_lb1 = o_inv + 64 * 4;
    o_sel = o_lb1 + 128 * 4;
  }
  __device__ WsParent parent(int g) const {
    unsigned char *b = pb + (size_t)g * pstride;
    WsParent Q;
    Q.fb = (uint32_t *)b;
    Q.c1 = (int *)(b + o_c);
    Q.c2 = Q.c1 + mmax;
    Q.rr = Q.c2 + mmax;
    Q.htf = (int2 *)(b + o_ht);
    Q.htb = Q.htf + mmax;
    Q.inv = (int *)(b + o_inv);
    Q.lb1 = (int *)(b + o_lb1);
    Q.sel = (int16_t *)(b + o_sel);
    return Q;
  }
};

// Forward then backward steps over the cnt <= CH positions of one chunk
// (cnt uniform), from the chunk-start state (Y, Pm) and the suffix maximum
// Sm of the positions after it; stores xa | xb << 16 in each job's row of X.
// um: this lane's membership mask (its parent's, one bit per job).
template <int CH>
__device__ __forceinline__ void lb2ws_chunk(const uint2 *__restrict__ ec, int cnt, uint64_t um,
                                            int K5x, int Y, int Pm, int &Sm,
                                            int *__restrict__ Xh) {
  constexpr int NEGX = -(1 << 14);
  int pt[CH];
  unsigned ke[CH];
  uint2 ev[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i)
    if (i < cnt) ev[i] = ec[i * 64];
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    if (i < cnt) {
      const uint2 e = ev[i];
      const int ng = __builtin_amdgcn_sbfe((int)(uint32_t)(um >> (e.y & 63u)), 0, 1);
      const int tt = Y + (int)(e.y >> 16);
      const int term = (tt & ng) | (NEGX & ~ng);
      pt[i] = (int)__builtin_amdgcn_perm((unsigned)term, (unsigned)(Pm - (int)e.x), 0x05040100u);
      Pm = max(Pm, term);
      Y = mad_i16(ng, (int)e.x, Y);
      ke[i] = e.x;
    }
  }
  int R = (int)__builtin_amdgcn_perm((unsigned)Sm, (unsigned)Sm, 0x05040100u);
#pragma unroll
  for (int i = CH - 1; i >= 0; --i) {
    if (i < cnt) {
      R = pk_max_hi(pt[i], R);
      *(int *)((char *)Xh + (ke[i] >> 16)) =
          (int)__builtin_amdgcn_perm((unsigned)(R + (int)ke[i] + K5x), (unsigned)R, 0x05040100u);
    }
  }
  Sm = R >> 16;
}

// One wave bounds the pool rows rows[0 .. G) (-1: none) from their prefetched
// inputs F.
template <int G>
__device__ void lb2ws_wave(const DevInst &I, const WsLds &S, const DevPool &pool,
                           const int (&rows)[G], const PackFetch (&F)[G], int ub,
                           int *__restrict__ out_lb, uint8_t *__restrict__ out_prune, int lane,
                           const GroupSrc<64, 64 / G> &tsrc) {
  constexpr int L = 64 / G, NB = 64 / L, CH = 32;
  constexpr int NEGX = -(1 << 14);
  const int n = I.n, m = I.m, P = I.P, ns = pool.n, ROW = S.ROW;
  const int gl = lane / L, l = lane % L;  // this lane's group and position in it
  int a_[G], r_[G];
  bool ok_[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int a = __builtin_amdgcn_readfirstlane(F[g].d1);
    const int b = __builtin_amdgcn_readfirstlane(F[g].d2);
    a_[g] = a;
    r_[g] = n - a - b;
    // c1 < 0 flags a row that the costs kernel found invalid
    ok_[g] = rows[g] >= 0 && r_[g] >= 1 && __builtin_amdgcn_readfirstlane(F[g].c1) >= 0;
    if (ok_[g]) {
      const WsParent Q = S.parent(g);
      if (lane < n) Q.inv[F[g].rb] = lane;
      if (lane < m) {
        Q.c1[lane] = F[g].c1;
        Q.c2[lane] = F[g].c2;
        Q.rr[lane] = F[g].rr;
        Q.htf[lane] = make_int2(F[g].c1, F[g].rr + F[g].c2);
        Q.htb[m - 1 - lane] = make_int2(F[g].c2, F[g].c1 + F[g].rr);
      }
    }
  }
  wave_sync();
  // membership masks (one bit per job, uniform per parent), the children's
  // LB1 and start times: lane q < 32 the forward child of job 32 c + q, lane
  // 32 + q its backward child (machines reversed, g stored under the
  // machine's own index)
  uint64_t um[G];
  uint64_t uany = 0;
  const bool bwd = lane >= 32;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    um[g] = 0;
    if (!ok_[g]) continue;
    const WsParent Q = S.parent(g);
    const int slot = lane < n ? Q.inv[lane] - a_[g] : -1;
    um[g] = __ballot(slot >= 0 && slot < r_[g]);
    uany |= um[g];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      int lb = 0;
      const int k = 32 * c + (lane & 31);
      if ((um[g] >> k) & 1ull) {
        const int2 *HT = bwd ? Q.htb : Q.htf;
        unsigned short *fb = (unsigned short *)Q.fb + 2 * k + (bwd ? 1 + 2 * (m - 1) * ROW : 0);
        const int fstep = bwd ? -2 * ROW : 2 * ROW;
        const unsigned short *PT = S.pt + k + (bwd ? (m - 1) * 64 : 0);
        const int pstep = bwd ? -64 : 64;
        int cc = 0;
#pragma unroll 4
        for (int s = 0; s < m; ++s) {
          const int2 ht = HT[s];
          const int f = max(cc, ht.x);
          cc = f + PT[s * pstep];
          fb[s * fstep] = (unsigned short)f;
          lb = max(lb, f + ht.y);
        }
      }
      Q.lb1[64 * c + lane] = lb;
    }
  }
  // compacted selections: pair indices whose bit is set, in index order
  int nsel[G];
  int nmax_sel = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    nsel[g] = 0;
    if (!ok_[g] || r_[g] < 2) continue;  // leaves: LB2 = LB1, no pair needed
    for (int base = 0; base < P; base += 64) {
      const int pi = base + lane;
      const uint32_t w = (uint32_t)__shfl((int)F[g].mw, (pi >> 5) & 63, kWave);
      const bool on = pi < P && ((w >> (pi & 31)) & 1u);
      const uint64_t bal = __ballot(on);
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (on) S.parent(g).sel[nsel[g] + pos] = (int16_t)pi;
      nsel[g] += __popcll(bal);
    }
    nmax_sel = max(nmax_sel, nsel[g]);
  }
  wave_sync();
  // this lane's parent
  uint64_t umask = 0;
  int nsg = 0, ag = 0, rg = 0, par = -1;
  bool okg = false;
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (gl == g) {
      umask = um[g];
      nsg = nsel[g];
      ag = a_[g];
      rg = r_[g];
      par = rows[g];
      okg = ok_[g];
    }
  const WsParent Q = S.parent(gl);
  int acc[64];  // pair maxima per job: forward | backward << 16 (int16 halves)
#pragma unroll
  for (int q = 0; q < 64; ++q) {  // set once (not repeated on the path into the loop)
    acc[q] = (int)0x80008000u;
    asm volatile("" : "+v"(acc[q]));
  }
  int *__restrict__ Xh = S.X + lane;
  for (int pc = 0; pc < nmax_sel; pc += L) {
    const int idx = pc + l;
    const int pi = nsg > 0 ? Q.sel[idx < nsg ? idx : 0] : 0;
    const int uvp = S.uv[pi];
    const int u = uvp & 0xff, v = uvp >> 8;
    const int K4 = Q.rr[v] + Q.c2[v], K5 = Q.c1[u] + Q.rr[v];
    const int K5x = K5 - K4;  // the high half is Xb + K5 (K4 is already inside)
    const uint2 *__restrict__ eb = I.entq + (size_t)(pi >> 6) * n * 64 + (pi & 63);
    // first sweep: the running sum and prefix maximum at position CH
    int Y = K4, Pm = NEGX;
    {
      uint2 ev[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) ev[i] = eb[i * 64];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const uint2 e = ev[i];
        const int ng = __builtin_amdgcn_sbfe((int)(uint32_t)(umask >> (e.y & 63u)), 0, 1);
        const int tt = Y + (int)(e.y >> 16);
        Pm = max(Pm, (tt & ng) | (NEGX & ~ng));
        Y = mad_i16(ng, (int)e.x, Y);
      }
    }
    // second sweep: positions CH .. n - 1, then 0 .. CH - 1
    int Sm = NEGX;
    lb2ws_chunk<CH>(eb + CH * 64, n - CH, umask, K5x, Y, Pm, Sm, Xh);
    lb2ws_chunk<CH>(eb, CH, umask, K5x, K4, NEGX, Sm, Xh);
    // children of the member jobs, four at a time: f_u + xa | g_v + xb
    const int *Fu = lds_opaque((const int *)Q.fb + u * ROW);
    const int *Gv = lds_opaque((const int *)Q.fb + v * ROW);
#pragma unroll
    for (int g0 = 0; g0 < 64; g0 += 4) {
      if ((uany >> g0) & 0xfull) {
        int h[4], fw[4], gw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // a group holding a member ends before row n + 3
          h[j] = Xh[(g0 + j) * 64];
          fw[j] = Fu[g0 + j];
          gw[j] = Gv[g0 + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)  // sums first: no wait state before each maximum
          h[j] = pk_add((int)__builtin_amdgcn_perm((unsigned)gw[j], (unsigned)fw[j], 0x07060100u),
                        h[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[g0 + j] = pk_max(acc[g0 + j], h[j]);
      }
    }
  }
  // fold over each group's lanes: lane l of block b ends with job b * L + l
  int t[NB];
  group_blocks<0, L, 64, NB>(acc, t, tsrc, lane);
  // outputs and MinMin per group
  int *lbrow = out_lb + (size_t)(par >= 0 ? par : 0) * 2 * ns;
  uint8_t *prow = out_prune + (size_t)(par >= 0 ? par : 0) * 2 * ns;
  int vmin = kInt32Max;
  int valf[NB], valb[NB];
  bool mem[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int q = b * L + l;
    const bool member = okg && q < n && ((umask >> q) & 1ull);
    const int sl = member ? Q.inv[q] - ag : 0;
    const int pf = nsg > 0 ? (int)(short)(t[b] & 0xffff) : kNeg;
    const int pb = nsg > 0 ? t[b] >> 16 : kNeg;
    const int vf = member ? max(Q.lb1[64 * (q >> 5) + (q & 31)], pf) : kInt32Max;
    const int vb = member ? max(Q.lb1[64 * (q >> 5) + 32 + (q & 31)], pb) : kInt32Max;
    if (member) {
      lbrow[sl] = vf;
      prow[sl] = vf >= ub;
      lbrow[ns + sl] = vb;
      prow[ns + sl] = vb >= ub;
    }
    valf[b] = vf;
    valb[b] = vb;
    mem[b] = member;
    vmin = min(vmin, min(vf, vb));
  }
  const int cmn = group_min<L>(vmin);
  int cf = 0, cb = 0, flo = 0, fhi = 0, blo = 0, bhi = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (mem[b]) {
      cf += valf[b] == cmn;
      flo += valf[b] & 0xffff;
      fhi += valf[b] >> 16;
      cb += valb[b] == cmn;
      blo += valb[b] & 0xffff;
      bhi += valb[b] >> 16;
    }
  }
  cf = group_sum<L>(cf);
  cb = group_sum<L>(cb);
  flo = group_sum<L>(flo);
  fhi = group_sum<L>(fhi);
  blo = group_sum<L>(blo);
  bhi = group_sum<L>(bhi);
  if (par >= 0) {
    for (int x = l; x < 2 * ns; x += L) {  // slots >= r of both directions (all if invalid)
      const int q = x < ns ? x : x - ns;
      if (!okg || q >= rg) {
        lbrow[x] = kInt32Max;
        prow[x] = 1;
      }
    }
    if (l == 0 && pool.dir) {
      MinMin mm;
      mm.init();
      mm.merge(cmn, cf, cb, ((long long)fhi << 16) + flo, ((long long)bhi << 16) + blo);
      pool.dir[par] = okg ? (uint8_t)mm.dir() : (uint8_t)0;
    }
  }
  wave_sync();  // the next parents rewrite this wave's tables
}

// Blocks of up to four waves (one per SIMD): the registers of the two-sweep
// scan over 32 positions, and the LDS of G parents' tables per wave.
template <int G>
__global__ void __launch_bounds__(256)
k_lb2ws(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
        uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw * G >= count) return;  // no parent for this block
  const WsLayout L{Ppad, I.n, I.m};
  const WsLds S(sm, L, w, G);
  const int n = I.n, m = I.m, P = I.P;
  for (int x = threadIdx.x; x < Ppad; x += blockDim.x) {
    const int q = x < P ? x : 0;
    S.uv[x] = P > 0 ? ((int)I.pu[q] | ((int)I.pv[q] << 8)) : 0;
  }
  for (int x = threadIdx.x; x < m * 64; x += blockDim.x) {
    const int s = x >> 6, k = x & 63;
    S.pt[x] = (unsigned short)(k < n ? I.p[k * m + s] : 0);
  }
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int step = gridDim.x * nw * G;
  int it0 = (blockIdx.x * nw + w) * G;
  auto row_of = [&](int it) { return it < count ? (pool.index ? pool.index[it] : it) : -1; };
  const GroupSrc<64, 64 / G> tsrc(lane);
  int rows[G];
  PackFetch F[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    rows[g] = row_of(it0 + g);
    F[g] = pack_fetch(pool, rows[g], n, m, costs, lane);
  }
  for (; it0 < count; it0 += step) {
    PackFetch C[G];
    int cur[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      C[g] = F[g];
      cur[g] = rows[g];
      rows[g] = row_of(it0 + step + g);
      F[g] = pack_fetch(pool, rows[g], n, m, costs, lane);
    }
    lb2ws_wave<G>(I, S, pool, cur, C, ub, out_lb, out_prune, lane, tsrc);
  }
}

// Single instance: the block stages the tables once, then each wave takes
// parents in a grid-stride loop.
template <int NMAX, bool SUBSET, bool LOG>
__global__ void __launch_bounds__(512)
k_lb2f(DevInst I, DevPool pool, int ub, const int *__restrict__ costs, int *__restrict__ out_lb,
       uint8_t *__restrict__ out_prune, int Ppad) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  if ((int)blockIdx.x * nw >= count) return;  // no parent for this block
  const FastLayout L{Ppad, I.n, I.m};
  const FastLds<NMAX> S(sm, L, w);
  lb2f_stage<NMAX>(I, Ppad, S);
  __syncthreads();
  if (pool.ub_dev) ub = *pool.ub_dev;
  const int m = I.m;
  for (int it = blockIdx.x * nw + w; it < count; it += gridDim.x * nw) {
    const int par = pool.index ? pool.index[it] : it;
    const int ns = pool.n;  // row stride (>= n)
    lb2f_parent<NMAX, SUBSET, LOG>(
        I, Ppad, S, pool.perm + (size_t)par * ns, pool.d1[par], pool.d2[par],
        costs + (size_t)par * 3 * m,
        SUBSET ? mask_row(pool, par) : nullptr, ns, ub,
        out_lb + (size_t)par * 2 * ns, out_prune + (size_t)par * 2 * ns,
        LOG ? pool.argpair + (size_t)par * 2 * ns : nullptr, pool.dir ? pool.dir + par : nullptr,
        lane);
  }
}

template <int NMAX, bool X16>
__device__ __forceinline__ auto make_lds(unsigned char *sm, const FastLayout &L, int w) {
  if constexpr (NMAX <= 32)
    return QuickLds<NMAX>(sm, QuickLayout{L.ppad, L.mmax, X16, 0}, w);
  else
    return FastLds<NMAX>(sm, L, w);
}

// Several instances in one persistent launch.  Work is a list of tiles (an
// instance and a range of its parents, tiles grouped by instance); each block
// takes tiles from a device counter, restages the LDS tables when the
// instance changes, and its waves decompose the tile's parents.  Pool rows
// and outputs use a common stride (the largest n); costs rows hold cstride
// ints.
template <int NMAX, bool X16>
__global__ void __launch_bounds__(X16 && NMAX <= 20 ? 1024 : NMAX <= 32 ? 768 : 512)
k_lb2m(const DevInst *__restrict__ insts, const MultiTile *__restrict__ tiles, int ntiles,
       int *__restrict__ queue, FastLayout L, const uint8_t *__restrict__ perm,
       const uint8_t *__restrict__ d1, const uint8_t *__restrict__ d2, int stride,
       const int *__restrict__ ubs, const int *__restrict__ costs, int cstride,
       int *__restrict__ out_lb, uint8_t *__restrict__ out_prune, uint8_t *__restrict__ dir) {
  extern __shared__ __align__(16) unsigned char sm[];
  __shared__ int s_tile;
  constexpr bool QUICK = NMAX <= 32;
  using Lds = typename std::conditional<QUICK, QuickLds<NMAX>, FastLds<NMAX>>::type;
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  const Lds S = make_lds<NMAX, X16>(sm, L, w);
  const int tsrc = tp_source<QUICK ? NMAX : 32>(lane);
  int cur = -1, Ppad = 0;
  DevInst I{};
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_tile;
    __syncthreads();  // every thread has read s_tile before it is overwritten
    if (t >= ntiles) break;
    const MultiTile T = tiles[t];
    if (T.inst != cur) {
      cur = T.inst;
      I = insts[cur];
      Ppad = (I.P + 63) / 64 * 64;
      if constexpr (QUICK)
        lb2q_stage<NMAX, X16>(I, Ppad, S);
      else
        lb2f_stage<NMAX>(I, Ppad, S);
      __syncthreads();
    }
    const int ub = ubs[cur];
    for (int par = T.begin + w; par < T.end; par += nw) {
      if constexpr (QUICK)
        lb2q_parent<NMAX, false, X16>(
            I, Ppad, S,
            row_fetch(perm + (size_t)par * stride, costs + (size_t)par * cstride, d1[par],
                      d2[par], I.n, I.m, lane),
            stride, ub, out_lb + (size_t)par * 2 * stride, out_prune + (size_t)par * 2 * stride,
            dir + par, lane, tsrc);
      else
        lb2f_parent<NMAX, false, false>(
            I, Ppad, S, perm + (size_t)par * stride, d1[par], d2[par],
            costs + (size_t)par * cstride, nullptr, stride, ub,
            out_lb + (size_t)par * 2 * stride, out_prune + (size_t)par * 2 * stride, nullptr,
            dir + par, lane);
    }
    __syncthreads();  // the tables may be restaged for the next tile
  }
}

// The wide kernel in the persistent multi-instance form of k_lb2m: L is the
// class layout (largest padded pair count, n and m of its instances).
template <int NMAX>
__global__ void __launch_bounds__(NMAX >= 128 ? 256 : 512)
k_lb2mw(const DevInst *__restrict__ insts, const MultiTile *__restrict__ tiles, int ntiles,
        int *__restrict__ queue, WideLayout L, const uint8_t *__restrict__ perm,
        const uint8_t *__restrict__ d1, const uint8_t *__restrict__ d2, int stride,
        const int *__restrict__ ubs, const int *__restrict__ costs, int cstride,
        int *__restrict__ out_lb, uint8_t *__restrict__ out_prune, uint8_t *__restrict__ dir) {
  extern __shared__ __align__(16) unsigned char sm[];
  __shared__ int s_tile;
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform
  const WideLds<NMAX> S(sm, L, w);
  int cur = -1, Ppad = 0;
  DevInst I{};
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_tile;
    __syncthreads();  // every thread has read s_tile before it is overwritten
    if (t >= ntiles) break;
    const MultiTile T = tiles[t];
    if (T.inst != cur) {
      cur = T.inst;
      I = insts[cur];
      Ppad = (I.P + 63) / 64 * 64;
      lb2w_stage<NMAX>(I, Ppad, S);
      __syncthreads();
    }
    const int ub = ubs[cur];
    for (int par = T.begin + w; par < T.end; par += nw)
      lb2w_parent<NMAX>(I, Ppad, S, perm + (size_t)par * stride, d1[par], d2[par],
                        costs + (size_t)par * cstride, stride, ub,
                        out_lb + (size_t)par * 2 * stride, out_prune + (size_t)par * 2 * stride,
                        dir + par, lane);
    __syncthreads();  // the tables may be restaged for the next tile
  }
}

// Waves per block that the single-instance kernels' launch bounds allow:
// with 16-bit X, up to 20 jobs fit 128 registers, four waves per SIMD.
static int quick_wmax(int nmax, int x16, bool log) {
  if (log) return 8;
  if (x16 && nmax <= 20) return 16;
  return nmax <= 24 ? 12 : 8;
}

// LDS of the single-instance fast kernels: the quick layout for n <= 32
// without argmax logging, the scan layout otherwise.
static size_t lb2f_lds(const Ctx *c, int nmax, int waves, bool log, bool subset) {
  const int ppad = (c->P + 63) / 64 * 64;
  if (nmax <= 32 && !log) {
    const QuickLayout L{ppad, c->m, c->x16, subset ? 1 : 0};
    return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
  }
  const FastLayout L{ppad, c->n, c->m};
  return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
}

template <int NMAX>
static void launch_lb2f_n(bool subset, bool log, dim3 g, dim3 b, size_t lds, hipStream_t s,
                          const DevInst &I, const DevPool &pool, int ub, const int *costs,
                          int *out_lb, uint8_t *out_prune, int Ppad) {
  if constexpr (NMAX <= 32) {
    if (!log) {
#define PFSP_Q(SUB, X)                                                                      \
  hipLaunchKernelGGL((k_lb2q<NMAX, SUB, X>), g, b, lds, s, I, pool, ub, costs, out_lb, out_prune, \
                     Ppad)
      if (subset) {
        if (I.x16) PFSP_Q(true, true); else PFSP_Q(true, false);
      } else {
        if (I.x16) PFSP_Q(false, true); else PFSP_Q(false, false);
      }
#undef PFSP_Q
      return;
    }
  }
  if (subset) {
    if (log)
      hipLaunchKernelGGL((k_lb2f<NMAX, true, true>), g, b, lds, s, I, pool, ub, costs, out_lb,
                         out_prune, Ppad);
    else
      hipLaunchKernelGGL((k_lb2f<NMAX, true, false>), g, b, lds, s, I, pool, ub, costs, out_lb,
                         out_prune, Ppad);
  } else {
    if (log)
      hipLaunchKernelGGL((k_lb2f<NMAX, false, true>), g, b, lds, s, I, pool, ub, costs, out_lb,
                         out_prune, Ppad);
    else
      hipLaunchKernelGGL((k_lb2f<NMAX, false, false>), g, b, lds, s, I, pool, ub, costs,
                         out_lb, out_prune, Ppad);
  }
}

// Smallest compiled NMAX >= n (0 if none); the variants up to 32 jobs need
// (m - 1) * max p below 2^16.
static int fast_nmax(int n, int l16) {
  static const int sizes[] = {8, 12, 16, 20, 24, 32, 64};
  for (int s : sizes)
    if (n <= s && (l16 || s == 64)) return s;
  return 0;
}

__global__ void k_zero(int *p) { *p = 0; }

// -------------------------------------------------------------------- host
size_t workspace_ints(const Ctx *c, int count) {
  return (size_t)(count > 0 ? count : 1) * 3 * c->m;
}

int ensure_costs(Ctx *c, int count) {
  const size_t need = workspace_ints(c, count);
  if (need > c->costs_cap) {
    if (c->d_costs) {
      PFSP_HIP(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->d_costs);
      c->d_costs = nullptr;
      c->costs_cap = 0;
    }
    size_t cap = need + need / 4;
    if (hipMalloc(&c->d_costs, cap * 4) != hipSuccess) {
      c->d_costs = nullptr;
      return set_err(c, PFSP_ENOMEM, "workspace allocation failed");
    }
    c->costs_cap = cap;
  }
  return PFSP_OK;
}

static size_t lb2_lds_inst(int n, int m, int P, int narrow, int waves, bool ent_lds,
                           int xrows) {
  const size_t esz = narrow ? 8 : 16;
  size_t s = ent_lds ? align16((size_t)n * P * esz) : 0;
  s += align16((size_t)n * m * 4);
  const size_t pw = align16((size_t)xrows * 64 * 8) + align16((size_t)xrows * m * 8) +
                    align16((size_t)3 * m * 4) + align16((size_t)2 * n * 4);
  return s + waves * pw;
}

static size_t lb2_lds(const Ctx *c, int waves, bool ent_lds, int xrows) {
  return lb2_lds_inst(c->n, c->m, c->P, c->narrow, waves, ent_lds, xrows);
}

size_t lb2_lds_bytes(const Ctx *c, int waves) {
  const int xrows = c->n < 32 ? c->n : 32;
  return lb2_lds(c, waves, true, xrows);
}

template <class E, bool ENT_LDS>
static void launch_lb2_e(bool subset, bool log, dim3 g, dim3 b, size_t lds, hipStream_t s,
                         const DevInst &I, const DevPool &pool, int ub, const int *costs,
                         int *out_lb, uint8_t *out_prune, int xrows) {
  if (subset) {
    if (log)
      hipLaunchKernelGGL((k_lb2<E, ENT_LDS, true, true>), g, b, lds, s, I, pool, ub, costs,
                         out_lb, out_prune, xrows);
    else
      hipLaunchKernelGGL((k_lb2<E, ENT_LDS, true, false>), g, b, lds, s, I, pool, ub, costs,
                         out_lb, out_prune, xrows);
  } else {
    if (log)
      hipLaunchKernelGGL((k_lb2<E, ENT_LDS, false, true>), g, b, lds, s, I, pool, ub, costs,
                         out_lb, out_prune, xrows);
    else
      hipLaunchKernelGGL((k_lb2<E, ENT_LDS, false, false>), g, b, lds, s, I, pool, ub, costs,
                         out_lb, out_prune, xrows);
  }
}

// Allows every bound kernel to use up to 160 KiB of dynamic LDS (the gfx950
// per-CU size); called once per process, before any launch or graph capture.
// Lets a kernel use the whole 160 KiB of gfx950 LDS minus its static LDS.
static void lds_limit(const void *f) {
  hipFuncAttributes at;
  size_t stat = 0;
  if (hipFuncGetAttributes(&at, f) == hipSuccess) stat = at.sharedSizeBytes;
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(160 * 1024 - stat));
}

template <class E, bool ENT_LDS>
static void attr_lb2() {
  lds_limit((const void *)k_lb2<E, ENT_LDS, true, true>);
  lds_limit((const void *)k_lb2<E, ENT_LDS, true, false>);
  lds_limit((const void *)k_lb2<E, ENT_LDS, false, true>);
  lds_limit((const void *)k_lb2<E, ENT_LDS, false, false>);
}

template <int NMAX, int G>
static void attr_lb2s() {
  lds_limit((const void *)k_lb2s<NMAX, G>);
}

template <int NMAX>
static void attr_lb2d() {
  lds_limit((const void *)k_lb2d<NMAX, 4>);
  lds_limit((const void *)k_lb2d<NMAX, 8>);
  lds_limit((const void *)k_lb2d<NMAX, 16>);
}

template <int NMAX>
static void attr_lb2f() {
  if constexpr (NMAX <= 32) {
    lds_limit((const void *)k_lb2q<NMAX, true, true>);
    lds_limit((const void *)k_lb2q<NMAX, false, true>);
    lds_limit((const void *)k_lb2q<NMAX, true, false>);
    lds_limit((const void *)k_lb2q<NMAX, false, false>);
  }
  lds_limit((const void *)k_lb2f<NMAX, true, true>);
  lds_limit((const void *)k_lb2f<NMAX, true, false>);
  lds_limit((const void *)k_lb2f<NMAX, false, true>);
  lds_limit((const void *)k_lb2f<NMAX, false, false>);
}

size_t lb2m_lds_bytes(int nmax, int ppad, int nmax_jobs, int mmax, int waves, int x16,
                      int wide) {
  if (wide) {
    const WideLayout L{ppad, nmax_jobs, mmax};
    return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
  }
  if (nmax <= 32) {
    const QuickLayout L{ppad, mmax, x16, 0};
    return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
  }
  const FastLayout L{ppad, nmax_jobs, mmax};
  return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
}

int launch_lb1m(Ctx *c, const DevInst *insts, const long long *seg, int ninst, long long total,
                const uint8_t *perm, const uint8_t *d1, const uint8_t *d2, int stride, int nmax,
                int mmax, const int *ubs, int *out_lb, uint8_t *out_prune, uint8_t *dir,
                int *costs, int write_out, hipStream_t s) {
  if (total <= 0) return PFSP_OK;
  const int B = 128;
  if (!write_out && nmax <= 128 && mmax <= 32) {
    const int mm = mmax <= 8 ? 8 : mmax <= 16 ? 16 : mmax <= 20 ? 20 : 32;
    const size_t lds = (size_t)128 * (mm | 1) * 4 + (size_t)B * stride;
    KTimer kt(c, s, "k_lb1m");
    switch (mm) {
#define PFSP_C(M)                                                                            \
  case M:                                                                                    \
    hipLaunchKernelGGL(k_costsm<M>, dim3((unsigned)((total + B - 1) / B)), dim3(B), lds, s,   \
                       insts, seg, ninst, perm, d1, d2, stride, mmax, costs, c->d_flag);     \
    break;
      PFSP_C(8) PFSP_C(16) PFSP_C(20) PFSP_C(32)
#undef PFSP_C
      default: break;
    }
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  }
  const size_t lds = (size_t)3 * mmax * B * 4;
  KTimer kt(c, s, "k_lb1m");
  hipLaunchKernelGGL(k_lb1m, dim3((unsigned)((total + B - 1) / B)), dim3(B), lds, s, insts, seg,
                     ninst, perm, d1, d2, stride, mmax, ubs, out_lb, out_prune, dir, costs,
                     write_out, c->d_flag);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int launch_lb2m(Ctx *c, const FastClassLaunch &L, const DevInst *insts, const uint8_t *perm,
                const uint8_t *d1, const uint8_t *d2, int stride, const int *ubs,
                const int *costs, int *out_lb, uint8_t *out_prune, uint8_t *dir, hipStream_t s) {
  if (L.ntiles <= 0) return PFSP_OK;
  const FastLayout FL{L.ppad, L.nmax_jobs, L.mmax};
  const size_t lds =
      lb2m_lds_bytes(L.nmax, L.ppad, L.nmax_jobs, L.mmax, L.waves, L.x16, L.wide);
  if (lds > 160 * 1024 - 64) return set_err(c, PFSP_ERANGE, "multi-instance class exceeds LDS");
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, L.queue);
  KTimer kt(c, s, "k_lb2m");
  if (L.wide) {
    const WideLayout WL{L.ppad, L.nmax_jobs, L.mmax};
#define PFSP_W(N)                                                                            \
  hipLaunchKernelGGL((k_lb2mw<N>), dim3(L.grid), dim3(64 * L.waves), lds, s, insts, L.tiles,    \
                     L.ntiles, L.queue, WL, perm, d1, d2, stride, ubs, costs, L.cstride, out_lb, \
                     out_prune, dir)
    if (L.nmax == 64)
      PFSP_W(64);
    else if (L.nmax == 128)
      PFSP_W(128);
    else
      return set_err(c, PFSP_EINVAL, "no wide multi-instance kernel for this class");
#undef PFSP_W
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  }
#define PFSP_M(N, X)                                                                        \
  hipLaunchKernelGGL((k_lb2m<N, X>), dim3(L.grid), dim3(64 * L.waves), lds, s, insts, L.tiles,  \
                     L.ntiles, L.queue, FL, perm, d1, d2, stride, ubs, costs, L.cstride, out_lb, \
                     out_prune, dir)
  if (L.nmax == 20 && L.x16)
    PFSP_M(20, true);
  else if (L.nmax == 20)
    PFSP_M(20, false);
  else if (L.nmax == 64)
    PFSP_M(64, false);
#undef PFSP_M
  else
    return set_err(c, PFSP_EINVAL, "no multi-instance kernel for this class");
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

void init_bound_attributes() {
  lds_limit((const void *)k_lb2w<64, false>);
  lds_limit((const void *)k_lb2w<128, false>);
  lds_limit((const void *)k_lb2w<64, true>);
  lds_limit((const void *)k_lb2w<128, true>);
  lds_limit((const void *)k_lb2mw<64>);
  lds_limit((const void *)k_lb2mw<128>);
  lds_limit((const void *)k_lb1m);
  lds_limit((const void *)k_lb2m<20, true>);
  lds_limit((const void *)k_lb2m<20, false>);
  lds_limit((const void *)k_lb2m<64, false>);
  lds_limit((const void *)k_lb1);
  attr_lb2<Narrow, true>();
  attr_lb2<Narrow, false>();
  attr_lb2<Wide, true>();
  attr_lb2<Wide, false>();
  attr_lb2s<16, 2>();
  attr_lb2s<20, 2>();
  attr_lb2s<32, 2>();
  attr_lb2s<16, 4>();
  attr_lb2s<20, 4>();
  attr_lb2f<8>();
  attr_lb2f<12>();
  attr_lb2f<16>();
  attr_lb2f<20>();
  attr_lb2f<24>();
  attr_lb2f<32>();
  attr_lb2f<64>();
  attr_lb2d<8>();
  attr_lb2d<12>();
  attr_lb2d<16>();
  attr_lb2d<20>();
  attr_lb2d<24>();
  attr_lb2d<32>();
  (void)hipGetLastError();  // a refused attribute must not surface as a later launch error
}

static void lb1_shape(const Ctx *c, int count, int &b1, size_t &lds1, int &g1) {
  const int n = c->n, m = c->m;
  b1 = 128;
  lds1 = ((size_t)n * m + 3 * (size_t)m * b1) * 4;
  if (lds1 > 64 * 1024) {
    b1 = 64;
    lds1 = ((size_t)n * m + 3 * (size_t)m * b1) * 4;
  }
  g1 = (count + b1 - 1) / b1;
}

// Parent front/back/remaining into the workspace (k_lb1 without outputs);
// with f, also the search-step filter (CostFilter).
int launch_costs(Ctx *c, const DevPool &pool, hipStream_t s, const CostFilter *f) {
  const CostFilter fv = f ? *f : CostFilter{};
  if (pool.count <= 0) return PFSP_OK;
  int rc = ensure_costs(c, pool.count);
  if (rc) return rc;
  if (c->n <= 32 && c->m <= 32) {
    const int mm = c->m <= 8 ? 8 : c->m <= 12 ? 12 : c->m <= 16 ? 16 : c->m <= 20 ? 20 : c->m <= 24 ? 24 : 32;
    const size_t lds = ((size_t)c->n * (mm | 1) + mm + 4 * 64 * (3 * (size_t)c->m + 1)) * 4;
    int grid = (pool.count + 255) / 256;
    if (grid > c->cu_count * 8) grid = c->cu_count * 8;
    if (grid < 1) grid = 1;
    KTimer kt(c, s, "k_costs");
    switch (mm) {
#define PFSP_C(M)                                                                          \
  case M:                                                                                  \
    hipLaunchKernelGGL(k_costs<M>, dim3(grid), dim3(256), lds, s, c->inst(), pool, c->d_costs, \
                       c->d_flag, fv);                                                     \
    break;
      PFSP_C(8) PFSP_C(12) PFSP_C(16) PFSP_C(20) PFSP_C(24) PFSP_C(32)
#undef PFSP_C
      default: break;
    }
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  }
  if (c->n <= 64 && c->m <= 32) {  // the same with 64-job rows
    const int mm = c->m <= 8 ? 8 : c->m <= 16 ? 16 : c->m <= 20 ? 20 : 32;
    const size_t lds = ((size_t)c->n * (mm | 1) + mm + 4 * 64 * (3 * (size_t)c->m + 1)) * 4;
    int grid = (pool.count + 255) / 256;
    if (grid > c->cu_count * 8) grid = c->cu_count * 8;
    if (grid < 1) grid = 1;
    KTimer kt(c, s, "k_costs");
    switch (mm) {
#define PFSP_C(M)                                                                          \
  case M:                                                                                  \
    hipLaunchKernelGGL((k_costs<M, 64>), dim3(grid), dim3(256), lds, s, c->inst(), pool,    \
                       c->d_costs, c->d_flag, fv);                                          \
    break;
      PFSP_C(8) PFSP_C(16) PFSP_C(20) PFSP_C(32)
#undef PFSP_C
      default: break;
    }
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  }
  int b1, g1;
  size_t lds1;
  lb1_shape(c, pool.count, b1, lds1, g1);
  KTimer kt(c, s, "k_lb1");
  hipLaunchKernelGGL(k_lb1, dim3(g1), dim3(b1), lds1, s, c->inst(), pool, 0, (int *)nullptr,
                     (uint8_t *)nullptr, c->d_costs, 0, c->d_flag, fv);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int subset_group_for(const Ctx *c, int k) {
  if (c->subset_group > 0) return (int)c->subset_group;
  // n <= 32: two parents per wave up to 32 pairs (four cost about as much per
  // parent, and the two-parent kernel runs three waves per SIMD); 32 < n <=
  // 64: four parents per wave up to 16 pairs, two up to 32
  if (c->n > 32 && c->n <= 64 && k <= 16) return 4;
  return k <= 32 ? 2 : 1;
}

int deep_bin_r(const Ctx *c, int kind, bool log) {
  if (kind != PFSP_LB2_FULL || log || c->deep_r < 2 || c->force_generic) return 0;
  // the quick kernels' tables with 16-bit X; the costs kernel bins the rows
  if (!c->narrow || !c->x16 || c->n > 32 || c->m > 32 || c->P < 1) return 0;
  const int nmax = fast_nmax(c->n, c->l16);
  return nmax && nmax <= 32 ? (int)c->deep_r : 0;
}

// LB1 of every child through the costs kernel and the quick LB2 kernel with
// no pair pass (LB2 over no pair is LB1): one wave per parent, a lane per
// child walking the m machines, instead of one thread walking every child's
// machines in turn.  For pools of up to kLb1QuickMax parents of n <= 32,
// m <= 32, where the per-thread walks of k_lb1 set the launch's latency; on
// larger pools one thread per parent does less work per parent and wins.
constexpr int kLb1QuickMax = 16384;

static bool lb1_quick_ok(const Ctx *c, const DevPool &pool) {
  if (pool.argpair || pool.count > kLb1QuickMax || !c->narrow || c->force_generic) return false;
  if (c->n > 32 || c->m > 32) return false;
  const int nmax = fast_nmax(c->n, c->l16);
  return nmax && nmax <= 32;
}

static int launch_lb1_quick(Ctx *c, const DevPool &pool, int ub, int *out_lb,
                            uint8_t *out_prune, hipStream_t s) {
  int rc = launch_costs(c, pool, s);
  if (rc) return rc;
  const DevInst I = c->inst();
  const int nmax = fast_nmax(c->n, c->l16);
  const QuickLayout L{0, c->m, c->x16, 0};  // no pair tables
  int waves = 0, best = 0;
  for (int w = quick_wmax(nmax, c->x16, false); w >= 1; --w) {
    const size_t l = L.block_bytes(nmax) + (size_t)w * L.wave_bytes(nmax) + kBinListLds;
    const int per_cu = l <= 160 * 1024 ? (int)((160 * 1024) / l) * w : 0;
    if (per_cu > best) {
      best = per_cu;
      waves = w;
    }
  }
  if (!waves) return set_err(c, PFSP_ERANGE, "LB1 tables exceed LDS");
  const size_t lds = L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
  int grid = (pool.count + waves - 1) / waves;
  const int cap = c->cu_count * 16;
  if (grid > cap) grid = cap;
  KTimer kt(c, s, "k_lb1");
  switch (nmax) {
#define PFSP_CASE(N)                                                                            \
  case N:                                                                                       \
    launch_lb2f_n<N>(false, false, dim3(grid), dim3(64 * waves), lds, s, I, pool, ub, c->d_costs, \
                     out_lb, out_prune, 0);                                                      \
    break;
    PFSP_CASE(8) PFSP_CASE(12) PFSP_CASE(16) PFSP_CASE(20) PFSP_CASE(24) PFSP_CASE(32)
#undef PFSP_CASE
    default: break;
  }
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int launch_bound(Ctx *c, const DevPool &pool, int kind, int ub, int *out_lb, uint8_t *out_prune,
                 hipStream_t s) {
  if (pool.count <= 0) return PFSP_OK;
  if (kind == PFSP_LB1 && lb1_quick_ok(c, pool))
    return launch_lb1_quick(c, pool, ub, out_lb, out_prune, s);
  if (kind == PFSP_LB1) {
    int b1, g1;
    size_t lds1;
    lb1_shape(c, pool.count, b1, lds1, g1);
    KTimer kt(c, s, "k_lb1");
    hipLaunchKernelGGL(k_lb1, dim3(g1), dim3(b1), lds1, s, c->inst(), pool, ub, out_lb,
                       out_prune, (int *)nullptr, 1, c->d_flag, CostFilter{});
    PFSP_HIP(c, hipGetLastError());
    return PFSP_OK;
  }
  int rc = launch_costs(c, pool, s);
  if (rc) return rc;
  if (deep_bin_r(c, kind, pool.argpair != nullptr))
    return launch_lb2_binned(c, pool, ub, out_lb, out_prune, s);
  return launch_bound_costs_ready(c, pool, kind, ub, out_lb, out_prune, s, 0);
}

static size_t lb2s_lds(const Ctx *c, int nmax, int G, int waves) {
  const PackLayout L{(c->P + 63) / 64 * 64, c->m};
  return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax, G);
}

// Packed subset kernel: G parents per wave.
static int launch_lb2s(Ctx *c, const DevPool &pool, int G, int ub, int *out_lb,
                       uint8_t *out_prune, hipStream_t s) {
  const int nmax = c->n <= 16 ? 16 : c->n <= 20 ? 20 : 32;
  if (nmax == 32) G = 2;  // four parents' state of 32 jobs does not fit the registers
  int waves = 0, best = 0;
  const int wmax = G == 2 && nmax <= 20 ? 12 : 8;  // the kernels' launch bounds
  for (int w = wmax; w >= 1; --w) {
    const size_t l = lb2s_lds(c, nmax, G, w);
    const int per_cu = l <= 160 * 1024 ? (int)((160 * 1024) / l) * w : 0;
    if (per_cu > best) {
      best = per_cu;
      waves = w;
    }
  }
  if (!waves) return set_err(c, PFSP_ERANGE, "packed subset kernel exceeds LDS");
  const size_t lds = lb2s_lds(c, nmax, G, waves);
  const int Ppad = (c->P + 63) / 64 * 64;
  const int per_block = waves * G;
  int grid = (pool.count + per_block - 1) / per_block;
  // twice the blocks that LDS lets a CU hold (each block stages its tables once)
  const int resident = std::max(1, (int)((160 * 1024) / std::max<size_t>(lds, 1)));
  const int cap = c->cu_count * (c->lb2_blocks_per_cu > 0 ? (int)c->lb2_blocks_per_cu
                                                          : 2 * resident);
  if (grid > cap) grid = cap;
  KTimer kt(c, s, "k_lb2");
#define PFSP_S(N, GG)                                                                       \
  hipLaunchKernelGGL((k_lb2s<N, GG>), dim3(grid), dim3(64 * waves), lds, s, c->inst(), pool, ub, \
                     c->d_costs, out_lb, out_prune, Ppad)
  if (G == 4) {
    if (nmax == 16) PFSP_S(16, 4); else PFSP_S(20, 4);
  } else {
    if (nmax == 16) PFSP_S(16, 2); else if (nmax == 20) PFSP_S(20, 2); else PFSP_S(32, 2);
  }
#undef PFSP_S
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

// Wide-kernel LDS of one block: the most resident waves per CU within 160 KiB.
static int wide_waves(const WideLayout &L, int nmax, int pref) {
  int waves = 0, best = 0;
  const int wmax = nmax >= 128 ? 4 : 8;  // the kernels' launch bounds
  if (pref > wmax) pref = 0;
  for (int w = wmax; w >= 1; --w) {
    const size_t l = L.block_bytes(nmax) + (size_t)w * L.wave_bytes(nmax);
    const int per_cu = l <= 160 * 1024 ? (int)((160 * 1024) / l) * w : 0;
    if (per_cu > best) {
      best = per_cu;
      waves = w;
    }
  }
  if (pref > 0 && pref <= 8 && L.block_bytes(nmax) + (size_t)pref * L.wave_bytes(nmax) <= 160 * 1024)
    waves = pref;
  return waves;
}

static int launch_lb2w(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                       hipStream_t s, bool subset) {
  const int Ppad = (c->P + 63) / 64 * 64;
  const int nmax = c->n <= 64 ? 64 : 128;
  WideLayout L{Ppad, c->n, c->m};
  L.subset = subset;
  const int waves = wide_waves(L, nmax, (int)c->lb2_waves);
  if (!waves) return set_err(c, PFSP_ERANGE, "wide LB2 tables exceed LDS");
  const size_t lds = L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
  int grid = (pool.count + waves - 1) / waves;
  const int cap = c->cu_count * (int)(c->lb2_blocks_per_cu > 0 ? c->lb2_blocks_per_cu : 16);
  if (grid > cap) grid = cap;
  const DevInst I = c->inst();
  KTimer kt(c, s, "k_lb2w");
#define PFSP_W(N, SUB)                                                                     \
  hipLaunchKernelGGL((k_lb2w<N, SUB>), dim3(grid), dim3(64 * waves), lds, s, I, pool, ub,   \
                     c->d_costs, out_lb, out_prune, Ppad)
  if (nmax == 64) {
    if (subset) PFSP_W(64, true); else PFSP_W(64, false);
  } else {
    if (subset) PFSP_W(128, true); else PFSP_W(128, false);
  }
#undef PFSP_W
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

// Packed wide subset kernel: G parents per wave for 32 < n <= 64, blocks of
// up to four waves (the most that fit 160 KiB of LDS).
static int launch_lb2ws(Ctx *c, const DevPool &pool, int G, int ub, int *out_lb,
                        uint8_t *out_prune, hipStream_t s) {
  const int Ppad = (c->P + 63) / 64 * 64;
  const WsLayout L{Ppad, c->n, c->m};
  int waves = 0;
  for (int w = 4; w >= 1 && !waves; --w)
    if (L.block_bytes() + (size_t)w * L.wave_bytes(G) <= 160 * 1024) waves = w;
  if (c->lb2_waves > 0 && c->lb2_waves <= 4 &&
      L.block_bytes() + (size_t)c->lb2_waves * L.wave_bytes(G) <= 160 * 1024)
    waves = (int)c->lb2_waves;
  if (!waves) return set_err(c, PFSP_ERANGE, "packed wide subset tables exceed LDS");
  const size_t lds = L.block_bytes() + (size_t)waves * L.wave_bytes(G);
  const int per_block = waves * G;
  int grid = (pool.count + per_block - 1) / per_block;
  // twice the blocks that LDS lets a CU hold (each block stages its tables once)
  const int resident = std::max(1, (int)((160 * 1024) / lds));
  const int cap = c->cu_count * (c->lb2_blocks_per_cu > 0 ? (int)c->lb2_blocks_per_cu
                                                          : 2 * resident);
  if (grid > cap) grid = cap;
  const DevInst I = c->inst();
  KTimer kt(c, s, "k_lb2w");
  if (G == 4)
    hipLaunchKernelGGL(k_lb2ws<4>, dim3(grid), dim3(64 * waves), lds, s, I, pool, ub, c->d_costs,
                       out_lb, out_prune, Ppad);
  else
    hipLaunchKernelGGL(k_lb2ws<2>, dim3(grid), dim3(64 * waves), lds, s, I, pool, ub, c->d_costs,
                       out_lb, out_prune, Ppad);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

static size_t lb2d_lds(const Ctx *c, int nmax, int rmax, int waves) {
  const DeepLayout L{(c->P + 63) / 64 * 64, c->m, rmax};
  return L.block_bytes(nmax) + (size_t)waves * L.wave_bytes(nmax);
}

int launch_lb2d(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                hipStream_t s) {
  if (pool.count <= 0) return PFSP_OK;
  const int nmax = fast_nmax(c->n, c->l16);
  const int r = deep_bin_r(c, PFSP_LB2_FULL, false);
  if (!r || !nmax || nmax > 32) return set_err(c, PFSP_EINVAL, "deep LB2 kernel does not apply");
  const int rmax = r <= 4 ? 4 : r <= 8 ? 8 : 16;
  // the kernel's static row list counts against the 160 KiB with the tables
  int waves = 0, best = 0;
  for (int w = 16; w >= 1; --w) {
    const size_t l = lb2d_lds(c, nmax, rmax, w) + kBinListLds;
    const int per_cu = l <= 160 * 1024 ? (int)((160 * 1024) / l) * w : 0;
    if (per_cu > best) {
      best = per_cu;
      waves = w;
    }
  }
  if (c->lb2_waves > 0 &&
      lb2d_lds(c, nmax, rmax, (int)c->lb2_waves) + kBinListLds <= 160 * 1024)
    waves = (int)c->lb2_waves;
  if (!waves) return set_err(c, PFSP_ERANGE, "deep LB2 tables exceed LDS");
  const size_t lds = lb2d_lds(c, nmax, rmax, waves);
  const int Ppad = (c->P + 63) / 64 * 64;
  int grid = (pool.count + waves - 1) / waves;
  const int resident =
      std::max(1, (int)((160 * 1024) / std::max<size_t>(lds + kBinListLds, 1)));
  const int cap = c->cu_count * (int)(c->lb2_blocks_per_cu > 0 ? c->lb2_blocks_per_cu
                                                               : 2 * resident);
  if (grid > cap) grid = cap;
  const DevInst I = c->inst();
  KTimer kt(c, s, "k_lb2d");
#define PFSP_D(N, R)                                                                          \
  hipLaunchKernelGGL((k_lb2d<N, R>), dim3(grid), dim3(64 * waves), lds, s, I, pool, ub,        \
                     c->d_costs, out_lb, out_prune, Ppad)
#define PFSP_DN(N)                    \
  case N:                             \
    if (rmax == 4) PFSP_D(N, 4);      \
    else if (rmax == 8) PFSP_D(N, 8); \
    else PFSP_D(N, 16);               \
    break;
  switch (nmax) {
    PFSP_DN(8) PFSP_DN(12) PFSP_DN(16) PFSP_DN(20) PFSP_DN(24) PFSP_DN(32)
    default: break;
  }
#undef PFSP_DN
#undef PFSP_D
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int launch_lb2_binned(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                      hipStream_t s) {
  const int r = deep_bin_r(c, PFSP_LB2_FULL, pool.argpair != nullptr);
  if (!r) return launch_bound_costs_ready(c, pool, PFSP_LB2_FULL, ub, out_lb, out_prune, s, 0);
  DevPool dp = pool, dd = pool;
  dp.bin = 1;
  dd.bin = 2;
  dp.bin_r = dd.bin_r = r;
  const int rc = launch_bound_costs_ready(c, dp, PFSP_LB2_FULL, ub, out_lb, out_prune, s, 0);
  if (rc) return rc;
  return launch_lb2d(c, dd, ub, out_lb, out_prune, s);
}

// LB2 kinds once launch_costs has run for the same pool.  group: parents per
// wave for subset bounds (1, 2 or 4; 0 = the context's "subset_group").
int launch_bound_costs_ready(Ctx *c, const DevPool &pool, int kind, int ub, int *out_lb,
                             uint8_t *out_prune, hipStream_t s, int group) {
  if (pool.count <= 0) return PFSP_OK;
  const DevInst I = c->inst();
  const int n = c->n;
  const bool subset = kind == PFSP_LB2_SUBSET;
  const bool log = pool.argpair != nullptr;
  if (group <= 0) group = (int)c->subset_group;
  if (!log && c->d_entq && c->wide_lb2 && !c->force_generic && n > 32 && n <= 128) {
    if (subset && n <= 64 && (group == 2 || group == 4))
      return launch_lb2ws(c, pool, group, ub, out_lb, out_prune, s);
    return launch_lb2w(c, pool, ub, out_lb, out_prune, s, subset);
  }
  const int nmax = c->narrow && !c->force_generic ? fast_nmax(n, c->l16) : 0;
  if (subset && !log && nmax && nmax <= 32 && c->x16 && (group == 2 || group == 4))
    return launch_lb2s(c, pool, group, ub, out_lb, out_prune, s);
  if (nmax) {
    // waves per block: the most resident waves per CU within 160 KiB of LDS
    int waves = 0, best = 0;
    const int wmax = quick_wmax(nmax, c->x16, log);  // the kernels' launch bounds
    // the quick kernel's static row list counts against the 160 KiB too
    const size_t st = nmax <= 32 && !log ? kBinListLds : 0;
    for (int w = wmax; w >= 1; --w) {
      const size_t l = lb2f_lds(c, nmax, w, log, subset) + st;
      const int per_cu = l <= 160 * 1024 ? (int)((160 * 1024) / l) * w : 0;
      if (per_cu > best) {
        best = per_cu;
        waves = w;
      }
    }
    if (c->lb2_waves > 0 && c->lb2_waves <= wmax &&
        lb2f_lds(c, nmax, (int)c->lb2_waves, log, subset) + st <= 160 * 1024)
      waves = (int)c->lb2_waves;
    const size_t lds = waves ? lb2f_lds(c, nmax, waves, log, subset) : 0;
    if (waves) {
      const int Ppad = (c->P + 63) / 64 * 64;
      int grid = (pool.count + waves - 1) / waves;
      // default: twice the blocks that LDS lets a CU hold, so that each block
      // stages its tables once and then loops over many parents
      const int resident = std::max(1, (int)((160 * 1024) / std::max<size_t>(lds + st, 1)));
      const int cap = c->cu_count * (int)(c->lb2_blocks_per_cu > 0 ? c->lb2_blocks_per_cu
                                                                   : 2 * resident);
      if (grid > cap) grid = cap;
      const dim3 g(grid), bl(64 * waves);
      KTimer kt(c, s, "k_lb2");
      switch (nmax) {
#define PFSP_CASE(N)                                                                         \
  case N:                                                                                    \
    launch_lb2f_n<N>(subset, log, g, bl, lds, s, I, pool, ub, c->d_costs, out_lb, out_prune, \
                     Ppad);                                                                  \
    break;
        PFSP_CASE(8) PFSP_CASE(12) PFSP_CASE(16) PFSP_CASE(20) PFSP_CASE(24) PFSP_CASE(32)
        PFSP_CASE(64)
#undef PFSP_CASE
        default: break;
      }
      PFSP_HIP(c, hipGetLastError());
      return PFSP_OK;
    }
  }
  const int xrows = n < 32 ? n : 32;
  int waves = 8;
  bool ent_lds = lb2_lds(c, 1, true, xrows) <= 64 * 1024;
  size_t lds = lb2_lds(c, waves, ent_lds, xrows);
  while (lds > 160 * 1024 && waves > 1) {
    waves >>= 1;
    lds = lb2_lds(c, waves, ent_lds, xrows);
  }
  int grid = (pool.count + waves - 1) / waves;
  const int cap = c->cu_count * 8;
  if (grid > cap) grid = cap;
  const dim3 g(grid), bl(64 * waves);
  KTimer kt(c, s, "k_lb2");
  if (c->narrow) {
    if (ent_lds)
      launch_lb2_e<Narrow, true>(subset, log, g, bl, lds, s, I, pool, ub, c->d_costs, out_lb,
                                 out_prune, xrows);
    else
      launch_lb2_e<Narrow, false>(subset, log, g, bl, lds, s, I, pool, ub, c->d_costs, out_lb,
                                  out_prune, xrows);
  } else {
    if (ent_lds)
      launch_lb2_e<Wide, true>(subset, log, g, bl, lds, s, I, pool, ub, c->d_costs, out_lb,
                               out_prune, xrows);
    else
      launch_lb2_e<Wide, false>(subset, log, g, bl, lds, s, I, pool, ub, c->d_costs, out_lb,
                                out_prune, xrows);
  }
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

// Generic kernels (any n, wide entries) on one staged instance that need not
// be the context's: costs into `costs` (stride 3 * I.m), then k_lb2.
int launch_generic_instance(Ctx *c, const DevInst &I, const DevPool &pool, int ub, int *costs,
                            int *out_lb, uint8_t *out_prune, hipStream_t s) {
  if (pool.count <= 0) return PFSP_OK;
  const int n = I.n, m = I.m;
  int b1 = 128;
  size_t lds1 = ((size_t)n * m + 3 * (size_t)m * b1) * 4;
  if (lds1 > 64 * 1024) {
    b1 = 64;
    lds1 = ((size_t)n * m + 3 * (size_t)m * b1) * 4;
  }
  {
    KTimer kt(c, s, "k_lb1");
    hipLaunchKernelGGL(k_lb1, dim3((pool.count + b1 - 1) / b1), dim3(b1), lds1, s, I, pool, ub,
                       out_lb, out_prune, costs, 0, c->d_flag, CostFilter{});
  }
  const int xrows = n < 32 ? n : 32;
  int waves = 8;
  const bool ent_lds = lb2_lds_inst(n, m, I.P, I.narrow, 1, true, xrows) <= 64 * 1024;
  size_t lds = lb2_lds_inst(n, m, I.P, I.narrow, waves, ent_lds, xrows);
  while (lds > 160 * 1024 && waves > 1) {
    waves >>= 1;
    lds = lb2_lds_inst(n, m, I.P, I.narrow, waves, ent_lds, xrows);
  }
  int grid = (pool.count + waves - 1) / waves;
  if (grid > c->cu_count * 8) grid = c->cu_count * 8;
  const dim3 g(grid), bl(64 * waves);
  KTimer kt(c, s, "k_lb2");
  if (I.narrow) {
    if (ent_lds)
      launch_lb2_e<Narrow, true>(false, false, g, bl, lds, s, I, pool, ub, costs, out_lb,
                                 out_prune, xrows);
    else
      launch_lb2_e<Narrow, false>(false, false, g, bl, lds, s, I, pool, ub, costs, out_lb,
                                  out_prune, xrows);
  } else {
    if (ent_lds)
      launch_lb2_e<Wide, true>(false, false, g, bl, lds, s, I, pool, ub, costs, out_lb, out_prune,
                               xrows);
    else
      launch_lb2_e<Wide, false>(false, false, g, bl, lds, s, I, pool, ub, costs, out_lb,
                                out_prune, xrows);
  }
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

}  // namespace pfsp
