// Wave64 helpers for gfx950 (CDNA4): 64 lanes execute in lockstep, so
// exchanging data through LDS inside one wave needs no workgroup barrier,
// only ordering of the LDS accesses.
#pragma once
#include <hip/hip_runtime.h>

namespace pfsp {

constexpr int kWave = 64;

// Orders this wave's LDS accesses around the call (no cross-wave effect).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// p (an LDS address) with its value hidden from the compiler: it then keeps
// the whole address in one register and puts the small constant offsets of
// the accesses through it into the instructions, instead of splitting off a
// large constant part that paired loads cannot encode and re-adding it
// before each pair.
template <class T>
__device__ __forceinline__ const T *lds_opaque(const T *p) {
  using LT = __attribute__((address_space(3))) const T;
  uint32_t a = (uint32_t)(uintptr_t)(LT *)p;
  asm("" : "+v"(a));
  return (const T *)(LT *)(uintptr_t)a;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
  return x;
}

__device__ __forceinline__ long long wave_sum64(long long x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ int wave_popc(bool pred) {
  return __popcll(__ballot(pred));
}

// Transposing max-reduction: lane L holds acc[0..63]; on return lane L holds
// in acc[0] the maximum over all lanes of the original acc[L].  63 exchanges
// instead of 64 separate 6-step reductions.  Each step is a template
// instance so that every array index is a compile-time constant (the array
// stays in registers).
template <int O>
__device__ __forceinline__ void transpose_max_step(int (&acc)[64], int lane) {
  const bool hi = (lane & O) != 0;
#pragma unroll
  for (int j = 0; j < O; ++j) {
    const int send = hi ? acc[j] : acc[O + j];
    const int keep = hi ? acc[O + j] : acc[j];
    acc[j] = max(keep, __shfl_xor(send, O, kWave));
  }
  if constexpr (O > 1) transpose_max_step<O / 2>(acc, lane);
}

__device__ __forceinline__ void transpose_max64(int (&acc)[64], int lane) {
  transpose_max_step<32>(acc, lane);
}

// The same reduction without the LDS crossbar (gfx950): the 32- and 16-lane
// exchanges use v_permlane32_swap / v_permlane16_swap, which swap the upper
// half-wave (odd 16-lane rows) of one register with the lower half-wave (even
// rows) of another, so max() of the two results is already the folded pair;
// the 8-, 4-, 2- and 1-lane steps use DPP (row rotation by 8, half-row mirror,
// quad permutations), each pairing lanes that differ in the step's bit.
template <int O>
__device__ __forceinline__ int dpp_partner(int x) {
  if constexpr (O == 8) return __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, false);  // row_ror:8
  if constexpr (O == 4) return __builtin_amdgcn_mov_dpp(x, 0x141, 0xf, 0xf, false);  // half mirror
  if constexpr (O == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, false);   // [2,3,0,1]
  return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, false);                         // [1,0,3,2]
}

template <int O, int N>
__device__ __forceinline__ void transpose_max_dpp(int (&acc)[N], int lane) {
  const bool hi = (lane & O) != 0;
#pragma unroll
  for (int j = 0; j < O; ++j) {
    const int send = hi ? acc[j] : acc[O + j];
    const int keep = hi ? acc[O + j] : acc[j];
    acc[j] = max(keep, dpp_partner<O>(send));
  }
  if constexpr (O > 1) transpose_max_dpp<O / 2>(acc, lane);
}

__device__ __forceinline__ void transpose_max64_xl(int (&acc)[64], int lane) {
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(acc[j], acc[32 + j], false, false);
    acc[j] = max((int)r[0], (int)r[1]);
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const auto r = __builtin_amdgcn_permlane16_swap(acc[j], acc[16 + j], false, false);
    acc[j] = max((int)r[0], (int)r[1]);
  }
  transpose_max_dpp<8>(acc, lane);
}

// Transposing max-reduction of per-job values held as two arrays, f (the
// forward children) and b (the backward children), NJ <= 32 entries each: on
// return lane q < 32 holds the maximum over all lanes of f[q] and lane 32 + q
// that of b[q] (lanes whose index is >= NJ hold NEG).  Entries that are
// known to be absent are never exchanged.
template <int NJ>
__device__ __forceinline__ int transpose_max_fb(const int (&f)[NJ], const int (&b)[NJ],
                                                int lane, int neg) {
  static_assert(NJ >= 1 && NJ <= 32, "one job per lane of a half-wave");
  int t[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(f[j], b[j], false, false);
    t[j] = max((int)r[0], (int)r[1]);
  }
  int acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (j < NJ) {
      const int hi = j + 16 < NJ ? t[j + 16 < NJ ? j + 16 : 0] : neg;
      const auto r = __builtin_amdgcn_permlane16_swap(t[j], hi, false, false);
      acc[j] = max((int)r[0], (int)r[1]);
    } else {
      acc[j] = neg;
    }
  }
  transpose_max_dpp<8>(acc, lane);
  return acc[0];
}

// Two int16 halves per register: wrapping add, signed max (v_pk_add_u16,
// v_pk_max_i16).
typedef short pk16 __attribute__((ext_vector_type(2)));
typedef unsigned short pku16 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int pk_add(int x, int y) {
  return __builtin_bit_cast(int, __builtin_bit_cast(pku16, x) + __builtin_bit_cast(pku16, y));
}
__device__ __forceinline__ int pk_max(int x, int y) {
  return __builtin_bit_cast(
      int, __builtin_elementwise_max(__builtin_bit_cast(pk16, x), __builtin_bit_cast(pk16, y)));
}

// a + b * c over the low 16 bits of a and b as signed integers
// (v_mad_i32_i16; the compiler forms it only as a sign extension and a
// 24-bit multiply-add, two instructions).
__device__ __forceinline__ int mad_i16(int a, int b, int c) {
  int d;
  asm("v_mad_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// pk_max with both halves of y replaced by its high half (an operand
// selection of the instruction, not a separate move).
__device__ __forceinline__ int pk_max_hi(int x, int y) {
  const pk16 b = __builtin_bit_cast(pk16, y);
  return __builtin_bit_cast(int, __builtin_elementwise_max(__builtin_bit_cast(pk16, x), b.yy));
}

// Transposing max-reduction of 32 per-job values held as int16 pairs
// (forward child low, backward child high), acc[OFF .. OFF + 32): on return
// lane q < 32 holds the maximum over all lanes of the low half of job q and
// lane 32 + q that of the high half (sign-extended).  Each step pairs two
// lanes that differ in one lane bit and keeps the jobs whose matching job bit
// equals the lane's: lane bit 5 <-> job bit 4 (permlane32 swap), 4 <-> 3
// (permlane16 swap), 3, 2, 1 <-> 2, 1, 0 (DPP); lane bit 0 folds last, so
// lane l ends with job l >> 1, and one lane gather puts job q in lanes q and
// 32 + q.
template <int O>
__device__ __forceinline__ void pk_split_dpp(int (&a)[2 * O], int lane, int lb_mask) {
  const bool hi = (lane & lb_mask) != 0;
#pragma unroll
  for (int j = 0; j < O; ++j) {
    const int send = hi ? a[j] : a[O + j];
    const int keep = hi ? a[O + j] : a[j];
    int got;
    if (lb_mask == 8) got = dpp_partner<8>(send);
    else if (lb_mask == 4) got = dpp_partner<4>(send);
    else got = dpp_partner<2>(send);
    a[j] = pk_max(keep, got);
  }
}

// Transposing max-reduction of NJ <= 32 such pairs without padding to 32
// jobs.  The lane bits are taken from 5 down to 0; while N > 1 registers are
// left, registers j and j + H (H = ceil(N / 2)) combine (lanes with the bit
// set keep the second's job, the others the first's, each taking the
// maximum with its partner lane across the bit), an odd N leaving register
// H - 1 to be folded with its partner unchanged; from one register on the
// remaining bits are folded.  Which lane ends with which job depends only on
// the lane's bits (tp_job); tp_source gives, for lane q or 32 + q, the first
// lane that ends with job q.
template <int LB>
__device__ __forceinline__ int tp_pair(int lo, int hi_job, bool hi) {
  if constexpr (LB == 5) {
    const auto r = __builtin_amdgcn_permlane32_swap(lo, hi_job, false, false);
    return pk_max((int)r[0], (int)r[1]);
  } else if constexpr (LB == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(lo, hi_job, false, false);
    return pk_max((int)r[0], (int)r[1]);
  } else {
    const int send = hi ? lo : hi_job, keep = hi ? hi_job : lo;
    return pk_max(keep, dpp_partner<(1 << LB)>(send));
  }
}

template <int LB>
__device__ __forceinline__ int tp_fold(int x) {
  if constexpr (LB == 5) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return pk_max((int)r[0], (int)r[1]);
  } else if constexpr (LB == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return pk_max((int)r[0], (int)r[1]);
  } else {
    return pk_max(x, dpp_partner<(1 << LB)>(x));
  }
}

template <int N, int LB, int NA>
__device__ __forceinline__ void tp_steps(int (&a)[NA], int lane) {
  if constexpr (LB >= 0) {
    constexpr int H = (N + 1) / 2;
    const bool hi = ((lane >> LB) & 1) != 0;
#pragma unroll
    for (int j = 0; j < N - H; ++j) a[j] = tp_pair<LB>(a[j], a[j + H], hi);
    if constexpr (N & 1) a[H - 1] = tp_fold<LB>(a[H - 1]);
    tp_steps<H, LB - 1>(a, lane);
  }
}

// The job that lane l holds after tp_steps<NJ, TOP> over NJ registers.
template <int NJ, int TOP = 5>
__host__ __device__ constexpr int tp_job(int l) {
  int ns[TOP + 1] = {};
  int n = NJ;
  for (int s = 0; s <= TOP; ++s) {
    ns[s] = n;
    n = (n + 1) / 2;
  }
  int j = 0;
  for (int s = TOP; s >= 0; --s) {  // step s takes lane bit TOP - s
    const int h = (ns[s] + 1) / 2;
    if (j < ns[s] - h && ((l >> (TOP - s)) & 1)) j += h;
  }
  return j;
}

// For groups of L lanes (lane bits below log2 L only): the lane of this
// lane's group that ends with job lane % L.
template <int L, int NJ>
__device__ __forceinline__ int tp_group_source(int lane) {
  constexpr int TOP = L == 64 ? 5 : L == 32 ? 4 : L == 16 ? 3 : L == 8 ? 2 : L == 4 ? 1 : 0;
  static_assert((1 << (TOP + 1)) == L && NJ <= L, "a power-of-two group of at most 64 lanes");
  const int q = lane & (L - 1);
  int src = 0;
#pragma unroll
  for (int l = L - 1; l >= 0; --l)
    if (tp_job<NJ, TOP>(l) == q) src = l;
  return (lane & ~(L - 1)) | src;
}

template <int NJ>
__device__ __forceinline__ int tp_source(int lane) {
  const int q = lane & 31;
  int src = 0;
#pragma unroll
  for (int l = 63; l >= 0; --l)
    if (tp_job<NJ>(l) == q) src = l;
  return src;
}

// acc[0 .. NJ) is consumed; src = tp_source<NJ>(lane).  Lane q < 32 returns
// job q's low-half maximum, lane 32 + q its high-half one (sign-extended).
template <int NJ>
__device__ __forceinline__ int transpose_pkmax(int (&acc)[NJ], int lane, int src) {
  static_assert(NJ >= 1 && NJ <= 32, "one job per lane of a half-wave");
  tp_steps<NJ, 5>(acc, lane);
  const int g = __shfl(acc[0], src, kWave);
  return lane < 32 ? (int)(short)(g & 0xffff) : g >> 16;
}

template <int OFF, int N>
__device__ __forceinline__ int transpose_pkmax32(const int (&acc)[N], int lane) {
  static_assert(OFF + 32 <= N, "32 jobs from OFF");
  int t[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(acc[OFF + j], acc[OFF + 16 + j], false, false);
    t[j] = pk_max((int)r[0], (int)r[1]);
  }
  int u[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const auto r = __builtin_amdgcn_permlane16_swap(t[j], t[8 + j], false, false);
    u[j] = pk_max((int)r[0], (int)r[1]);
  }
  pk_split_dpp<4>(u, lane, 8);
  int (&u4)[4] = *reinterpret_cast<int (*)[4]>(&u[0]);
  pk_split_dpp<2>(u4, lane, 4);
  int (&u2)[2] = *reinterpret_cast<int (*)[2]>(&u[0]);
  pk_split_dpp<1>(u2, lane, 2);
  const int w = pk_max(u[0], dpp_partner<1>(u[0]));
  const int g = __shfl(w, 2 * (lane & 31), kWave);
  return lane < 32 ? (int)(short)(g & 0xffff) : g >> 16;
}

// Minimum over the wave through permlane swaps and DPP (no LDS crossbar).
__device__ __forceinline__ int wave_min_xl(int x) {
  auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  x = min((int)r[0], (int)r[1]);
  r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = min((int)r[0], (int)r[1]);
  x = min(x, dpp_partner<8>(x));
  x = min(x, dpp_partner<4>(x));
  x = min(x, dpp_partner<2>(x));
  return min(x, dpp_partner<1>(x));
}

// Sum over each half-wave separately (lanes 0-31 and lanes 32-63); every
// lane of a half receives its half's sum.
__device__ __forceinline__ int half_sum(int x) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = (int)r[0] + (int)r[1];
  x += dpp_partner<8>(x);
  x += dpp_partner<4>(x);
  x += dpp_partner<2>(x);
  return x + dpp_partner<1>(x);
}

// Same reduction carrying an argument: the larger value wins, equal values
// keep the smaller argument.
template <int O>
__device__ __forceinline__ void transpose_argmax_step(int (&acc)[64], int (&arg)[64], int lane) {
  const bool hi = (lane & O) != 0;
#pragma unroll
  for (int j = 0; j < O; ++j) {
    const int sv = hi ? acc[j] : acc[O + j];
    const int sa = hi ? arg[j] : arg[O + j];
    const int kv = hi ? acc[O + j] : acc[j];
    const int ka = hi ? arg[O + j] : arg[j];
    const int rv = __shfl_xor(sv, O, kWave);
    const int ra = __shfl_xor(sa, O, kWave);
    const bool take = rv > kv || (rv == kv && ra < ka);
    acc[j] = take ? rv : kv;
    arg[j] = take ? ra : ka;
  }
  if constexpr (O > 1) transpose_argmax_step<O / 2>(acc, arg, lane);
}

__device__ __forceinline__ void transpose_argmax64(int (&acc)[64], int (&arg)[64], int lane) {
  transpose_argmax_step<32>(acc, arg, lane);
}

// MinMin accumulator (Section 2.3): minimum LB over both children sets,
// how often each set attains it, and the LB sums.
struct MinMin {
  int mn;
  int cf, cb;
  long long sf, sb;
  __device__ __forceinline__ void init() {
    mn = 0x7fffffff;
    cf = cb = 0;
    sf = sb = 0;
  }
  __device__ __forceinline__ void add(int x, bool backward) {
    if (x < mn) {
      mn = x;
      cf = cb = 0;
    }
    if (x == mn) {
      if (backward) ++cb; else ++cf;
    }
    if (backward) sb += x; else sf += x;
  }
  // merge a partial state (same definitions) into this one
  __device__ __forceinline__ void merge(int mn2, int cf2, int cb2, long long sf2, long long sb2) {
    if (mn2 < mn) {
      mn = mn2;
      cf = cf2;
      cb = cb2;
    } else if (mn2 == mn) {
      cf += cf2;
      cb += cb2;
    }
    sf += sf2;
    sb += sb2;
  }
  // 0 = forward, 1 = backward: fewer occurrences of the minimum wins, then
  // the larger sum, then forward.
  __device__ __forceinline__ int dir() const {
    if (cf != cb) return cb < cf ? 1 : 0;
    return sb > sf ? 1 : 0;
  }
};

}  // namespace pfsp
