// Learned machine-pair selector for LB2.
//
// Section 2.4 allows LB2 variants that evaluate anywhere between m and
// m(m-1)/2 machine pairs; a maximum over any subset of pairs is still a valid
// lower bound (max(LB1, subset maximum) <= full LB2).  The selector chooses
// the subset per parent: an MLP 64 -> 64 -> 64 -> 190 (ReLU; weights rounded to
// bfloat16, fp32 accumulation) scores the pairs of a 20-machine layout from 64
// features of the parent, and the `learned_topk` best pairs that exist on the
// instance are bounded exactly.  It is trained on the GPU from logged nodes:
// the target of a node is the share of its children whose full LB2 is
// attained first by each pair.
//
// Features (per parent, norm = the largest machine load of the instance):
//   [0,20) front C1[k]/norm, [20,40) back C2[k]/norm, [40,60) remaining
//   R[k]/norm for machines k < min(m, 20) (zero beyond), 60: d1/n, 61: d2/n,
//   62: (n - d1 - d2)/n, 63: LB1(parent)/norm.
#include <limits.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "internal.h"
#include "wave.h"

namespace pfsp {

constexpr int kIn = 64, kHid = 64, kOut = 190, kMMax = 20;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
              kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid,
              kParams = kOffB3 + kOut;
constexpr int kTopKMax = 32;   // float model and pfsp_selector_select
constexpr int kTopKMaxQ = 64;  // integer model

struct Selector {
  float *master = nullptr;  // fp32 parameters, layout W1[64][64] b1 W2[64][64] b2 W3[190][64] b3
  float *wq = nullptr;      // same layout, weights rounded to bfloat16 (biases copied)
  uint4 *bops = nullptr;    // wq's weights as bf16 MFMA B operands (float inference)
  float *grad = nullptr, *am = nullptr, *av = nullptr;
  long long step = 0;
  int loaded = 0;
  // per-batch workspaces (grown on demand)
  float *feat = nullptr, *scores = nullptr;
  uint32_t *mask = nullptr;
  int *reopen = nullptr;        // learned_exact: pool rows re-bounded with all pairs
  int *reopen_count = nullptr;  // [1]
  size_t rows_cap = 0;
  int mask_words = 0;
  // training workspaces
  float *h1 = nullptr, *h2 = nullptr, *ds = nullptr, *dh1 = nullptr, *dh2 = nullptr,
        *rowloss = nullptr, *loss = nullptr;
  float *part = nullptr;    // weight-gradient partials [row ranges][parameters]
  int *nvalid = nullptr;    // [1] rows of a training batch with a target
  uint4 *bopsT = nullptr;   // W2, W3 transposed as bf16 MFMA B operands (training)
  size_t train_cap = 0;
  int *to_inst = nullptr;  // [190]: instance pair index of each layout pair, -1 if absent
  int to_inst_m = -1;
  // integer-only model (used by the learned bound when set)
  uint2 *qops = nullptr;  // int8 MFMA B operands
  int *qbias = nullptr;   // per-lane biases
  float sx = 0.f;
  int M1 = 0, S1 = 0, M2 = 0, S2 = 0;
  int qloaded = 0;
};

// round to nearest even bfloat16, kept as float
__device__ __forceinline__ float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return x;  // NaN
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  return __uint_as_float(u);
}

__global__ void k_round_weights(const float *__restrict__ master, float *__restrict__ wq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const bool bias = (i >= kOffB1 && i < kOffW2) || (i >= kOffB2 && i < kOffW3) || i >= kOffB3;
  wq[i] = bias ? master[i] : bf16r(master[i]);
}

__global__ void k_features(DevInst I, DevPool pool, const int *__restrict__ costs, float norm,
                           float *__restrict__ feat) {
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int n = I.n, m = I.m;
  const int *cs = costs + (size_t)i * 3 * m;
  float *f = feat + (size_t)i * kIn;
  const int a = pool.d1[i], b = pool.d2[i];
  const bool bad = cs[0] < 0;  // invalid row flagged by k_lb1
  int lb1 = 0;
  for (int k = 0; k < m; ++k) lb1 = max(lb1, cs[k] + cs[2 * m + k] + cs[m + k]);
  for (int k = 0; k < kMMax; ++k) {
    const bool on = k < m && !bad;
    f[k] = on ? (float)cs[k] / norm : 0.f;
    f[20 + k] = on ? (float)cs[m + k] / norm : 0.f;
    f[40 + k] = on ? (float)cs[2 * m + k] / norm : 0.f;
  }
  f[60] = (float)a / (float)n;
  f[61] = (float)b / (float)n;
  f[62] = (float)(n - a - b) / (float)n;
  f[63] = bad ? 0.f : (float)lb1 / norm;
}

// Features of one parent from its costs row (the formula of k_features).
__device__ __forceinline__ void parent_features(int n, int m, const int *__restrict__ cs, int a,
                                                int b, float norm, float (&f)[kIn]) {
  const bool bad = cs[0] < 0;  // invalid row flagged by the costs kernel
  int lb1 = 0;
  for (int k = 0; k < m; ++k) lb1 = max(lb1, cs[k] + cs[2 * m + k] + cs[m + k]);
#pragma unroll
  for (int k = 0; k < kMMax; ++k) {
    const bool on = k < m && !bad;
    f[k] = on ? (float)cs[k] / norm : 0.f;
    f[20 + k] = on ? (float)cs[m + k] / norm : 0.f;
    f[40 + k] = on ? (float)cs[2 * m + k] / norm : 0.f;
  }
  f[60] = (float)a / (float)n;
  f[61] = (float)b / (float)n;
  f[62] = (float)(n - a - b) / (float)n;
  f[63] = bad ? 0.f : (float)lb1 / norm;
}

// ------------------------------------------------- integer-only inference
// The deployed selector is the MLP above quantized to int8 weights and
// activations with int32 accumulation, so every score is an exact integer
// and the ranking does not depend on the order of the sums:
//   features   xq[j] = clamp(rint(float(c) * q), 0, 127), c the integer
//              feature numerator (C1, C2, R, LB1 with q = sx / norm; d1, d2,
//              n - d1 - d2 with q = sx / n; zero for absent machines and
//              invalid rows), sx the feature scale (float32);
//   hidden     a = b + W.in (int32), h = min(127, (max(a, 0) * M + 2^(S-1)) >> S)
//              per layer (M in [1, 1023], S in [1, 30]);
//   scores     s = b3 + W3.h2 (int32); top-k pairs by s, ties to the lower
//              layout index (key s * 256 + 255 - index, unique).
// Blob (int32): sx bits, M1, S1, M2, S2, W1[64][64], b1[64], W2[64][64],
// b2[64], W3[190][64], b3[190]; weights in [-127, 127], |b| < 2^19.
constexpr int kQHead = 5;
constexpr int kQOffW1 = kQHead, kQOffB1 = kQOffW1 + kHid * kIn, kQOffW2 = kQOffB1 + kHid,
              kQOffB2 = kQOffW2 + kHid * kHid, kQOffW3 = kQOffB2 + kHid,
              kQOffB3 = kQOffW3 + kOut * kHid, kQParams = kQOffB3 + kOut;
// Device form: int8 MFMA B operands per (layer, column tile t, k step, lane)
// and per-lane biases.  v_mfma_i32_16x16x32_i8: lane l holds A row l % 16
// and B column l % 16 over k = 8 (l / 16) .. + 7; D register j is row
// 4 (l / 16) + j, column l % 16.  Hidden layers: tile t, column c computes
// unit 4c + t, so each lane's four tiles give four consecutive units (one
// 32-bit LDS store per row); the output layer: tile t, column c is pair
// 16t + c (t < 12).
constexpr int kQT1 = 4, kQT3 = 12;
constexpr int kQOpB1 = 0, kQOpB2 = kQOpB1 + kQT1 * 2 * 64, kQOpB3 = kQOpB2 + kQT1 * 2 * 64,
              kQOps = kQOpB3 + kQT3 * 2 * 64;  // uint2 entries
constexpr int kQBias1 = 0, kQBias2 = kQT1 * 64, kQBias3 = 2 * kQT1 * 64,
              kQBiases = kQBias3 + kQT3 * 64;  // int entries
// A wave takes 16 rows (one MFMA row tile); four lanes share a row's top-k.
constexpr int kQRows = 16, kQWaves = 4;
constexpr int kQRowStride = 72;                // bytes per LDS activation row (8-aligned)
constexpr int kQKeyStride = 68;                // ints per LDS key row: 4 tiles, 16-aligned
constexpr size_t kQWaveLds = 2 * kQRows * kQRowStride + kQRows * kQKeyStride * 4;

typedef int qv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int q8(float v) {  // rint, clamp to [0, 127]
  return (int)fminf(fmaxf(rintf(v), 0.f), 127.f);
}

// Bitonic networks over unique keys (max/min exchanges).
template <int N>
__device__ __forceinline__ void bitonic_sort_desc(int (&a)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const int hi = max(a[i], a[l]), lo = min(a[i], a[l]);
          const bool desc = (i & k) == 0;
          a[i] = desc ? hi : lo;
          a[l] = desc ? lo : hi;
        }
      }
}

template <int N>
__device__ __forceinline__ void bitonic_merge_desc(int (&a)[N]) {
#pragma unroll
  for (int j = N >> 1; j > 0; j >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int l = i ^ j;
      if (l > i) {
        const int hi = max(a[i], a[l]), lo = min(a[i], a[l]);
        a[i] = hi;
        a[l] = lo;
      }
    }
}

// Top-KMAX keys (larger first) of the wave's 16 rows over the 12 output
// tiles of 16 pairs.  tile_keys(t, tq) writes tile t's keys of every row to
// LDS slots [row][16 tq .. 16 tq + 15] of `keys` (stride kQKeyStride); four
// tiles go through LDS per round.  Lanes 4q .. 4q + 3 take row q: lane part
// p sorts tile 4u + p of each round with a bitonic network and merges it into
// a running list; two exchange-and-merge rounds (partners l ^ 1, l ^ 2)
// leave the row's top-KMAX in all four lanes.  Keys are unique per row.
template <int KMAX, class F>
__device__ __forceinline__ void topk_keys(int *keys, int lane, int (&best)[KMAX], F tile_keys) {
  const int srow = lane >> 2, p = lane & 3;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) best[q] = INT_MIN;
#pragma unroll 1
  for (int u = 0; u < kQT3 / 4; ++u) {
#pragma unroll
    for (int tq = 0; tq < 4; ++tq) tile_keys(4 * u + tq, tq);
    wave_sync();
    const int *kr = keys + srow * kQKeyStride + 16 * p;
    int ch[16];
#pragma unroll
    for (int q = 0; q < 16; q += 4) {
      const int4 v = *(const int4 *)(kr + q);
      ch[q] = v.x;
      ch[q + 1] = v.y;
      ch[q + 2] = v.z;
      ch[q + 3] = v.w;
    }
    wave_sync();  // the next round rewrites the keys
    bitonic_sort_desc<16>(ch);
    if (u == 0) {  // the first sorted tile is the running list as it stands
#pragma unroll
      for (int q = 0; q < KMAX; ++q) best[q] = q < 16 ? ch[q < 16 ? q : 0] : INT_MIN;
    } else {
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        const int r = KMAX - 1 - q;
        best[q] = max(best[q], r < 16 ? ch[r < 16 ? r : 0] : INT_MIN);
      }
      bitonic_merge_desc<KMAX>(best);
    }
  }
#pragma unroll
  for (int d = 1; d <= 2; d <<= 1) {  // merge with the partner's list
    int other[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) other[q] = __shfl_xor(best[q], d, kWave);
#pragma unroll
    for (int q = 0; q < KMAX; ++q) best[q] = max(best[q], other[KMAX - 1 - q]);
    bitonic_merge_desc<KMAX>(best);
  }
}

// Pair mask of the first k keys of a row (key low byte: 255 - layout index).
template <int KMAX>
__device__ __forceinline__ void write_mask(const int (&best)[KMAX], int k,
                                           const int *__restrict__ to_inst,
                                           uint32_t *__restrict__ mi, int words) {
  uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;  // 190 pairs fit 6 words
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < k && best[q] != INT_MIN) {
      const int pi = to_inst[255 - (best[q] & 255)];
      const uint32_t bit = 1u << (pi & 31);
      const int wd = pi >> 5;
      w0 |= wd == 0 ? bit : 0u;
      w1 |= wd == 1 ? bit : 0u;
      w2 |= wd == 2 ? bit : 0u;
      w3 |= wd == 3 ? bit : 0u;
      w4 |= wd == 4 ? bit : 0u;
      w5 |= wd == 5 ? bit : 0u;
    }
  }
  const uint32_t ws[6] = {w0, w1, w2, w3, w4, w5};
#pragma unroll
  for (int wd = 0; wd < 6; ++wd)
    if (wd < words) mi[wd] = ws[wd];
}

// One hidden layer for the wave's rows: A from `in` (row-major bytes), int8
// codes of the 64 units to `out`.
__device__ __forceinline__ void q_hidden(const unsigned char *in, unsigned char *out,
                                         const uint2 *__restrict__ ops, const int *__restrict__ bias,
                                         int M, int S, int lane) {
  const int c = lane & 15, g = lane >> 4;
  long bq[kQT1][2];
  int bb[kQT1];
#pragma unroll
  for (int t = 0; t < kQT1; ++t) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const uint2 e = ops[(t * 2 + ks) * 64 + lane];
      bq[t][ks] = (long)(((unsigned long)e.y << 32) | e.x);
    }
    bb[t] = bias[t * 64 + lane];
  }
  const unsigned rnd = 1u << (S - 1);
#pragma unroll
  for (int s = 0; s < kQRows / 16; ++s) {
    const unsigned char *row = in + (16 * s + c) * kQRowStride + 8 * g;
    const long a0 = *(const long *)row, a1 = *(const long *)(row + 32);
    unsigned code[4] = {0u, 0u, 0u, 0u};  // rows 4g + j: units 4c .. 4c + 3
#pragma unroll
    for (int t = 0; t < kQT1; ++t) {
      qv4 d = {0, 0, 0, 0};
      d = __builtin_amdgcn_mfma_i32_16x16x32_i8(a0, bq[t][0], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_i32_16x16x32_i8(a1, bq[t][1], d, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned h = (unsigned)max(d[j] + bb[t], 0);
        code[j] |= min((h * (unsigned)M + rnd) >> S, 127u) << (8 * t);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *(unsigned *)(out + (16 * s + 4 * g + j) * kQRowStride + 4 * c) = code[j];
  }
}

// Fused integer inference: features from the costs workspace, the three
// layers on int8 MFMA, the top-KMAX keys per row, the pair masks.  Each wave
// takes 16 consecutive pool rows.  Features: lane l computes features
// 16 (l / 16) .. + 15 of row l % 16.  Selection: lanes 4q .. 4q + 3 share row
// q; the output layer runs four 16-pair tiles at a time through LDS and lane
// part p keeps the top-KMAX of tiles p, p + 4, p + 8; two exchange-and-merge
// rounds (lanes l ^ 1, then l ^ 2) give all four the row's top-KMAX.
template <int KMAX>
__global__ void __launch_bounds__(64 * kQWaves)
k_infer_q(DevInst I, DevPool pool, const int *__restrict__ costs, float qs, float qd,
          const uint2 *__restrict__ ops, const int *__restrict__ bias, int M1, int S1, int M2,
          int S2, const int *__restrict__ to_inst, int k, int words,
          uint32_t *__restrict__ mask) {
  extern __shared__ __align__(16) unsigned char qsm[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int base = (blockIdx.x * kQWaves + w) * kQRows;
  if (base >= count) return;  // waves never synchronize across the block
  unsigned char *xa = qsm + (size_t)w * kQWaveLds;
  unsigned char *xb = xa + kQRows * kQRowStride;
  int *keys = (int *)(xb + kQRows * kQRowStride);
  const int n = I.n, m = I.m;
  // features: 16 of row lane % 16
  {
    const int fr = lane & 15, fg = lane >> 4;
    const int it = base + fr;
    unsigned f[4] = {0u, 0u, 0u, 0u};
    if (it < count) {
      const int i = pool.index ? pool.index[it] : it;
      const int *cs = costs + (size_t)i * 3 * m;
      const bool bad = cs[0] < 0;  // invalid row flagged by the costs kernel
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int x = 16 * fg + e;  // feature index
        unsigned code = 0u;
        if (x < 60) {
          const int part = x / 20, kk = x - 20 * part;  // C1, C2, R of machine kk
          if (kk < m && !bad) code = (unsigned)q8((float)cs[part * m + kk] * qs);
        } else {
          const int a = pool.d1[i], b = pool.d2[i];
          if (x == 60) code = (unsigned)q8((float)a * qd);
          if (x == 61) code = (unsigned)q8((float)b * qd);
          if (x == 62) code = (unsigned)q8((float)(n - a - b) * qd);
          if (x == 63 && !bad) {
            int lb1 = 0;
            for (int y = 0; y < m; ++y) lb1 = max(lb1, cs[y] + cs[2 * m + y] + cs[m + y]);
            code = (unsigned)q8((float)lb1 * qs);
          }
        }
        f[e >> 2] |= code << (8 * (e & 3));
      }
    }
    unsigned char *dst = xa + fr * kQRowStride + 16 * fg;
    *(uint2 *)dst = make_uint2(f[0], f[1]);
    *(uint2 *)(dst + 8) = make_uint2(f[2], f[3]);
  }
  wave_sync();
  q_hidden(xa, xb, ops + kQOpB1, bias + kQBias1, M1, S1, lane);
  wave_sync();
  q_hidden(xb, xa, ops + kQOpB2, bias + kQBias2, M2, S2, lane);
  wave_sync();
  // output layer: keys of 16 pairs per tile, four tiles per round
  const int c = lane & 15, g = lane >> 4;
  const unsigned char *arow = xa + c * kQRowStride + 8 * g;
  const long a0 = *(const long *)arow, a1 = *(const long *)(arow + 32);
  int best[KMAX];
  topk_keys<KMAX>(keys, lane, best, [&](int t, int tq) {
    const uint2 e0 = ops[kQOpB3 + (t * 2) * 64 + lane];
    const uint2 e1 = ops[kQOpB3 + (t * 2 + 1) * 64 + lane];
    const long b0 = (long)(((unsigned long)e0.y << 32) | e0.x);
    const long b1 = (long)(((unsigned long)e1.y << 32) | e1.x);
    const int o = 16 * t + c;
    const bool valid = o < kOut && to_inst[o < kOut ? o : 0] >= 0;
    const int kb = bias[kQBias3 + t * 64 + lane];
    qv4 d = {0, 0, 0, 0};
    d = __builtin_amdgcn_mfma_i32_16x16x32_i8(a0, b0, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_i32_16x16x32_i8(a1, b1, d, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      keys[(4 * g + j) * kQKeyStride + 16 * tq + c] =
          valid ? (d[j] + kb) * 256 + (255 - o) : INT_MIN;
  });
  const int it = base + (lane >> 2);
  if ((lane & 3) != 0 || it >= count) return;
  const int i = pool.index ? pool.index[it] : it;
  write_mask<KMAX>(best, k, to_inst, mask + (size_t)i * words, words);
}

// ---------------------------------------------- float inference on MFMA
// The float form (bf16-rounded weights, fp32 activations and sums) on
// v_mfma_f32_16x16x32_bf16, with the layout of k_infer_q: a wave takes 16
// rows.  The MFMA multiplies bf16 operands, so every activation x (features,
// hidden units) enters as two bf16 numbers, hi = bf16(x) and lo = bf16(x -
// hi), and each tile is accumulated over both: w hi + w lo is exact in fp32
// and differs from w x by at most |w x| 2^-17.  Scores rank by a key that
// keeps their leading 24 bits (sign, exponent, 15 mantissa bits, in an
// order-preserving integer form) and puts 255 - layout index in the low byte:
// scores that agree in those bits go to the lower index.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kBRowStride = 272;  // bytes per LDS row: 64 hi + 64 lo bf16, padded
constexpr int kBLo = 128;         // byte offset of the lo half
constexpr size_t kBWaveLds = 2 * kQRows * kBRowStride + kQRows * kQKeyStride * 4;
// B operands (8 bf16 = one uint4 per lane): hidden layers as the integer
// model (tile t, column c = unit 4c + t), output tile t, column c = pair 16t + c
constexpr int kBOpB1 = 0, kBOpB2 = kQT1 * 2 * 64, kBOpB3 = 2 * kQT1 * 2 * 64,
              kBOps = kBOpB3 + kQT3 * 2 * 64;

__device__ __forceinline__ uint32_t bf16_bits(float x) { return __float_as_uint(bf16r(x)) >> 16; }

// Order-preserving key of a float score with the layout index in the low byte.
__device__ __forceinline__ int score_key(float s, int o) {
  const uint32_t u = __float_as_uint(s);
  const int ord = (u & 0x80000000u) ? (int)(u ^ 0x7fffffffu) : (int)u;
  return (ord & ~0xff) | (255 - o);
}

// Packs the bf16-rounded weights into MFMA B operands.
__global__ void k_pack_bf16(const float *__restrict__ wq, uint4 *__restrict__ ops) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kBOps) return;
  const int lane = e & 63, ks = (e >> 6) & 1, tile = e >> 7;
  const int c = lane & 15, k0 = 32 * ks + 8 * (lane >> 4);
  const float *w = nullptr;
  if (e < kBOpB3) {
    const int L = tile / kQT1, t = tile - L * kQT1;
    w = wq + (L == 0 ? kOffW1 : kOffW2) + (4 * c + t) * kIn + k0;
  } else {
    const int o = 16 * (tile - 2 * kQT1) + c;
    if (o < kOut) w = wq + kOffW3 + o * kHid + k0;
  }
  uint32_t h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = w ? bf16_bits(w[i]) : 0u;
  ops[e] = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16,
                      h[6] | h[7] << 16);
}

__device__ __forceinline__ void bf_store8(unsigned char *row, int unit0, const float (&x)[4]) {
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float h = bf16r(x[i]);
    hi[i] = __float_as_uint(h) >> 16;
    lo[i] = bf16_bits(x[i] - h);
  }
  *(uint2 *)(row + 2 * unit0) = make_uint2(hi[0] | hi[1] << 16, hi[2] | hi[3] << 16);
  *(uint2 *)(row + kBLo + 2 * unit0) = make_uint2(lo[0] | lo[1] << 16, lo[2] | lo[3] << 16);
}

// A operands (hi, lo) of row lane % 16 for k-step ks.
__device__ __forceinline__ void bf_a(const unsigned char *rows, int lane, int ks, bf16x8 &hi,
                                     bf16x8 &lo) {
  const unsigned char *row = rows + (lane & 15) * kBRowStride + 2 * (32 * ks + 8 * (lane >> 4));
  hi = *(const bf16x8 *)row;
  lo = *(const bf16x8 *)(row + kBLo);
}

__device__ __forceinline__ f32x4 bf_tile(const bf16x8 (&ah)[2], const bf16x8 (&al)[2],
                                         const uint4 *__restrict__ ops, int lane) {
  f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const uint4 e = ops[ks * 64 + lane];
    const bf16x8 b = __builtin_bit_cast(bf16x8, e);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], b, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], b, d, 0, 0, 0);
  }
  return d;
}

// One hidden layer: relu(W in + b) of the wave's 16 rows into `out`.
__device__ __forceinline__ void bf_hidden(const unsigned char *in, unsigned char *out,
                                          const uint4 *__restrict__ ops,
                                          const float *__restrict__ bias, int lane) {
  const int c = lane & 15, g = lane >> 4;
  bf16x8 ah[2], al[2];
  bf_a(in, lane, 0, ah[0], al[0]);
  bf_a(in, lane, 1, ah[1], al[1]);
  float h[4][4];  // [row 4g + j][unit 4c + t]
#pragma unroll
  for (int t = 0; t < kQT1; ++t) {
    const f32x4 d = bf_tile(ah, al, ops + t * 2 * 64, lane);
    const float b = bias[4 * c + t];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j][t] = fmaxf(d[j] + b, 0.f);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) bf_store8(out + (4 * g + j) * kBRowStride, 4 * c, h[j]);
}

// XIN: the features are rows of x [count][64] instead of being computed from
// the costs workspace.  scores_out (optional, [count][190]) receives every
// score (-inf for pairs absent on the instance); mask (optional) the top-k
// pair masks.
template <int KMAX, bool XIN>
__global__ void __launch_bounds__(64 * kQWaves)
k_infer_bf(DevInst I, DevPool pool, const int *__restrict__ costs, const float *__restrict__ xin,
           float norm, const uint4 *__restrict__ ops, const float *__restrict__ wq,
           const int *__restrict__ to_inst, int k, int words, uint32_t *__restrict__ mask,
           float *__restrict__ scores_out) {
  extern __shared__ __align__(16) unsigned char bsm[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int base = (blockIdx.x * kQWaves + w) * kQRows;
  if (base >= count) return;  // waves never synchronize across the block
  unsigned char *xa = bsm + (size_t)w * kBWaveLds;
  unsigned char *xb = xa + kQRows * kBRowStride;
  int *keys = (int *)(xb + kQRows * kBRowStride);
  const int n = I.n, m = I.m;
  {  // features 16 (lane / 16) .. + 15 of row lane % 16 (the formulas of k_features)
    const int fr = lane & 15, fg = lane >> 4;
    const int it = base + fr;
    float f[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) f[e] = 0.f;
    if (XIN && it < count) {
      const float4 *src = (const float4 *)(xin + (size_t)it * kIn + 16 * fg);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = src[q];
        f[4 * q] = v.x;
        f[4 * q + 1] = v.y;
        f[4 * q + 2] = v.z;
        f[4 * q + 3] = v.w;
      }
    } else if (it < count) {
      const int i = pool.index ? pool.index[it] : it;
      const int *cs = costs + (size_t)i * 3 * m;
      const bool bad = cs[0] < 0;
      const int a = pool.d1[i], b = pool.d2[i];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int x = 16 * fg + e;
        if (x < 60) {
          const int part = x / 20, kk = x - 20 * part;
          if (kk < m && !bad) f[e] = (float)cs[part * m + kk] / norm;
        } else if (x == 60) {
          f[e] = (float)a / (float)n;
        } else if (x == 61) {
          f[e] = (float)b / (float)n;
        } else if (x == 62) {
          f[e] = (float)(n - a - b) / (float)n;
        } else if (!bad) {
          int lb1 = 0;
          for (int y = 0; y < m; ++y) lb1 = max(lb1, cs[y] + cs[2 * m + y] + cs[m + y]);
          f[e] = (float)lb1 / norm;
        }
      }
    }
    unsigned char *row = xa + fr * kBRowStride;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x4[4] = {f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]};
      bf_store8(row, 16 * fg + 4 * q, x4);
    }
  }
  wave_sync();
  bf_hidden(xa, xb, ops + kBOpB1, wq + kOffB1, lane);
  wave_sync();
  bf_hidden(xb, xa, ops + kBOpB2, wq + kOffB2, lane);
  wave_sync();
  const int c = lane & 15, g = lane >> 4;
  bf16x8 ah[2], al[2];
  bf_a(xa, lane, 0, ah[0], al[0]);
  bf_a(xa, lane, 1, ah[1], al[1]);
  int best[KMAX];
  topk_keys<KMAX>(keys, lane, best, [&](int t, int tq) {
    const int o = 16 * t + c;
    const bool valid = o < kOut && to_inst[o < kOut ? o : 0] >= 0;
    const float b3 = wq[kOffB3 + (o < kOut ? o : 0)];
    const f32x4 d = bf_tile(ah, al, ops + kBOpB3 + t * 2 * 64, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float sc = d[j] + b3;
      keys[(4 * g + j) * kQKeyStride + 16 * tq + c] = valid ? score_key(sc, o) : INT_MIN;
      const int row = base + 4 * g + j;
      if (scores_out && o < kOut && row < count)
        scores_out[(size_t)row * kOut + o] = valid ? sc : -INFINITY;
    }
  });
  const int it = base + (lane >> 2);
  if (!mask || (lane & 3) != 0 || it >= count) return;
  const int i = pool.index ? pool.index[it] : it;
  write_mask<KMAX>(best, k, to_inst, mask + (size_t)i * words, words);
}

// Top-k layout pairs per row (larger score first; equal scores: lower index),
// written as a bit mask over the instance's pair indices.
__global__ void k_select(const float *__restrict__ scores, int rows, const int *__restrict__ rows_dev,
                         int k, const int *__restrict__ to_inst, int words,
                         uint32_t *__restrict__ mask) {
  const int B = rows_dev ? *rows_dev : rows;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const float *si = scores + (size_t)i * kOut;
  float best[kTopKMax];
  int idx[kTopKMax];
#pragma unroll
  for (int t = 0; t < kTopKMax; ++t) {
    best[t] = -INFINITY;
    idx[t] = -1;
  }
  for (int o = 0; o < kOut; ++o) {
    if (to_inst[o] < 0) continue;
    float v = si[o];
    int id = o;
    // insertion into the descending list best[0..k); scanning o upwards and
    // moving an entry down only past strictly smaller ones keeps lower indices
    // first among equal scores
#pragma unroll
    for (int t = 0; t < kTopKMax; ++t) {
      if (t < k && (idx[t] < 0 || v > best[t])) {
        const float tv = best[t];
        const int ti = idx[t];
        best[t] = v;
        idx[t] = id;
        v = tv;
        id = ti;
      }
    }
  }
  uint32_t *mi = mask + (size_t)i * words;
  for (int w = 0; w < words; ++w) mi[w] = 0;
#pragma unroll
  for (int t = 0; t < kTopKMax; ++t)
    if (t < k && idx[t] >= 0) {
      const int pi = to_inst[idx[t]];
      mi[pi >> 5] |= 1u << (pi & 31);
    }
}

// Training targets from logged argmax pairs: share of the node's children
// whose LB2 is attained first by each layout pair.
__global__ void k_targets(DevInst I, DevPool pool, const int16_t *__restrict__ argpair,
                          const int *__restrict__ inst_to20, float *__restrict__ target) {
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int n = I.n;
  float *t = target + (size_t)i * kOut;
  for (int o = 0; o < kOut; ++o) t[o] = 0.f;
  const int r = n - pool.d1[i] - pool.d2[i];
  int tot = 0;
  for (int dir = 0; dir < 2; ++dir)
    for (int q = 0; q < r && q < n; ++q) tot += argpair[((size_t)i * 2 + dir) * n + q] >= 0;
  if (tot == 0) return;
  const float w = 1.f / (float)tot;
  for (int dir = 0; dir < 2; ++dir)
    for (int q = 0; q < r && q < n; ++q) {
      const int a = argpair[((size_t)i * 2 + dir) * n + q];
      if (a >= 0) t[inst_to20[a]] += w;
    }
}

// ------------------------------------------------------ training on MFMA
// One training step runs the forward and backward passes of 16 rows per
// wave on v_mfma_f32_16x16x32_bf16 with the operand layout of k_infer_bf
// (activations and errors as bf16 hi + lo pairs, weights as their bf16
// values), then the weight gradients as tiled products over the batch rows
// on the same instruction (both operands as hi + lo pairs, three products per
// step), summed over row ranges in a fixed order.
//
// Backward B operands: W2 and W3 transposed (tile t, column c = input unit
// 4c + t, k = output unit), so that the errors of a layer's inputs, dOut W,
// come out in the layout of the forward layers.
constexpr int kTOpW2 = 0;                        // 4 tiles x 2 k-steps x 64 lanes
constexpr int kTOpW3 = kQT1 * 2 * 64;            // 4 tiles x 6 k-steps x 64 lanes
constexpr int kTOps = kTOpW3 + kQT1 * 6 * 64;
constexpr int kTDRow = 2 * 192 * 2 + 16;         // bytes per LDS row of output errors
constexpr int kTDLo = 384;                       // byte offset of their lo half
constexpr size_t kTWaveLds = 2 * kQRows * kBRowStride + kQRows * kTDRow;
constexpr int kTTiles = 16 + 16 + 48;            // 16 x 16 weight-gradient tiles: W1, W2, W3
constexpr int kTRowsPerSplit = 256;              // batch rows per weight-gradient partial

__global__ void k_pack_bf16t(const float *__restrict__ wq, uint4 *__restrict__ ops) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kTOps) return;
  const int lane = e & 63, c = lane & 15, k0 = 8 * (lane >> 4);
  int t, ks, off, nout;
  if (e < kTOpW3) {
    const int idx = e >> 6;
    t = idx >> 1;
    ks = idx & 1;
    off = kOffW2;
    nout = kHid;
  } else {
    const int idx = (e - kTOpW3) >> 6;
    t = idx / 6;
    ks = idx - 6 * t;
    off = kOffW3;
    nout = kOut;
  }
  const int j = 4 * c + t;
  uint32_t h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int o = 32 * ks + k0 + i;
    h[i] = o < nout ? bf16_bits(wq[off + o * kHid + j]) : 0u;
  }
  ops[e] = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16,
                      h[6] | h[7] << 16);
}

// One hidden layer of the training pass: h = relu(W in + b) into `out` (hi,
// lo rows) and h[j][t] (row 4g + j, unit 4c + t) in registers.
__device__ __forceinline__ void train_layer(const unsigned char *in, unsigned char *out,
                                            const uint4 *__restrict__ ops,
                                            const float *__restrict__ bias, int lane,
                                            float (&h)[4][4]) {
  const int c = lane & 15, g = lane >> 4;
  bf16x8 ah[2], al[2];
  bf_a(in, lane, 0, ah[0], al[0]);
  bf_a(in, lane, 1, ah[1], al[1]);
#pragma unroll
  for (int t = 0; t < kQT1; ++t) {
    const f32x4 d = bf_tile(ah, al, ops + t * 2 * 64, lane);
    const float b = bias[4 * c + t];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j][t] = fmaxf(d[j] + b, 0.f);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) bf_store8(out + (4 * g + j) * kBRowStride, 4 * c, h[j]);
}

__device__ __forceinline__ float group16_max(float x) {
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ float group16_sum(float x) {
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ bf16x8 bf_pack8(const uint32_t (&h)[8]) {
  return __builtin_bit_cast(bf16x8, make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16,
                                               h[4] | h[5] << 16, h[6] | h[7] << 16));
}

// Forward pass, soft-target cross-entropy and backpropagated errors of the
// wave's 16 rows: H1, H2 (after relu), DS = softmax - t over the instance's
// pairs (0 for a row without target), DH2 and DH1 (masked by the relu), each
// row's loss, and the number of rows with a target added to *nvalid (the
// gradients are scaled by its inverse when the partials are summed).
__global__ void __launch_bounds__(64 * kQWaves)
k_train_fb(const float *__restrict__ x, const float *__restrict__ target, int B,
           int *__restrict__ nvalid,
           const uint4 *__restrict__ ops, const uint4 *__restrict__ opsT,
           const float *__restrict__ wq, const int *__restrict__ to_inst, float *__restrict__ H1,
           float *__restrict__ H2, float *__restrict__ DS, float *__restrict__ DH1,
           float *__restrict__ DH2, float *__restrict__ rowloss) {
  extern __shared__ __align__(16) unsigned char tsm[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int base = (blockIdx.x * kQWaves + w) * kQRows;
  if (base >= B) return;  // waves never synchronize across the block
  unsigned char *xa = tsm + (size_t)w * kTWaveLds;
  unsigned char *xb = xa + kQRows * kBRowStride;
  unsigned char *dr = xb + kQRows * kBRowStride;
  const int c = lane & 15, g = lane >> 4;
  {  // inputs 16 (lane / 16) .. + 15 of row lane % 16
    const int it = base + c;
    float f[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) f[e] = 0.f;
    if (it < B) {
      const float4 *src = (const float4 *)(x + (size_t)it * kIn + 16 * g);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = src[q];
        f[4 * q] = v.x;
        f[4 * q + 1] = v.y;
        f[4 * q + 2] = v.z;
        f[4 * q + 3] = v.w;
      }
    }
    unsigned char *row = xa + c * kBRowStride;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float x4[4] = {f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]};
      bf_store8(row, 16 * g + 4 * q, x4);
    }
  }
  wave_sync();
  float h1[4][4], h2[4][4];
  train_layer(xa, xb, ops + kBOpB1, wq + kOffB1, lane, h1);
  wave_sync();
  train_layer(xb, xa, ops + kBOpB2, wq + kOffB2, lane, h2);
  wave_sync();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = base + 4 * g + j;
    if (row < B) {
      *(float4 *)(H1 + (size_t)row * kHid + 4 * c) = make_float4(h1[j][0], h1[j][1], h1[j][2], h1[j][3]);
      *(float4 *)(H2 + (size_t)row * kHid + 4 * c) = make_float4(h2[j][0], h2[j][1], h2[j][2], h2[j][3]);
    }
  }
  // scores of pairs o = 16 t + c, rows 4 g + j
  float sc[kQT3][4];
  bool val[kQT3];
  {
    bf16x8 ah[2], al[2];
    bf_a(xa, lane, 0, ah[0], al[0]);
    bf_a(xa, lane, 1, ah[1], al[1]);
#pragma unroll
    for (int t = 0; t < kQT3; ++t) {
      const int o = 16 * t + c;
      val[t] = o < kOut && to_inst[o < kOut ? o : 0] >= 0;
      const float b3 = wq[kOffB3 + (o < kOut ? o : 0)];
      const f32x4 d = bf_tile(ah, al, ops + kBOpB3 + t * 2 * 64, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) sc[t][j] = d[j] + b3;
    }
  }
  // per row: log-sum-exp over the instance's pairs, target mass, loss, errors
  float ds[kQT3][4];
  int nv = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = base + 4 * g + j;
    float mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < kQT3; ++t)
      if (val[t]) mx = fmaxf(mx, sc[t][j]);
    mx = group16_max(mx);
    float se = 0.f;
#pragma unroll
    for (int t = 0; t < kQT3; ++t)
      if (val[t]) se += expf(sc[t][j] - mx);
    const float lse = mx + logf(group16_sum(se));
    float tv[kQT3], tsum = 0.f, loss = 0.f;
#pragma unroll
    for (int t = 0; t < kQT3; ++t) {
      const int o = 16 * t + c;
      tv[t] = row < B && o < kOut ? target[(size_t)row * kOut + o] : 0.f;
      tsum += tv[t];
      if (val[t]) loss -= tv[t] * (sc[t][j] - lse);
    }
    tsum = group16_sum(tsum);
    loss = group16_sum(loss);
    const float sr = tsum > 0.f ? 1.f : 0.f;
    nv += __popcll(__ballot(c == 0 && row < B && tsum > 0.f));
#pragma unroll
    for (int t = 0; t < kQT3; ++t) {
      ds[t][j] = val[t] ? (expf(sc[t][j] - lse) - tv[t]) * sr : 0.f;
      const int o = 16 * t + c;
      if (row < B && o < kOut) DS[(size_t)row * kOut + o] = ds[t][j];
    }
    if (row < B && c == 0) rowloss[row] = tsum > 0.f ? loss : 0.f;
  }
  if (lane == 0 && nv) atomicAdd(nvalid, nv);
  // the errors as hi, lo rows of 192 (pairs 190, 191 are zero)
#pragma unroll
  for (int t = 0; t < kQT3; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned char *row = dr + (4 * g + j) * kTDRow + 2 * (16 * t + c);
      const float hv = bf16r(ds[t][j]);
      *(unsigned short *)row = (unsigned short)(__float_as_uint(hv) >> 16);
      *(unsigned short *)(row + kTDLo) = (unsigned short)bf16_bits(ds[t][j] - hv);
    }
  wave_sync();
  // DH2 = DS W3, masked by the relu of H2
  float dh2[4][4];
  {
    bf16x8 ah[6], al[6];
#pragma unroll
    for (int ks = 0; ks < 6; ++ks) {
      const unsigned char *row = dr + c * kTDRow + 2 * (32 * ks + 8 * g);
      ah[ks] = *(const bf16x8 *)row;
      al[ks] = *(const bf16x8 *)(row + kTDLo);
    }
#pragma unroll
    for (int t = 0; t < kQT1; ++t) {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 6; ++ks) {
        const bf16x8 b = __builtin_bit_cast(bf16x8, opsT[kTOpW3 + (t * 6 + ks) * 64 + lane]);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], b, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], b, d, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) dh2[j][t] = h2[j][t] > 0.f ? d[j] : 0.f;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = base + 4 * g + j;
    if (row < B)
      *(float4 *)(DH2 + (size_t)row * kHid + 4 * c) =
          make_float4(dh2[j][0], dh2[j][1], dh2[j][2], dh2[j][3]);
    bf_store8(xb + (4 * g + j) * kBRowStride, 4 * c, dh2[j]);
  }
  wave_sync();
  // DH1 = DH2 W2, masked by the relu of H1
  {
    bf16x8 ah[2], al[2];
    bf_a(xb, lane, 0, ah[0], al[0]);
    bf_a(xb, lane, 1, ah[1], al[1]);
    float dh1[4][4];
#pragma unroll
    for (int t = 0; t < kQT1; ++t) {
      const f32x4 d = bf_tile(ah, al, opsT + kTOpW2 + t * 2 * 64, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) dh1[j][t] = h1[j][t] > 0.f ? d[j] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = base + 4 * g + j;
      if (row < B)
        *(float4 *)(DH1 + (size_t)row * kHid + 4 * c) =
            make_float4(dh1[j][0], dh1[j][1], dh1[j][2], dh1[j][3]);
    }
  }
}

// Weight and bias gradients over one range of kTRowsPerSplit batch rows:
// wave (tile, split) computes the 16 x 16 tile of dW = sum over rows of
// D[r][u] A[r][v] (u output unit, v input unit; W1: DH1 and X, W2: DH2 and
// H1, W3: DS and H2), and the tiles of the first input units also the bias
// gradients sum over rows of D[r][u].  part[split][parameter].
__global__ void __launch_bounds__(256)
k_train_wgrad(const float *__restrict__ x, const float *__restrict__ H1,
              const float *__restrict__ H2, const float *__restrict__ DS,
              const float *__restrict__ DH1, const float *__restrict__ DH2, int B,
              float *__restrict__ part) {
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int tile = wv % kTTiles, split = wv / kTTiles;
  const int r0 = split * kTRowsPerSplit, r1 = min(B, r0 + kTRowsPerSplit);
  if (r0 >= B) return;  // uniform per wave
  const float *Dm, *Am;
  int dstride, woff, boff, nout, to, tj;
  if (tile < 16) {
    Dm = DH1; Am = x; dstride = kHid; woff = kOffW1; boff = kOffB1; nout = kHid;
    to = tile >> 2; tj = tile & 3;
  } else if (tile < 32) {
    Dm = DH2; Am = H1; dstride = kHid; woff = kOffW2; boff = kOffB2; nout = kHid;
    to = (tile - 16) >> 2; tj = (tile - 16) & 3;
  } else {
    Dm = DS; Am = H2; dstride = kOut; woff = kOffW3; boff = kOffB3; nout = kOut;
    to = (tile - 32) >> 2; tj = (tile - 32) & 3;
  }
  const int i = lane & 15, kg = lane >> 4;
  const int u = 16 * to + i, v = 16 * tj + i;
  const bool uok = u < nout;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int rk = r0; rk < r1; rk += 32) {
    float a[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = rk + 8 * kg + e;
      const bool ok = r < r1;
      a[e] = ok && uok ? Dm[(size_t)r * dstride + u] : 0.f;
      b[e] = ok ? Am[(size_t)r * kHid + v] : 0.f;
    }
    uint32_t ahb[8], alb[8], bhb[8], blb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      bsum += a[e];
      const float ah = bf16r(a[e]), bh = bf16r(b[e]);
      ahb[e] = __float_as_uint(ah) >> 16;
      alb[e] = bf16_bits(a[e] - ah);
      bhb[e] = __float_as_uint(bh) >> 16;
      blb[e] = bf16_bits(b[e] - bh);
    }
    const bf16x8 Ah = bf_pack8(ahb), Al = bf_pack8(alb), Bh = bf_pack8(bhb), Bl = bf_pack8(blb);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc, 0, 0, 0);
  }
  float *pp = part + (size_t)split * kParams;
  // D register j: output unit 16 to + 4 kg + j, input unit 16 tj + i
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int uo = 16 * to + 4 * kg + j;
    if (uo < nout) pp[woff + uo * kHid + 16 * tj + i] = acc[j];
  }
  if (tj == 0) {  // bias: the four row groups of output unit u
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (kg == 0 && uok) pp[boff + u] = bsum;
  }
}

// grad = the row-range partials summed in range order, over the rows with
// a target (at least one).
__global__ void k_train_reduce(const float *__restrict__ part, int splits,
                               const int *__restrict__ nvalid, float *__restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float g = 0.f;
  for (int s = 0; s < splits; ++s) g += part[(size_t)s * kParams + p];
  grad[p] = g / (float)max(1, *nvalid);
}

__global__ void k_sum(const float *__restrict__ v, int B, float *__restrict__ out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < B; i += 256) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void k_adam(float *__restrict__ master, const float *__restrict__ grad,
                       float *__restrict__ am, float *__restrict__ av, float lr, float bc1,
                       float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = grad[p];
  const float mm = 0.9f * am[p] + 0.1f * g;
  const float vv = 0.999f * av[p] + 0.001f * g * g;
  am[p] = mm;
  av[p] = vv;
  master[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// ----------------------------------------------------------------- host side
static int sel_get(Ctx *c, Selector **out) {
  if (!c->sel) {
    Selector *S = new (std::nothrow) Selector();
    if (!S) return set_err(c, PFSP_ENOMEM, "host allocation failed");
    bool ok = true;
    for (float **p : {&S->master, &S->wq, &S->grad, &S->am, &S->av})
      ok = ok && hipMalloc(p, kParams * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&S->to_inst, kOut * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(&S->bops, kBOps * sizeof(uint4)) == hipSuccess;
    ok = ok && hipMalloc(&S->loss, sizeof(float)) == hipSuccess;
    c->sel = S;
    if (!ok) {
      selector_free(c);
      return set_err(c, PFSP_ENOMEM, "selector allocation failed");
    }
  }
  *out = c->sel;
  return PFSP_OK;
}

void selector_free(Ctx *c) {
  Selector *S = c->sel;
  if (!S) return;
  void *bufs[] = {S->master, S->wq, S->grad, S->am, S->av, S->feat, S->scores, S->mask, S->h1,
                  S->h2, S->ds, S->dh1, S->dh2, S->rowloss, S->loss, S->to_inst, S->qops,
                  S->qbias, S->reopen, S->reopen_count, S->bops, S->part, S->bopsT,
                  S->nvalid};
  for (void *p : bufs) (void)hipFree(p);
  delete S;
  c->sel = nullptr;
}

// layout pair -> instance pair index table for the loaded instance
static int sel_tables(Ctx *c, Selector *S) {
  if (S->to_inst_m == c->m) return PFSP_OK;
  int h[kOut];
  for (int o = 0; o < kOut; ++o) h[o] = -1;
  const int m = c->m;
  for (int u = 0; u < m && u < kMMax; ++u)
    for (int v = u + 1; v < m && v < kMMax; ++v)
      h[u * (2 * kMMax - u - 1) / 2 + (v - u - 1)] = u * (2 * m - u - 1) / 2 + (v - u - 1);
  PFSP_HIP(c, hipMemcpy(S->to_inst, h, sizeof(h), hipMemcpyHostToDevice));
  S->to_inst_m = m;
  return PFSP_OK;
}

static int sel_rows(Ctx *c, Selector *S, size_t rows) {
  const int words = (c->P + 31) / 32;
  if (rows <= S->rows_cap && words <= S->mask_words) return PFSP_OK;
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  (void)hipFree(S->feat);
  (void)hipFree(S->scores);
  (void)hipFree(S->mask);
  (void)hipFree(S->reopen);
  (void)hipFree(S->reopen_count);
  S->feat = S->scores = nullptr;
  S->mask = nullptr;
  S->reopen = S->reopen_count = nullptr;
  const size_t cap = rows > S->rows_cap ? rows : S->rows_cap;
  S->rows_cap = 0;
  const int w = words > S->mask_words ? words : S->mask_words;
  if (hipMalloc(&S->feat, cap * kIn * 4) != hipSuccess ||
      hipMalloc(&S->scores, cap * kOut * 4) != hipSuccess ||
      hipMalloc(&S->mask, cap * (size_t)w * 4) != hipSuccess ||
      hipMalloc(&S->reopen, cap * 4) != hipSuccess ||
      hipMalloc(&S->reopen_count, 4) != hipSuccess)
    return set_err(c, PFSP_ENOMEM, "selector workspace allocation failed");
  S->rows_cap = cap;
  S->mask_words = w;
  return PFSP_OK;
}

static float instance_norm(const Ctx *c) {
  long long best = 1;
  for (int k = 0; k < c->m; ++k) {
    long long s = 0;
    for (int j = 0; j < c->n; ++j) s += c->p_host[(size_t)j * c->m + k];
    if (s > best) best = s;
  }
  return (float)best;
}

int selector_mode(const Ctx *c) {
  if (!c->sel) return 0;
  return c->sel->qloaded ? 2 : c->sel->loaded ? 1 : 0;
}

int learned_prepare(Ctx *c, int rows) {
  if (!c->sel || !(c->sel->loaded || c->sel->qloaded))
    return set_err(c, PFSP_EINVAL, "no selector parameters set");
  if (c->m > kMMax) return set_err(c, PFSP_ERANGE, "the learned selector covers m <= 20");
  if (c->learned_topk > (c->sel->qloaded ? kTopKMaxQ : kTopKMax))
    return set_err(c, PFSP_ERANGE,
                   "learned_topk must be <= 32 (float selector) or <= 64 (integer selector)");
  Selector *S = c->sel;
  int rc = sel_tables(c, S);
  if (rc) return rc;
  return sel_rows(c, S, rows > 0 ? rows : 1);
}

// Pair masks of the pool's rows (costs already in the workspace) into
// `mask`: the integer model when set (k <= 64), else the float one (k <= 32).
static void launch_infer(Ctx *c, const DevPool &pool, int k, uint32_t *mask, hipStream_t s) {
  Selector *S = c->sel;
  const DevInst I = c->inst();
  const int words = (c->P + 31) / 32;
  if (S->qloaded) {
    const float qs = S->sx / instance_norm(c), qd = S->sx / (float)c->n;
    const dim3 g((pool.count + kQRows * kQWaves - 1) / (kQRows * kQWaves)), b(64 * kQWaves);
    const size_t lds = kQWaves * kQWaveLds;
#define PFSP_IQ(K)                                                                         \
  hipLaunchKernelGGL(k_infer_q<K>, g, b, lds, s, I, pool, c->d_costs, qs, qd, S->qops,       \
                     S->qbias, S->M1, S->S1, S->M2, S->S2, S->to_inst, k, words, mask)
    if (k <= 16)
      PFSP_IQ(16);
    else if (k <= 32)
      PFSP_IQ(32);
    else
      PFSP_IQ(64);
#undef PFSP_IQ
  } else {
    const dim3 g((pool.count + kQRows * kQWaves - 1) / (kQRows * kQWaves)), b(64 * kQWaves);
    const size_t lds = kQWaves * kBWaveLds;
    if (k <= 16)
      hipLaunchKernelGGL((k_infer_bf<16, false>), g, b, lds, s, I, pool, c->d_costs,
                         (const float *)nullptr, instance_norm(c), S->bops, S->wq, S->to_inst, k,
                         words, mask, (float *)nullptr);
    else
      hipLaunchKernelGGL((k_infer_bf<32, false>), g, b, lds, s, I, pool, c->d_costs,
                         (const float *)nullptr, instance_norm(c), S->bops, S->wq, S->to_inst, k,
                         words, mask, (float *)nullptr);
  }
}

__global__ void k_zero_count(int *p) { *p = 0; }

// Appends to rows[] every pool row of the launch that has an unpruned child
// in either direction and more than one unscheduled job (with one, both
// children are leaves whose bound is the makespan under every kind).
__global__ void __launch_bounds__(256)
k_reopen(DevPool pool, int n, const uint8_t *__restrict__ out_prune, int *__restrict__ rows,
         int *__restrict__ count_out) {
  const int count = pool.count_dev ? *pool.count_dev : pool.count;
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= count) return;
  const int i = pool.index ? pool.index[it] : it;
  const int r = n - pool.d1[i] - pool.d2[i];
  if (r < 2) return;
  const uint8_t *pr = out_prune + (size_t)i * 2 * n;
  bool keep = false;
  for (int q = 0; q < r && !keep; ++q) keep = pr[q] == 0 || pr[n + q] == 0;
  if (keep) rows[atomicAdd(count_out, 1)] = i;
}

int launch_learned(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                   hipStream_t s) {
  int rc = learned_prepare(c, pool.count);
  if (rc) return rc;
  if (pool.count <= 0) return PFSP_OK;
  rc = ensure_costs(c, pool.count);
  if (rc) return rc;
  // parent costs (front, back, remaining) for the features
  rc = launch_costs(c, pool, s);
  if (rc) return rc;
  return launch_learned_ready(c, pool, ub, out_lb, out_prune, s);
}

// The learned bound once the costs of the pool are in the workspace.
int launch_learned_ready(Ctx *c, const DevPool &pool, int ub, int *out_lb, uint8_t *out_prune,
                         hipStream_t s) {
  int rc = learned_prepare(c, pool.count);
  if (rc) return rc;
  Selector *S = c->sel;
  if (pool.count <= 0) return PFSP_OK;
  const int words = (c->P + 31) / 32;
  const int k = (int)c->learned_topk;
  {
    KTimer kt(c, s, "k_infer");
    launch_infer(c, pool, k, S->mask, s);
  }
  PFSP_HIP(c, hipGetLastError());
  DevPool sp = pool;
  sp.mask = S->mask;
  sp.mask_words = words;
  // a top-k of at most 32 (16) pairs fills half (a quarter of) a wave: two
  // (four) parents per wave
  const int group = subset_group_for(c, k);
  rc = launch_bound_costs_ready(c, sp, PFSP_LB2_SUBSET, ub, out_lb, out_prune, s, group);
  if (rc || !c->learned_exact) return rc;
  // Exact mode: a parent that keeps a child under the subset bound is bounded
  // again with all pairs.  A parent whose children the subset bound prunes
  // entirely loses them under full LB2 as well (full >= subset), so every
  // prune flag, and the tree of a search, is that of PFSP_LB2_FULL.
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, S->reopen_count);
  {
    KTimer kt(c, s, "k_reopen");
    hipLaunchKernelGGL(k_reopen, dim3((pool.count + 255) / 256), dim3(256), 0, s, pool, c->n,
                       out_prune, S->reopen, S->reopen_count);
  }
  PFSP_HIP(c, hipGetLastError());
  DevPool fp = pool;
  fp.index = S->reopen;
  fp.count_dev = S->reopen_count;
  fp.mask = nullptr;
  fp.mask_words = 0;
  return launch_lb2_binned(c, fp, ub, out_lb, out_prune, s);
}

// The inference kernels fit the default LDS limit; kept as the hook called
// once per process with the bound kernels' attributes.
void init_selector_attributes() {}

// Device form of an integer-model blob (layout above).
static void q_pack(const int32_t *blob, std::vector<uint2> &ops, std::vector<int> &bias) {
  ops.assign(kQOps, make_uint2(0u, 0u));
  bias.assign(kQBiases, 0);
  auto pack8 = [](const int32_t *w) {  // eight int8 codes, little-endian
    uint32_t lo = 0, hi = 0;
    for (int i = 0; i < 4; ++i) lo |= (uint32_t)(uint8_t)(int8_t)w[i] << (8 * i);
    for (int i = 0; i < 4; ++i) hi |= (uint32_t)(uint8_t)(int8_t)w[4 + i] << (8 * i);
    return make_uint2(lo, hi);
  };
  for (int L = 0; L < 2; ++L) {
    const int32_t *W = blob + (L == 0 ? kQOffW1 : kQOffW2);
    const int32_t *B = blob + (L == 0 ? kQOffB1 : kQOffB2);
    for (int t = 0; t < kQT1; ++t)
      for (int lane = 0; lane < 64; ++lane) {
        const int c = lane & 15, g = lane >> 4, u = 4 * c + t;
        for (int ks = 0; ks < 2; ++ks)
          ops[(L == 0 ? kQOpB1 : kQOpB2) + (t * 2 + ks) * 64 + lane] =
              pack8(W + u * kIn + 32 * ks + 8 * g);
        bias[(L == 0 ? kQBias1 : kQBias2) + t * 64 + lane] = B[u];
      }
  }
  const int32_t *W3 = blob + kQOffW3, *B3 = blob + kQOffB3;
  for (int t = 0; t < kQT3; ++t)
    for (int lane = 0; lane < 64; ++lane) {
      const int c = lane & 15, g = lane >> 4, o = 16 * t + c;
      if (o >= kOut) continue;
      for (int ks = 0; ks < 2; ++ks)
        ops[kQOpB3 + (t * 2 + ks) * 64 + lane] = pack8(W3 + o * kHid + 32 * ks + 8 * g);
      bias[kQBias3 + t * 64 + lane] = B3[o];
    }
}

}  // namespace pfsp

using namespace pfsp;

extern "C" {

int pfsp_selector_set_quant(pfsp_ctx *h, const int32_t *blob, int64_t count) {
  if (!h) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  PFSP_HIP(c, hipSetDevice(c->device));
  Selector *S;
  int rc = sel_get(c, &S);
  if (rc) return rc;
  if (!blob) {  // back to the float model
    S->qloaded = 0;
    return PFSP_OK;
  }
  if (count != kQParams) return set_err(c, PFSP_EINVAL, "integer selector expects 20675 values");
  float sx;
  memcpy(&sx, blob, 4);
  if (!(sx > 0.f) || !isfinite(sx)) return set_err(c, PFSP_ERANGE, "feature scale must be > 0");
  for (int L = 0; L < 2; ++L) {
    const int M = blob[1 + 2 * L], Sh = blob[2 + 2 * L];
    if (M < 1 || M > 1023 || Sh < 1 || Sh > 30)
      return set_err(c, PFSP_ERANGE, "requantization needs M in [1, 1023] and S in [1, 30]");
  }
  for (int x = kQOffW1; x < kQParams; ++x) {
    const bool isb = (x >= kQOffB1 && x < kQOffW2) || (x >= kQOffB2 && x < kQOffW3) ||
                     x >= kQOffB3;
    const int v = blob[x];
    if (isb ? (v <= -(1 << 19) || v >= (1 << 19)) : (v < -127 || v > 127))
      return set_err(c, PFSP_ERANGE, "weights must lie in [-127, 127] and biases in (-2^19, 2^19)");
  }
  std::vector<uint2> ops;
  std::vector<int> bias;
  q_pack(blob, ops, bias);
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  if (!S->qops && hipMalloc(&S->qops, kQOps * sizeof(uint2)) != hipSuccess)
    return set_err(c, PFSP_ENOMEM, "selector allocation failed");
  if (!S->qbias && hipMalloc(&S->qbias, kQBiases * sizeof(int)) != hipSuccess)
    return set_err(c, PFSP_ENOMEM, "selector allocation failed");
  PFSP_HIP(c, hipMemcpy(S->qops, ops.data(), kQOps * sizeof(uint2), hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemcpy(S->qbias, bias.data(), kQBiases * sizeof(int), hipMemcpyHostToDevice));
  S->sx = sx;
  S->M1 = blob[1];
  S->S1 = blob[2];
  S->M2 = blob[3];
  S->S2 = blob[4];
  S->qloaded = 1;
  return PFSP_OK;
}

int pfsp_selector_infer(pfsp_ctx *h, const pfsp_pool *pool, int32_t k, uint32_t *mask_out) {
  if (!h || !pool || (pool->count > 0 && !mask_out)) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (pool->count < 0 || pool->n != c->n) return set_err(c, PFSP_EINVAL, "bad pool");
  if (k < 1 || k > kTopKMaxQ) return set_err(c, PFSP_ERANGE, "k must be in [1, 64]");
  if (c->m > kMMax || c->m < 2) return set_err(c, PFSP_ERANGE, "selection needs 2 <= m <= 20");
  PFSP_HIP(c, hipSetDevice(c->device));
  const int64_t saved = c->learned_topk;
  c->learned_topk = k;
  int rc = learned_prepare(c, pool->count);
  c->learned_topk = saved;
  if (rc) return rc;
  if (pool->count == 0) return PFSP_OK;
  DevPool dp{};
  dp.count = pool->count;
  dp.n = pool->n;
  dp.perm = pool->perm;
  dp.d1 = pool->d1;
  dp.d2 = pool->d2;
  rc = ensure_costs(c, pool->count);
  if (rc) return rc;
  rc = launch_costs(c, dp, c->stream);
  if (rc) return rc;
  launch_infer(c, dp, k, mask_out, c->stream);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int pfsp_selector_set(pfsp_ctx *h, const float *params, int64_t count) {
  if (!h || !params) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (count != kParams) return set_err(c, PFSP_EINVAL, "selector expects 20670 parameters");
  PFSP_HIP(c, hipSetDevice(c->device));
  Selector *S;
  int rc = sel_get(c, &S);
  if (rc) return rc;
  PFSP_HIP(c, hipMemcpy(S->master, params, kParams * 4, hipMemcpyHostToDevice));
  PFSP_HIP(c, hipMemset(S->am, 0, kParams * 4));
  PFSP_HIP(c, hipMemset(S->av, 0, kParams * 4));
  S->step = 0;
  hipLaunchKernelGGL(k_round_weights, dim3((kParams + 255) / 256), dim3(256), 0, c->stream,
                     S->master, S->wq);
  hipLaunchKernelGGL(k_pack_bf16, dim3((kBOps + 255) / 256), dim3(256), 0, c->stream, S->wq,
                     S->bops);
  PFSP_HIP(c, hipGetLastError());
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  S->loaded = 1;
  return PFSP_OK;
}

int pfsp_selector_get(pfsp_ctx *h, float *params, int64_t count) {
  if (!h || !params) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (!c->sel || !c->sel->loaded) return set_err(c, PFSP_EINVAL, "no selector parameters set");
  if (count != kParams) return set_err(c, PFSP_EINVAL, "selector has 20670 parameters");
  PFSP_HIP(c, hipSetDevice(c->device));
  PFSP_HIP(c, hipStreamSynchronize(c->stream));
  PFSP_HIP(c, hipMemcpy(params, c->sel->master, kParams * 4, hipMemcpyDeviceToHost));
  return PFSP_OK;
}

int pfsp_selector_features(pfsp_ctx *h, const pfsp_pool *pool, float *feat_out) {
  if (!h || !pool || !feat_out) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (pool->count < 0 || pool->n != c->n) return set_err(c, PFSP_EINVAL, "bad pool");
  if (pool->count == 0) return PFSP_OK;
  PFSP_HIP(c, hipSetDevice(c->device));
  DevPool dp{};
  dp.count = pool->count;
  dp.n = pool->n;
  dp.perm = pool->perm;
  dp.d1 = pool->d1;
  dp.d2 = pool->d2;
  int rc = ensure_costs(c, pool->count);
  if (rc) return rc;
  rc = launch_costs(c, dp, c->stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_features, dim3((pool->count + 255) / 256), dim3(256), 0, c->stream,
                     c->inst(), dp, c->d_costs, instance_norm(c), feat_out);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int pfsp_selector_forward(pfsp_ctx *h, const float *x, int32_t rows, float *scores_out) {
  if (!h || (rows > 0 && (!x || !scores_out)) || rows < 0) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  int rc = learned_prepare(c, rows);
  if (rc) return rc;
  if (!c->sel->loaded) return set_err(c, PFSP_EINVAL, "no float selector parameters set");
  if (rows == 0) return PFSP_OK;
  // the float form's arithmetic of the learned bound (bf16 MFMA, hi/lo activations)
  DevPool pool;
  pool.count = rows;
  pool.n = c->n;
  pool.perm = pool.d1 = pool.d2 = nullptr;
  pool.mask = nullptr;
  pool.mask_words = 0;
  pool.dir = nullptr;
  pool.argpair = nullptr;
  const dim3 g((rows + kQRows * kQWaves - 1) / (kQRows * kQWaves)), b(64 * kQWaves);
  hipLaunchKernelGGL((k_infer_bf<16, true>), g, b, kQWaves * kBWaveLds, c->stream, c->inst(),
                     pool, (const int *)nullptr, x, 1.f, c->sel->bops, c->sel->wq,
                     c->sel->to_inst, 1, 0, (uint32_t *)nullptr, scores_out);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int pfsp_selector_select(pfsp_ctx *h, const float *scores, int32_t rows, int32_t k,
                         uint32_t *mask_out) {
  if (!h || rows < 0 || (rows > 0 && (!scores || !mask_out))) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (k < 1 || k > kTopKMax) return set_err(c, PFSP_ERANGE, "k must be in [1, 32]");
  if (c->m > kMMax || c->m < 2) return set_err(c, PFSP_ERANGE, "selection needs 2 <= m <= 20");
  Selector *S;
  int rc = sel_get(c, &S);
  if (rc) return rc;
  rc = sel_tables(c, S);
  if (rc) return rc;
  if (rows == 0) return PFSP_OK;
  hipLaunchKernelGGL(k_select, dim3((rows + 255) / 256), dim3(256), 0, c->stream, scores, rows,
                     (const int *)nullptr, (int)k, S->to_inst, (c->P + 31) / 32, mask_out);
  PFSP_HIP(c, hipGetLastError());
  return PFSP_OK;
}

int pfsp_selector_targets(pfsp_ctx *h, const pfsp_pool *pool, const int16_t *argpair,
                          float *target_out) {
  if (!h || !pool || !argpair || !target_out) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  if (c->m > kMMax || c->m < 2) return set_err(c, PFSP_ERANGE, "targets need 2 <= m <= 20");
  if (pool->count < 0 || pool->n != c->n) return set_err(c, PFSP_EINVAL, "bad pool");
  if (pool->count == 0) return PFSP_OK;
  Selector *S;
  int rc = sel_get(c, &S);
  if (rc) return rc;
  // instance pair -> layout pair
  int inst_to20[kOut];
  const int m = c->m;
  for (int u = 0; u < m; ++u)
    for (int v = u + 1; v < m; ++v)
      inst_to20[u * (2 * m - u - 1) / 2 + (v - u - 1)] = u * (2 * kMMax - u - 1) / 2 + (v - u - 1);
  int *d_map = nullptr;
  PFSP_HIP(c, hipMalloc(&d_map, sizeof(inst_to20)));
  PFSP_HIP(c, hipMemcpyAsync(d_map, inst_to20, sizeof(inst_to20), hipMemcpyHostToDevice,
                             c->stream));
  DevPool dp{};
  dp.count = pool->count;
  dp.n = pool->n;
  dp.perm = pool->perm;
  dp.d1 = pool->d1;
  dp.d2 = pool->d2;
  hipLaunchKernelGGL(k_targets, dim3((pool->count + 255) / 256), dim3(256), 0, c->stream,
                     c->inst(), dp, argpair, d_map, target_out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d_map);
  if (e != hipSuccess) return hip_err(c, e, "k_targets");
  return PFSP_OK;
}

int pfsp_selector_train_step(pfsp_ctx *h, const float *x, const float *target, int32_t rows,
                             float lr, float *loss_out, float *grad_out) {
  if (!h || !x || !target || rows <= 0) return PFSP_EINVAL;
  Ctx *c = &h->impl;
  if (c->n == 0) return set_err(c, PFSP_ENOINST, "no instance loaded");
  int rc = learned_prepare(c, 1);
  if (rc) return rc;
  Selector *S = c->sel;
  if (!S->loaded) return set_err(c, PFSP_EINVAL, "no float selector parameters set");
  PFSP_HIP(c, hipSetDevice(c->device));
  if ((size_t)rows > S->train_cap) {
    PFSP_HIP(c, hipStreamSynchronize(c->stream));
    for (float **p : {&S->h1, &S->h2, &S->ds, &S->dh1, &S->dh2, &S->rowloss, &S->part}) {
      (void)hipFree(*p);
      *p = nullptr;
    }
    const size_t splits = ((size_t)rows + kTRowsPerSplit - 1) / kTRowsPerSplit;
    bool ok = hipMalloc(&S->h1, (size_t)rows * kHid * 4) == hipSuccess &&
              hipMalloc(&S->h2, (size_t)rows * kHid * 4) == hipSuccess &&
              hipMalloc(&S->dh1, (size_t)rows * kHid * 4) == hipSuccess &&
              hipMalloc(&S->dh2, (size_t)rows * kHid * 4) == hipSuccess &&
              hipMalloc(&S->ds, (size_t)rows * kOut * 4) == hipSuccess &&
              hipMalloc(&S->rowloss, (size_t)rows * 4) == hipSuccess &&
              hipMalloc(&S->part, splits * kParams * 4) == hipSuccess;
    if (ok && !S->bopsT) ok = hipMalloc(&S->bopsT, kTOps * sizeof(uint4)) == hipSuccess;
    if (ok && !S->nvalid) ok = hipMalloc(&S->nvalid, sizeof(int)) == hipSuccess;
    if (!ok) return set_err(c, PFSP_ENOMEM, "training workspace allocation failed");
    S->train_cap = rows;
  }
  // the mean runs over the rows with a non-empty target (counted on the device)
  hipStream_t s = c->stream;
  const int splits = (rows + kTRowsPerSplit - 1) / kTRowsPerSplit;
  int *nvalid_dev = S->nvalid;
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, nvalid_dev);
  hipLaunchKernelGGL(k_pack_bf16t, dim3((kTOps + 255) / 256), dim3(256), 0, s, S->wq, S->bopsT);
  hipLaunchKernelGGL(k_train_fb, dim3((rows + kQRows * kQWaves - 1) / (kQRows * kQWaves)),
                     dim3(64 * kQWaves), kQWaves * kTWaveLds, s, x, target, (int)rows,
                     nvalid_dev, S->bops, S->bopsT, S->wq, S->to_inst, S->h1, S->h2, S->ds,
                     S->dh1, S->dh2, S->rowloss);
  hipLaunchKernelGGL(k_train_wgrad, dim3((kTTiles * splits + 3) / 4), dim3(256), 0, s, x, S->h1,
                     S->h2, S->ds, S->dh1, S->dh2, (int)rows, S->part);
  hipLaunchKernelGGL(k_train_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, S->part,
                     splits, nvalid_dev, S->grad);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, S->rowloss, (int)rows, S->loss);
  PFSP_HIP(c, hipGetLastError());
  if (grad_out)
    PFSP_HIP(c, hipMemcpyAsync(grad_out, S->grad, kParams * 4, hipMemcpyDeviceToDevice, s));
  if (lr > 0.f) {
    S->step += 1;
    const float bc1 = 1.f - powf(0.9f, (float)S->step);
    const float bc2 = 1.f - powf(0.999f, (float)S->step);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, S->master, S->grad,
                       S->am, S->av, lr, bc1, bc2);
    hipLaunchKernelGGL(k_round_weights, dim3((kParams + 255) / 256), dim3(256), 0, s, S->master,
                       S->wq);
    hipLaunchKernelGGL(k_pack_bf16, dim3((kBOps + 255) / 256), dim3(256), 0, s, S->wq, S->bops);
    PFSP_HIP(c, hipGetLastError());
  }
  float l = 0.f;
  int nvalid = 0;
  PFSP_HIP(c, hipMemcpyAsync(&l, S->loss, 4, hipMemcpyDeviceToHost, s));
  PFSP_HIP(c, hipMemcpyAsync(&nvalid, nvalid_dev, 4, hipMemcpyDeviceToHost, s));
  PFSP_HIP(c, hipStreamSynchronize(s));
  if (loss_out) *loss_out = l / (float)std::max(1, nvalid);
  return PFSP_OK;
}

}  // extern "C"
