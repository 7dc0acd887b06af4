// Instance staging on the device (run once per loaded instance).
//
// For every machine pair u < v the two-machine relaxation of Section 2.4
// (the bound of Lageweg et al. that the paper names LB2) sees job j as
// a_j = p[j][u] on the first machine, b_j = p[j][v] on the second, and a time
// lag l_j = sum of p[j][q] for u < q < v spent on the machines in between,
// treated as non-bottleneck.  Johnson's rule extended to lags orders the jobs:
// jobs with a_j <= b_j first by ascending a_j + l_j, then the others by
// descending b_j + l_j.  The order of all n jobs is computed once here; the
// restriction of a Johnson order to any subset of jobs is again a Johnson
// order of that subset, so the bound kernels reuse it for every node (the
// "pre-sorted" schedules of Section 2.4).  Equal keys are kept in job order;
// the two-machine value does not depend on how ties are ordered.
#include "internal.h"

namespace pfsp {

__device__ __forceinline__ bool johnson_less(int ax, int bx, int lx, int x, int ay, int by,
                                             int ly, int y) {
  const int gx = ax <= bx ? 0 : 1, gy = ay <= by ? 0 : 1;
  if (gx != gy) return gx < gy;
  const int kx = gx == 0 ? ax + lx : -(bx + lx);
  const int ky = gy == 0 ? ay + ly : -(by + ly);
  if (kx != ky) return kx < ky;
  return x < y;
}

__global__ void k_stage(int n, int m, int P, const int *__restrict__ p, int *__restrict__ T,
                        uint8_t *__restrict__ ord, uint2 *__restrict__ ent,
                        uint4 *__restrict__ entw, uint8_t *__restrict__ pu,
                        uint8_t *__restrict__ pv, int narrow) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) {
    int s = 0;
    for (int j = 0; j < n; ++j) s += p[j * m + t];
    T[t] = s;
  }
  if (t >= P) return;
  // pair index -> (u, v), lexicographic
  int u = 0, rem = t;
  while (rem >= m - 1 - u) {
    rem -= m - 1 - u;
    ++u;
  }
  const int v = u + 1 + rem;
  pu[t] = (uint8_t)u;
  pv[t] = (uint8_t)v;
  uint8_t *o = ord + (size_t)t * n;
  for (int j = 0; j < n; ++j) o[j] = (uint8_t)j;
  auto lag = [&](int j) {
    int s = 0;
    for (int q = u + 1; q < v; ++q) s += p[j * m + q];
    return s;
  };
  for (int i = 1; i < n; ++i) {
    const int x = o[i];
    const int ax = p[x * m + u], bx = p[x * m + v], lx = lag(x);
    int k = i - 1;
    while (k >= 0) {
      const int y = o[k];
      if (!johnson_less(ax, bx, lx, x, p[y * m + u], p[y * m + v], lag(y), y)) break;
      o[k + 1] = o[k];
      --k;
    }
    o[k + 1] = (uint8_t)x;
  }
  for (int i = 0; i < n; ++i) {
    const int k = o[i];
    const unsigned a = (unsigned)p[k * m + u], b = (unsigned)p[k * m + v];
    const unsigned l = (unsigned)lag(k);
    if (narrow)
      ent[(size_t)i * P + t] = make_uint2(a | (b << 16), l | ((unsigned)k << 24));
    else
      entw[(size_t)i * P + t] = make_uint4(a, b, l, (unsigned)k);
  }
}

int stage_tables(Ctx *c, hipStream_t s, int n, int m, const int *d_p, int *d_T, uint2 *d_ent,
                 uint4 *d_entw, uint8_t *d_pu, uint8_t *d_pv, int narrow) {
  const int P = m * (m - 1) / 2;
  uint8_t *d_ord = nullptr;
  const int threads = 64;
  const int work = P > m ? P : m;
  PFSP_HIP(c, hipMalloc(&d_ord, (size_t)(P > 0 ? P : 1) * n));
  hipLaunchKernelGGL(k_stage, dim3((work + threads - 1) / threads), dim3(threads), 0, s, n, m, P,
                     d_p, d_T, d_ord, d_ent, d_entw, d_pu, d_pv, narrow);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_ord);
  if (e != hipSuccess) return hip_err(c, e, "k_stage");
  return PFSP_OK;
}

__global__ void k_stage_q(int n, int P, int Ppad, const uint2 *__restrict__ ent,
                          uint2 *__restrict__ entq) {
  const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (x >= (long long)Ppad * n) return;
  const int pass = (int)(x / (64LL * n));
  const int rem = (int)(x - (long long)pass * 64 * n);
  const int i = rem >> 6, pi = pass * 64 + (rem & 63);
  const uint2 s = ent[(size_t)i * P + (pi < P ? pi : 0)];
  const unsigned a = s.x & 0xffffu, b = s.x >> 16, l = s.y & 0xffffffu, k = s.y >> 24;
  entq[x] = make_uint2(((b - a) & 0xffffu) | (k << 24), k | ((a + l) << 16));
}

int stage_quick(Ctx *c, hipStream_t s, int n, int m, const uint2 *d_ent, uint2 **d_entq) {
  const int P = m * (m - 1) / 2;
  *d_entq = nullptr;
  if (P == 0) return PFSP_OK;
  const int Ppad = (P + 63) / 64 * 64;
  PFSP_HIP(c, hipMalloc(d_entq, (size_t)Ppad * n * 8));
  const long long tot = (long long)Ppad * n;
  hipLaunchKernelGGL(k_stage_q, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, P, Ppad,
                     d_ent, *d_entq);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "k_stage_q");
  return PFSP_OK;
}

int stage_instance(Ctx *c) {
  return stage_tables(c, c->stream, c->n, c->m, c->d_p, c->d_T, c->d_ent, c->d_entw, c->d_pu,
                      c->d_pv, c->narrow);
}

}  // namespace pfsp
