/* Plain CPU oracle for the permutation flow-shop bounds and branch-and-bound
 * of Gmys (2020), "Solving large permutation flow-shop scheduling problems on
 * GPU-accelerated supercomputers".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code with the HIP library.
 *
 * Conventions: p is row-major p[j*m + k] (job j, machine k), int32 >= 0.
 * A node is (perm[n], d1, d2): sigma1 = perm[0, d1), unscheduled U =
 * perm[d1, n - d2) in list order, sigma2 = perm[n - d2, n).  All times are
 * computed in int64.  Pair index of machines u < v is lexicographic:
 * idx(u, v) = u*(2m - u - 1)/2 + (v - u - 1).
 */
#ifndef PFSP_ORACLE_H
#define PFSP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_LB1 1
#define OR_LB2_FULL 2
#define OR_LB2_SUBSET 3

int64_t or_makespan(int m, const int32_t *p, const uint8_t *seq, int len);
void or_front(int m, const int32_t *p, const uint8_t *seq, int len, int64_t *C);
void or_back(int m, const int32_t *p, const uint8_t *seq, int len, int64_t *Cb);
int64_t or_lb1_parts(int m, const int64_t *C1, const int64_t *R, const int64_t *C2);
int64_t or_pair_value(int m, const int32_t *p, const uint8_t *jobs, int nj, int u, int v,
                      int64_t hu, int64_t hv, int64_t tu, int64_t tv);
int64_t or_pair_value_bruteforce(int m, const int32_t *p, const uint8_t *jobs, int nj,
                                 int u, int v, int64_t hu, int64_t hv, int64_t tu,
                                 int64_t tv);
void or_johnson_lag_order(int m, const int32_t *p, uint8_t *jobs, int nj, int u, int v);
int64_t or_node_bound(int n, int m, const int32_t *p, const uint8_t *perm, int d1, int d2,
                      int kind, const uint32_t *pair_mask, int32_t *argpair);
int64_t or_best_completion(int n, int m, const int32_t *p, const uint8_t *perm, int d1,
                           int d2, uint8_t *best_perm);
int or_minmin(int r, const int64_t *lbf, const int64_t *lbb);
int or_bound_children(int n, int m, const int32_t *p, int count, const uint8_t *perm,
                      const uint8_t *d1, const uint8_t *d2, int kind, int64_t ub,
                      const uint32_t *pair_mask, int mask_words, int32_t *out_lb,
                      uint8_t *out_prune, uint8_t *out_dir, int32_t *out_argpair,
                      int threads);
int or_search(int n, int m, const int32_t *p, int64_t ub0, int kind, int64_t budget,
              int64_t *best_cmax, uint8_t *best_perm, int64_t *nodes,
              int64_t *children, int *found, int *proven);
int or_search_ex(int n, int m, const int32_t *p, int64_t ub0, int kind,
                 const uint32_t *pair_mask, int64_t budget, int threads, int lb1_r,
                 int64_t *best_cmax, uint8_t *best_perm, int64_t *nodes, int64_t *children,
                 int *found, int *proven);
int64_t or_bruteforce(int n, int m, const int32_t *p, uint8_t *best_perm);
int64_t or_neh(int n, int m, const int32_t *p, uint8_t *perm_out);

#ifdef __cplusplus
}
#endif
#endif
