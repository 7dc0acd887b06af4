// Nawaz-Enscore-Ham heuristic for the initial incumbent (host side; it is
// not part of the bounding path and runs once per search).
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pfsp.h"

namespace pfsp {

// Makespan of a job sequence by Eq. (1) of Section 2.1, rolling one row of
// completion times over the machines.
static int64_t seq_makespan(int m, const int *p, const int *seq, int len, std::vector<int64_t> &row) {
  std::fill(row.begin(), row.end(), 0);
  for (int i = 0; i < len; ++i) {
    const int *pj = p + (size_t)seq[i] * m;
    int64_t prev = 0;
    for (int k = 0; k < m; ++k) {
      prev = std::max(prev, row[k]) + pj[k];
      row[k] = prev;
    }
  }
  return len ? row[m - 1] : 0;
}

int neh_host(int n, int m, const int *p, int *perm_out, int *cmax_out) {
  std::vector<int> order(n), seq, trial;
  std::vector<int64_t> total(n, 0), row(m);
  for (int j = 0; j < n; ++j) {
    order[j] = j;
    for (int k = 0; k < m; ++k) total[j] += p[(size_t)j * m + k];
  }
  // decreasing total time, lower id first among equals
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return total[x] > total[y]; });
  seq.reserve(n);
  for (int i = 0; i < n; ++i) {
    int best_pos = 0;
    int64_t best = INT64_MAX;
    for (int pos = 0; pos <= (int)seq.size(); ++pos) {
      trial.assign(seq.begin(), seq.begin() + pos);
      trial.push_back(order[i]);
      trial.insert(trial.end(), seq.begin() + pos, seq.end());
      const int64_t c = seq_makespan(m, p, trial.data(), (int)trial.size(), row);
      if (c < best) {
        best = c;
        best_pos = pos;
      }
    }
    seq.insert(seq.begin() + best_pos, order[i]);
  }
  for (int j = 0; j < n; ++j) perm_out[j] = seq[j];
  *cmax_out = (int)seq_makespan(m, p, seq.data(), n, row);
  return PFSP_OK;
}

}  // namespace pfsp
