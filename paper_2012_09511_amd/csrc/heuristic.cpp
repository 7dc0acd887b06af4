// Incumbent improvement beside the device search (host threads).
//
// The time a branch-and-bound needs to prove optimality depends strongly on
// how early it holds a good incumbent (Section 1; the paper runs heuristic
// searches beside its explorers, Section 4.2).  While pfsp_search runs, each
// thread here runs an iterated greedy local search on the instance (Ruiz and
// Stuetzle's scheme: remove a few jobs at random, reinsert each at its best
// position, improve by best-position reinsertion of every job, accept a worse
// schedule with a temperature-dependent probability), started from NEH and
// from complete schedules that the search loop builds from open nodes of the
// device stack.  A strictly better makespan is published; the search loop
// lowers the device incumbent to it.  Insertions are evaluated for all
// positions at once with heads and tails of the partial sequence (Taillard's
// acceleration), O(k m) per job for a sequence of k jobs.
#include "heuristic.h"

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <random>

namespace pfsp {

namespace {

// Completion-time heads e[i][k] of the first i jobs of seq and tails q[i][k]
// of the jobs from position i on (machines in reverse), for i = 0 .. len.
struct InsertTables {
  int m = 0;
  std::vector<int64_t> e, q;
  void size(int len, int mm) {
    m = mm;
    e.assign((size_t)(len + 1) * m, 0);
    q.assign((size_t)(len + 2) * m, 0);
  }
};

int64_t makespan(const int *p, int m, const std::vector<int> &seq, std::vector<int64_t> &row) {
  std::fill(row.begin(), row.end(), 0);
  for (int j : seq) {
    const int *pj = p + (size_t)j * m;
    int64_t prev = 0;
    for (int k = 0; k < m; ++k) {
      prev = std::max(prev, row[k]) + pj[k];
      row[k] = prev;
    }
  }
  return seq.empty() ? 0 : row[m - 1];
}

// Best position (first among equals) for inserting job j into seq, and the
// makespan there.
std::pair<int, int64_t> best_insertion(const int *p, int m, const std::vector<int> &seq, int j,
                                       InsertTables &T) {
  const int len = (int)seq.size();
  T.size(len, m);
  int64_t *e = T.e.data(), *q = T.q.data();
  for (int i = 1; i <= len; ++i) {
    const int *pj = p + (size_t)seq[i - 1] * m;
    int64_t prev = 0;
    for (int k = 0; k < m; ++k) {
      prev = std::max(prev, e[(size_t)(i - 1) * m + k]) + pj[k];
      e[(size_t)i * m + k] = prev;
    }
  }
  for (int i = len - 1; i >= 0; --i) {
    const int *pj = p + (size_t)seq[i] * m;
    int64_t next = 0;
    for (int k = m - 1; k >= 0; --k) {
      next = std::max(next, q[(size_t)(i + 1) * m + k]) + pj[k];
      q[(size_t)i * m + k] = next;
    }
  }
  const int *pj = p + (size_t)j * m;
  int best_pos = 0;
  int64_t best = INT64_MAX;
  for (int i = 0; i <= len; ++i) {
    int64_t prev = 0, c = 0;
    for (int k = 0; k < m; ++k) {
      prev = std::max(prev, e[(size_t)i * m + k]) + pj[k];
      c = std::max(c, prev + q[(size_t)i * m + k]);
    }
    if (c < best) {
      best = c;
      best_pos = i;
    }
  }
  return {best_pos, best};
}

// Reinserts every job at its best position while that improves the makespan.
int64_t local_search(const int *p, int m, std::vector<int> &seq, int64_t c, std::mt19937 &rng,
                     InsertTables &T, const std::atomic<int> &stop) {
  bool improved = true;
  std::vector<int> order(seq);
  while (improved && !stop.load(std::memory_order_relaxed)) {
    improved = false;
    std::shuffle(order.begin(), order.end(), rng);
    for (int j : order) {
      auto it = std::find(seq.begin(), seq.end(), j);
      seq.erase(it);
      const auto bi = best_insertion(p, m, seq, j, T);
      seq.insert(seq.begin() + bi.first, j);
      if (bi.second < c) {
        c = bi.second;
        improved = true;
      }
    }
  }
  return c;
}

}  // namespace

void Heuristic::publish(const std::vector<int> &seq, int64_t c) {
  if (c >= best.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lock(mu);
  if (c < best.load(std::memory_order_relaxed)) {
    best_perm = seq;
    best.store((int)c, std::memory_order_relaxed);
  }
}

void Heuristic::offer(const std::vector<int> &seq) {
  std::lock_guard<std::mutex> lock(mu);
  if (seeds.size() < 64) seeds.push_back(seq);
}

void Heuristic::run(int tid) {
  std::mt19937 rng((uint32_t)(seed * 7919 + tid * 104729 + 1));
  std::vector<int64_t> row(m);
  InsertTables T;
  int64_t total = 0;
  for (int x = 0; x < n * m; ++x) total += p[x];
  const double temp = 0.4 * (double)total / (10.0 * n * m);
  const int d = std::min(4, std::max(1, n / 5));
  std::vector<int> cur = start;
  int64_t cc = makespan(p.data(), m, cur, row);
  cc = local_search(p.data(), m, cur, cc, rng, T, stop);
  publish(cur, cc);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  while (!stop.load(std::memory_order_relaxed)) {
    {  // an offered schedule from the search restarts this thread now and then
      std::lock_guard<std::mutex> lock(mu);
      if (!seeds.empty() && U(rng) < 0.25) {
        cur = seeds.back();
        seeds.pop_back();
        cc = makespan(p.data(), m, cur, row);
      }
    }
    std::vector<int> s = cur, removed;
    for (int r = 0; r < d; ++r) {
      const int at = (int)(rng() % s.size());
      removed.push_back(s[at]);
      s.erase(s.begin() + at);
    }
    for (int j : removed) {
      const auto bi = best_insertion(p.data(), m, s, j, T);
      s.insert(s.begin() + bi.first, j);
    }
    int64_t c = makespan(p.data(), m, s, row);
    c = local_search(p.data(), m, s, c, rng, T, stop);
    if (c < cc) {
      cur = s;
      cc = c;
      publish(cur, cc);
    } else if (U(rng) < std::exp(-(double)(c - cc) / temp)) {
      cur = s;
      cc = c;
    }
    iterations.fetch_add(1, std::memory_order_relaxed);
  }
}

void Heuristic::launch(int threads, const std::vector<int> &neh, int neh_cmax) {
  start = neh;
  best.store(neh_cmax);
  best_perm = neh;
  stop.store(0);
  for (int t = 0; t < threads; ++t) pool.emplace_back([this, t] { run(t); });
}

void Heuristic::finish() {
  stop.store(1);
  for (auto &t : pool) t.join();
  pool.clear();
}

std::vector<int> complete_node(const int *p, int n, int m, const uint8_t *perm, int d1, int d2) {
  // sigma1, then the unscheduled jobs inserted one by one at their best
  // position among themselves (their list order), then sigma2
  std::vector<int> mid;
  const std::vector<int> tail(perm + (n - d2), perm + n);
  std::vector<int64_t> row(m);
  for (int x = d1; x < n - d2; ++x) {
    const int j = perm[x];
    int best_pos = 0;
    int64_t best = INT64_MAX;
    for (int i = 0; i <= (int)mid.size(); ++i) {
      std::vector<int> s(perm, perm + d1);
      s.insert(s.end(), mid.begin(), mid.begin() + i);
      s.push_back(j);
      s.insert(s.end(), mid.begin() + i, mid.end());
      s.insert(s.end(), tail.begin(), tail.end());
      const int64_t c = makespan(p, m, s, row);
      if (c < best) {
        best = c;
        best_pos = i;
      }
    }
    mid.insert(mid.begin() + best_pos, j);
  }
  std::vector<int> s(perm, perm + d1);
  s.insert(s.end(), mid.begin(), mid.end());
  s.insert(s.end(), perm + (n - d2), perm + n);
  return s;
}

int64_t sequence_makespan(const int *p, int m, const std::vector<int> &seq) {
  std::vector<int64_t> row(m);
  return makespan(p, m, seq, row);
}

}  // namespace pfsp
