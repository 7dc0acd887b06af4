// Host-side incumbent improvement (heuristic.cpp).
#pragma once

#include <stdint.h>

#include <atomic>
#include <mutex>
#include <thread>
#include <vector>

namespace pfsp {

// Iterated greedy threads over one instance.  best / best_perm hold the
// best makespan seen (starting from the NEH schedule given to launch).
struct Heuristic {
  int n = 0, m = 0;
  std::vector<int> p;  // [n][m]
  uint64_t seed = 0;
  std::atomic<int> best{0};
  std::atomic<int> stop{0};
  std::atomic<long long> iterations{0};
  std::mutex mu;
  std::vector<int> best_perm, start;
  std::vector<std::vector<int>> seeds;  // complete schedules offered by the search
  std::vector<std::thread> pool;
  void launch(int threads, const std::vector<int> &neh, int neh_cmax);
  void finish();
  void offer(const std::vector<int> &seq);
  void publish(const std::vector<int> &seq, int64_t c);
  void run(int tid);
};

// A complete schedule from a node: sigma1, the unscheduled jobs inserted one
// by one (list order) at their best place among those already inserted, sigma2.
std::vector<int> complete_node(const int *p, int n, int m, const uint8_t *perm, int d1, int d2);
int64_t sequence_makespan(const int *p, int m, const std::vector<int> &seq);

}  // namespace pfsp
