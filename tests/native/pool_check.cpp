// Host-pool check: loops of many sizes from two threads at once; every item
// must be visited exactly once (callers that find the pool busy run alone).
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "host_pool.hpp"

int main() {
  std::atomic<long> bad{0}, calls{0};
  auto body = [&](int seed) {
    for (int it = 0; it < 2000; ++it) {
      const int n = (it * 7919 + seed * 104729) % 6000;
      std::vector<std::atomic<int>> hit(n);
      gsmat::host_parallel_for(n, 16, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) hit[i]++;
      });
      for (int i = 0; i < n; ++i)
        if (hit[i] != 1) ++bad;
      ++calls;
    }
  };
  std::thread a(body, 1), b(body, 2);
  body(3);
  a.join();
  b.join();
  std::printf("calls %ld bad %ld\n", calls.load(), bad.load());
  return bad.load() == 0 ? 0 : 1;
}
