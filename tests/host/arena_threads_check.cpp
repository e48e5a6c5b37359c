// Host test of the pieces the solver's lanes share from several threads (no GPU), built
// with the thread sanitizer: the arena (allocations and releases from four threads at
// once, each checking its own blocks for alignment, bounds and overlap with the other
// threads' live blocks through a shared registry) and the host trace table (phases
// timed from every thread). The sanitizer reports any unsynchronised access.
#include <stdint.h>
#include <stdio.h>

#include <atomic>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2609_02394_amd/csrc/host_util.h"

int main() {
  const size_t size = (size_t)256 << 20;
  std::vector<char> fake(16);  // the arena only does arithmetic on its base pointer
  char* base = fake.data();
  rmc::Arena A;
  A.init(base, size);
  std::mutex reg_mu;
  std::map<size_t, size_t> live;  // offset -> bytes, every thread's live blocks
  std::atomic<int> errors{0};
  auto worker = [&](int t) {
    std::mt19937_64 rng(2609 + t);
    std::vector<std::pair<char*, size_t>> mine;
    for (int step = 0; step < 20000; ++step) {
      if (mine.empty() || rng() % 100 < 55) {
        const size_t b = 1 + rng() % 200000;
        char* p;
        try {
          p = static_cast<char*>(A.alloc(b));
        } catch (const rmc::Error& e) {
          if (e.code != RMC_ERR_OOM) errors++;
          continue;
        }
        const size_t off = (size_t)(p - base), need = (b + 255) / 256 * 256;
        if (off % 256 != 0 || off + need > size) errors++;
        {
          std::lock_guard<std::mutex> lk(reg_mu);
          auto nx = live.lower_bound(off);
          if (nx != live.end() && nx->first < off + need) errors++;
          if (nx != live.begin() && std::prev(nx)->first + std::prev(nx)->second > off) errors++;
          live[off] = need;
        }
        mine.push_back({p, need});
      } else {
        const size_t i = rng() % mine.size();
        {
          std::lock_guard<std::mutex> lk(reg_mu);
          live.erase((size_t)(mine[i].first - base));
        }
        A.release(mine[i].first);
        mine.erase(mine.begin() + (long)i);
      }
      if (step % 64 == 0) rmc::host_trace_add(t % 2 ? "lane.odd" : "lane.even", 0.001);
    }
    for (auto& m : mine) {
      {
        std::lock_guard<std::mutex> lk(reg_mu);
        live.erase((size_t)(m.first - base));
      }
      A.release(m.first);
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) th.emplace_back(worker, t);
  for (auto& x : th) x.join();
  if (errors.load() != 0 || A.in_use() != 0 || A.free_blocks() != 1 || !live.empty()) {
    fprintf(stderr, "arena_threads_check: %d errors, %zu bytes in use, %zu free blocks\n", errors.load(),
            A.in_use(), A.free_blocks());
    return 1;
  }
  printf("arena_threads_check ok\n");
  return 0;
}
