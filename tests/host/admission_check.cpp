// Host test of the serving admission policy (rmc::admit_pass; no GPU), built with the
// address / undefined-behaviour sanitizers: a seeded random stream of submissions and
// completions drives a queue and a set of jobs in flight, and after every pass checks
// that the memory in flight stays within the budget and the jobs in flight within the
// slots, that jobs leave the queue in arrival order, that exactly the jobs above the
// budget are rejected, and that a pass ends only when the slots are full, the queue is
// empty, or the job at its head does not fit beside the jobs in flight.
#include <stdint.h>
#include <stdio.h>

#include <deque>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2609_02394_amd/csrc/host_util.h"

#define EXPECT(c)                                                              \
  do {                                                                         \
    if (!(c)) {                                                                \
      fprintf(stderr, "admission_check: %s failed (line %d)\n", #c, __LINE__); \
      return 1;                                                                \
    }                                                                          \
  } while (0)

struct Job {
  long id;
  size_t mem;
};

int main() {
  std::mt19937_64 rng(2609);
  long admitted = 0, rejected = 0, next_id = 0, last_left = -1;
  for (int trial = 0; trial < 200; ++trial) {
    const size_t budget = 1000 + rng() % 100000;
    const int slots = 1 + (int)(rng() % 64);
    std::deque<Job> queue;
    std::vector<Job> flight;
    size_t flight_mem = 0;
    for (int step = 0; step < 2000; ++step) {
      // arrivals (some above the budget) and completions
      const int arrive = (int)(rng() % 4);
      for (int a = 0; a < arrive; ++a) {
        const size_t mem = (rng() % 10 == 0) ? budget + 1 + rng() % budget : 1 + rng() % budget;
        queue.push_back({next_id++, mem});
      }
      if (!flight.empty() && rng() % 3 == 0) {
        const size_t i = rng() % flight.size();
        flight_mem -= flight[i].mem;
        flight.erase(flight.begin() + (long)i);
      }
      std::vector<size_t> mem;
      for (const Job& j : queue) mem.push_back(j.mem);
      const std::string d = rmc::admit_pass(mem, flight_mem, (int)flight.size(), slots, budget);
      EXPECT(d.size() <= queue.size());
      for (char c : d) {
        EXPECT(c == 'a' || c == 'r');
        const Job j = queue.front();
        queue.pop_front();
        EXPECT(j.id > last_left);  // arrival order
        last_left = j.id;
        if (c == 'r') {
          EXPECT(j.mem > budget);
          ++rejected;
        } else {
          EXPECT(j.mem <= budget);
          flight.push_back(j);
          flight_mem += j.mem;
          ++admitted;
        }
        EXPECT(flight_mem <= budget);
        EXPECT((int)flight.size() <= slots);
      }
      // why the pass ended
      if (!queue.empty() && (int)flight.size() < slots) {
        EXPECT(queue.front().mem <= budget);
        EXPECT(!flight.empty() && flight_mem + queue.front().mem > budget);
      }
    }
  }
  EXPECT(admitted > 0 && rejected > 0);
  printf("admission_check ok: %ld admitted, %ld rejected\n", admitted, rejected);
  return 0;
}
