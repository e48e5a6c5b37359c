// Host test of the device-arena sub-allocator (built with the host compiler and the
// address / undefined-behaviour sanitizers; no GPU): a seeded random sequence of
// allocations and releases against a plain model of the live blocks. Checks that
// blocks are 256-byte aligned, lie inside the arena and never overlap, that the
// in-use count is the sum of the live blocks, that an allocation that cannot fit
// throws RMC_ERR_OOM and leaves the arena as it was, and that releasing every block
// merges the free space back into one block of the whole arena; then the scoped
// scratch carved from it (alignment, bounds, disjoint pieces, release at scope end).
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <random>
#include <vector>

#include "../../paper_2609_02394_amd/csrc/host_util.h"

#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "arena_check: %s failed (line %d)\n", #c, __LINE__); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

int main() {
  const size_t size = (size_t)64 << 20;
  std::vector<char> fake(16);  // the arena only does arithmetic on its base pointer
  char* base = fake.data();
  rmc::Arena A;
  A.init(base, size);
  std::mt19937_64 rng(2609);
  std::map<size_t, size_t> live;  // offset -> rounded bytes
  size_t model_in_use = 0;
  long ooms = 0;
  for (int step = 0; step < 200000; ++step) {
    const bool grow = live.empty() || rng() % 100 < 55;
    if (grow) {
      size_t b = (rng() % 4 == 0) ? (rng() % (size_t)(8 << 20)) : (rng() % 70000);
      const size_t need = b == 0 ? 256 : (b + 255) / 256 * 256;
      const size_t before = A.in_use();
      try {
        char* p = static_cast<char*>(A.alloc(b));
        const size_t off = (size_t)(p - base);
        EXPECT(off % 256 == 0);
        EXPECT(off + need <= size);
        auto nx = live.lower_bound(off);
        if (nx != live.end()) EXPECT(off + need <= nx->first);
        if (nx != live.begin()) {
          auto pv = std::prev(nx);
          EXPECT(pv->first + pv->second <= off);
        }
        live[off] = need;
        model_in_use += need;
      } catch (const rmc::Error& e) {
        EXPECT(e.code == RMC_ERR_OOM);
        EXPECT(A.in_use() == before);
        EXPECT(A.largest_free() < need);
        ++ooms;
      }
    } else {
      auto it = live.begin();
      std::advance(it, (long)(rng() % live.size()));
      A.release(base + it->first);
      model_in_use -= it->second;
      live.erase(it);
    }
    EXPECT(A.in_use() == model_in_use);
    EXPECT(A.peak() >= A.in_use());
  }
  A.release(nullptr);
  A.release(base + 1);  // not handed out: ignored
  for (auto& kv : live) A.release(base + kv.first);
  EXPECT(A.in_use() == 0);
  EXPECT(A.free_blocks() == 1);
  EXPECT(A.largest_free() == size);
  // Scoped scratch: requests up to 1 MiB carved in order from 4 MiB blocks, larger ones
  // a block each; every piece 256-byte aligned, inside the arena, disjoint from the
  // others of its scope (and of an enclosing scope), and everything released at the
  // end of the scope.
  {
    struct Piece { size_t off, bytes; };
    std::vector<Piece> outer;
    rmc::Scratch so(&A);
    auto take = [&](rmc::Scratch& sc, std::vector<Piece>& v, size_t count) -> int {
      double* p = sc.get<double>(count);
      const size_t off = (size_t)((char*)p - base), bytes = (count ? count : 1) * sizeof(double);
      EXPECT(off % 256 == 0);
      EXPECT(off + bytes <= size);
      v.push_back({off, bytes});
      return 0;
    };
    for (int i = 0; i < 300; ++i) EXPECT(take(so, outer, rng() % 3000) == 0);
    const size_t used_outer = A.in_use();
    for (int round = 0; round < 20; ++round) {
      std::vector<Piece> inner;
      {
        rmc::Scratch si(&A);
        for (int i = 0; i < 100; ++i) {
          const size_t c = rng() % 10 == 0 ? (size_t)(1 << 17) + rng() % 200000 : rng() % 20000;
          EXPECT(take(si, inner, c) == 0);
        }
        std::vector<Piece> all(outer);
        all.insert(all.end(), inner.begin(), inner.end());
        std::sort(all.begin(), all.end(), [](const Piece& x, const Piece& y) { return x.off < y.off; });
        for (size_t i = 1; i < all.size(); ++i) EXPECT(all[i - 1].off + all[i - 1].bytes <= all[i].off);
        EXPECT(A.in_use() > used_outer);
      }
      EXPECT(A.in_use() == used_outer);
    }
  }
  EXPECT(A.in_use() == 0);
  EXPECT(A.free_blocks() == 1);
  printf("arena_check ok: %ld allocations refused for lack of space\n", ooms);
  return 0;
}
