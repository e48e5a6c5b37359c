// Host-only pieces of librmc that need no HIP: the error type, phase timing, the
// device-arena sub-allocator and scoped scratch over it (which only do offset
// arithmetic on a base pointer).
// Compiled into the library and, on its own, into the host sanitizer test.
#pragma once
#include <stddef.h>

#include <map>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/rmc.h"

namespace rmc {

struct Error : std::runtime_error {
  rmc_status code;
  Error(rmc_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RMC_CHECK(cond, code, msg) \
  do {                             \
    if (!(cond)) throw ::rmc::Error((code), (msg)); \
  } while (0)

// Host-side phase timing, on when RMC_TRACE_HOST is set: wall time per named phase,
// summed over calls and threads (lanes overlap, so sums can exceed the elapsed time);
// host_trace_dump prints the table to stderr and clears it.
bool host_trace_on();
void host_trace_add(const char* name, double ms);
void host_trace_dump(const char* title);
struct HostScope {
  const char* name;
  double t0 = 0.0;
  explicit HostScope(const char* n);
  ~HostScope();
};
#define RMC_HOST_SCOPE_CAT2(a, b) a##b
#define RMC_HOST_SCOPE_CAT(a, b) RMC_HOST_SCOPE_CAT2(a, b)
#define RMC_HOST_SCOPE(name) ::rmc::HostScope RMC_HOST_SCOPE_CAT(host_scope_, __LINE__)(name)

// Best-fit sub-allocator over one device buffer (256-byte granules): the free blocks
// are indexed by offset (to merge neighbours on release) and by (size, offset) (to find
// the smallest block that fits in O(log n)), so that the tens of thousands of scratch
// allocations of a large batched level cost microseconds, not a scan of every block.
// Throws Error(RMC_ERR_OOM) when no free block fits; releasing a pointer it did not
// hand out is ignored.
class Arena {
 public:
  void init(char* base, size_t size);
  void* alloc(size_t bytes);
  void release(void* p);
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }
  size_t largest_free() const;
  size_t free_blocks() const;

 private:
  void add_free(size_t off, size_t sz);
  void del_free(std::map<size_t, size_t>::iterator it);
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0, peak_ = 0;
  mutable std::mutex mu_;                        // the solver's lanes allocate from their own threads
  std::map<size_t, size_t> free_;                // offset -> bytes
  std::set<std::pair<size_t, size_t>> by_size_;  // (bytes, offset) of the free blocks
  std::unordered_map<size_t, size_t> used_;      // offset -> bytes
};


// Serving admission, the policy alone (host only, unit-tested without a GPU). In: the
// queued jobs' memory estimates in arrival order, the memory and number of the jobs in
// flight, the slot limit and the memory budget. Jobs go into flight in order while a
// slot is free and the job fits beside those in flight; a job above the budget can never
// run and is rejected where it stands (when a slot is free); the first job that has to
// wait ends the pass, so no later job overtakes it. Returns one letter per queued job
// the pass decided, in order: 'a' admitted, 'r' rejected; the others stay queued.
std::string admit_pass(const std::vector<size_t>& queued, size_t inflight_mem, int inflight,
                       int max_inflight, size_t budget);

// Scoped scratch memory, released together at the end of its scope. Requests up to
// 1 MiB are carved in order from 4 MiB arena blocks (256-byte aligned, as the arena's
// own blocks), so the many small tables of a batched level cost one arena call per
// block rather than one each; larger requests take an arena block of their own.
struct Scratch {
  static constexpr size_t kBlock = (size_t)4 << 20, kOwn = (size_t)1 << 20;
  Arena* arena;
  std::vector<void*> ptrs;
  char* cur = nullptr;
  size_t left = 0;
  explicit Scratch(Arena* a) : arena(a) {}
  ~Scratch() {
    for (void* p : ptrs) arena->release(p);
  }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  template <class T>
  T* get(size_t count) {
    size_t b = count * sizeof(T) > 0 ? count * sizeof(T) : 8;
    b = (b + 255) & ~(size_t)255;
    if (b > kOwn) {
      void* p = arena->alloc(b);
      ptrs.push_back(p);
      return static_cast<T*>(p);
    }
    if (b > left) {
      cur = static_cast<char*>(arena->alloc(kBlock));
      ptrs.push_back(cur);
      left = kBlock;
    }
    T* r = reinterpret_cast<T*>(cur);
    cur += b;
    left -= b;
    return r;
  }
};

}  // namespace rmc
