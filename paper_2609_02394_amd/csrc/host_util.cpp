// Host-only pieces of librmc (no HIP): phase timing and the device-arena sub-allocator.
#include "host_util.h"

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>

namespace rmc {

static constexpr size_t kAlign = 256;

namespace {
std::mutex host_trace_mu;
std::map<std::string, std::pair<long, double>> host_trace_tab;  // calls, ms
double host_now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
}  // namespace

bool host_trace_on() {
  static const bool on = getenv("RMC_TRACE_HOST") != nullptr;
  return on;
}
void host_trace_add(const char* name, double ms) {
  std::lock_guard<std::mutex> lk(host_trace_mu);
  auto& e = host_trace_tab[name];
  e.first++;
  e.second += ms;
}
void host_trace_dump(const char* title) {
  if (!host_trace_on()) return;
  std::lock_guard<std::mutex> lk(host_trace_mu);
  fprintf(stderr, "[rmc host] %s\n", title);
  for (auto& kv : host_trace_tab)
    fprintf(stderr, "[rmc host]   %-28s %8ld calls %10.2f ms\n", kv.first.c_str(), kv.second.first,
            kv.second.second);
  host_trace_tab.clear();
}
HostScope::HostScope(const char* n) : name(n) {
  if (host_trace_on()) t0 = host_now_ms();
}
HostScope::~HostScope() {
  if (host_trace_on()) host_trace_add(name, host_now_ms() - t0);
}

std::string admit_pass(const std::vector<size_t>& queued, size_t inflight_mem, int inflight,
                       int max_inflight, size_t budget) {
  std::string out;
  for (size_t i = 0; i < queued.size() && inflight < max_inflight; ++i) {
    const size_t m = queued[i];
    if (m > budget) {
      out.push_back('r');
      continue;
    }
    if (inflight > 0 && inflight_mem + m > budget) break;
    inflight_mem += m;
    ++inflight;
    out.push_back('a');
  }
  return out;
}

void Arena::init(char* base, size_t size) {
  base_ = base;
  size_ = size & ~(kAlign - 1);
  free_.clear();
  by_size_.clear();
  used_.clear();
  if (size_) add_free(0, size_);
  in_use_ = peak_ = 0;
}

void Arena::add_free(size_t off, size_t sz) {
  free_[off] = sz;
  by_size_.insert({sz, off});
}

void Arena::del_free(std::map<size_t, size_t>::iterator it) {
  by_size_.erase({it->second, it->first});
  free_.erase(it);
}

void* Arena::alloc(size_t bytes) {
  RMC_HOST_SCOPE("arena.alloc");
  std::lock_guard<std::mutex> lk(mu_);
  size_t need = (bytes + kAlign - 1) & ~(kAlign - 1);
  if (need == 0) need = kAlign;
  auto bs = by_size_.lower_bound({need, 0});  // the smallest free block that fits
  if (bs == by_size_.end())
    throw Error(RMC_ERR_OOM, "device arena exhausted (" + std::to_string(bytes) + " bytes requested, " +
                                 std::to_string(size_ - in_use_) + " free)");
  const size_t off = bs->second, sz = bs->first;
  del_free(free_.find(off));
  if (sz > need) add_free(off + need, sz - need);
  used_[off] = need;
  in_use_ += need;
  peak_ = std::max(peak_, in_use_);
  return base_ + off;
}

void Arena::release(void* p) {
  if (!p) return;
  RMC_HOST_SCOPE("arena.release");
  std::lock_guard<std::mutex> lk(mu_);
  size_t off = (size_t)((char*)p - base_);
  auto it = used_.find(off);
  if (it == used_.end()) return;
  size_t sz = it->second;
  used_.erase(it);
  in_use_ -= sz;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == off + sz) {  // merge with the block after
    sz += nx->second;
    del_free(nx);
  }
  auto pv = free_.lower_bound(off);
  if (pv != free_.begin()) {  // and with the block before
    --pv;
    if (pv->first + pv->second == off) {
      off = pv->first;
      sz += pv->second;
      del_free(pv);
    }
  }
  add_free(off, sz);
}

size_t Arena::largest_free() const {
  std::lock_guard<std::mutex> lk(mu_);
  return by_size_.empty() ? 0 : by_size_.rbegin()->first;
}

size_t Arena::free_blocks() const {
  std::lock_guard<std::mutex> lk(mu_);
  return free_.size();
}

}  // namespace rmc
