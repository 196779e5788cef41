// Host-side policy of the serving loop: the HBM pool allocator and the choice
// of the next request to admit.  Plain C++ (no HIP), so the policy can be
// exercised on a host without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>

namespace rlu {
namespace serve {

constexpr size_t kGranule = 256;  // workspace alignment the compute calls require

inline size_t round_up(size_t v) { return (v + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over [0, size): free ranges keyed by offset, merged
// with their neighbours on release.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    size_ = size / kGranule * kGranule;
    free_.clear();
    if (size_) free_[0] = size_;
    used_ = 0;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t b = 0;
    for (const auto &f : free_)
      if (f.second > b) b = f.second;
    return b;
  }
  // true and *off set when `bytes` (rounded up to the granule) fits somewhere
  bool alloc(size_t bytes, size_t *off) {
    const size_t need = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        *off = it->first;
        const size_t rest = it->second - need;
        const size_t at = it->first + need;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += need;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    const size_t len = round_up(bytes ? bytes : 1);
    used_ -= len;
    auto next = free_.lower_bound(off);
    size_t start = off, end = off + len;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        free_.erase(prev);
      }
    }
    next = free_.lower_bound(end);
    if (next != free_.end() && next->first == end) {
      end += next->second;
      free_.erase(next);
    }
    free_[start] = end - start;
  }
  size_t free_ranges() const { return free_.size(); }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

// Admission: the oldest queued request if its workspace fits the pool and
// its LU panel blocks fit `blocks_free` (what the running requests leave of
// the compute units).  If it does not, a younger one that fits may go first
// (so small requests keep the device busy while memory or blocks for a large
// one free up), but at most `max_bypass` times for the same head, after
// which the loop waits for the head.  Returns the queue index to admit and
// its offset, or -1.
template <typename Req>
int pick_next(std::deque<Req> &queue, PoolAlloc &pool, int blocks_free, int max_bypass, size_t *off) {
  if (queue.empty()) return -1;
  auto fits = [&](const Req &r) { return r.blocks <= blocks_free && pool.alloc(r.bytes, off); };
  if (fits(queue.front())) return 0;
  if (queue.front().bypassed >= max_bypass) return -1;
  for (size_t i = 1; i < queue.size(); ++i) {
    if (fits(queue[i])) {
      ++queue.front().bypassed;
      return (int)i;
    }
  }
  return -1;
}

}  // namespace serve
}  // namespace rlu
