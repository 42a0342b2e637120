// Device-memory pool and admission bookkeeping of the serving loop.
// Header-only and free of HIP calls, so the host logic can be exercised
// without a device.
#pragma once

#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <vector>

namespace rl {

// First-fit allocator over one slab [0, capacity) with coalescing frees.
// Offsets and sizes are multiples of `align` (a power of two).
class SlabAllocator {
 public:
  explicit SlabAllocator(uint64_t capacity = 0, uint64_t align = 256) { reset(capacity, align); }

  void reset(uint64_t capacity, uint64_t align) {
    align_ = align;
    capacity_ = capacity / align * align;
    free_.clear();
    used_.clear();
    if (capacity_) free_[0] = capacity_;
    in_use_ = 0;
  }

  uint64_t round(uint64_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

  // Offset of a block of `bytes` (rounded up), or UINT64_MAX if none fits.
  uint64_t alloc(uint64_t bytes) {
    const uint64_t need = std::max<uint64_t>(round(bytes), align_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first;
      const uint64_t rest = it->second - need;
      free_.erase(it);
      if (rest) free_[off + need] = rest;
      used_[off] = need;
      in_use_ += need;
      return off;
    }
    return UINT64_MAX;
  }

  // Whether blocks of these sizes could all be placed now.
  bool fits(const std::vector<uint64_t>& sizes) const {
    std::map<uint64_t, uint64_t> f = free_;
    for (uint64_t b : sizes) {
      const uint64_t need = std::max<uint64_t>(round(b), align_);
      bool ok = false;
      for (auto it = f.begin(); it != f.end(); ++it) {
        if (it->second < need) continue;
        const uint64_t off = it->first, rest = it->second - need;
        f.erase(it);
        if (rest) f[off + need] = rest;
        ok = true;
        break;
      }
      if (!ok) return false;
    }
    return true;
  }

  void release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    uint64_t start = off, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }

  uint64_t in_use() const { return in_use_; }
  uint64_t capacity() const { return capacity_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  uint64_t align_ = 256, capacity_ = 0, in_use_ = 0;
  std::map<uint64_t, uint64_t> free_;   // offset -> length
  std::map<uint64_t, uint64_t> used_;   // offset -> length
};

// Nearest-rank percentile of a sample (p in [0, 100]).
inline double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

}  // namespace rl
