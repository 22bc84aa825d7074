// serve_arena.hpp -- host-side admission bookkeeping of the served form:
// a first-fit allocator over one device region (offsets only, no device
// calls) and the admission decision.  Header-only plain C++.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>
#include <utility>
#include <vector>

namespace fmc {
namespace serve {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

class Arena {
 public:
  void init(size_t n) {
    size_ = n;
    used_ = 0;
    free_.clear();
    if (n) free_[0] = n;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t n_free_blocks() const { return free_.size(); }
  // First fit; false if no free block is large enough.
  bool alloc(size_t n, size_t* off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o2 = it->first + n;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  // Return a block; neighbouring free blocks are merged.
  void release(size_t off, size_t n) {
    n = align_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // Allocate every part of a request or none of them (offsets in out).
  bool alloc_all(const std::vector<size_t>& parts, std::vector<std::pair<size_t, size_t>>* out) {
    out->clear();
    for (size_t p : parts) {
      if (p == 0) continue;
      size_t off = 0;
      if (!alloc(p, &off)) {
        for (auto& b : *out) release(b.first, b.second);
        out->clear();
        return false;
      }
      out->push_back({off, p});
    }
    return true;
  }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

// Sum of a request's parts as the arena counts them.
inline size_t footprint(const std::vector<size_t>& parts) {
  size_t t = 0;
  for (size_t p : parts) t += p ? align_up(p) : 0;
  return t;
}

enum Decision { ADMIT = 0, NEVER = 1, NOT_NOW = 2 };

// NEVER: larger than the whole arena; NOT_NOW: every slot is taken or no room
// now (the parts are then not allocated); ADMIT: the parts are allocated.
inline Decision admit(Arena& a, const std::vector<size_t>& parts, int slots_used, int max_slots,
                      std::vector<std::pair<size_t, size_t>>* blocks) {
  if (footprint(parts) > a.size()) return NEVER;
  if (slots_used >= max_slots) return NOT_NOW;
  return a.alloc_all(parts, blocks) ? ADMIT : NOT_NOW;
}

}  // namespace serve
}  // namespace fmc
