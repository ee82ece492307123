// arena.h -- the served form's request-state allocator (host-only; no HIP
// types, so that a plain C++ compiler can build and test it).
#pragma once
#include <atomic>
#include <cstdint>
#include <iterator>
#include <map>

namespace pg {

// First-fit allocator over [0, size) with coalescing, 256-byte granules.
struct Arena {
  std::map<int64_t, int64_t> free_;  // offset -> length
  int64_t size = 0;
  std::atomic<int64_t> used{0};
  void reset(int64_t sz) {
    free_.clear();
    size = sz;
    used = 0;
    if (sz > 0) free_[0] = sz;
  }
  int64_t alloc(int64_t len) {
    len = (len + 255) & ~(int64_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const int64_t off = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest > 0) free_[off + len] = rest;
        used += len;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t len) {
    len = (len + 255) & ~(int64_t)255;
    used -= len;
    auto it = free_.emplace(off, len).first;
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
};

}  // namespace pg
