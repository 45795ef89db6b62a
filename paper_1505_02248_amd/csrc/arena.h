// First-fit sub-allocator over one device allocation (host-side bookkeeping).
//
// The serving loop admits and retires requests continuously; taking their
// memory from one pre-allocated pool avoids hipMalloc/hipFree (the latter
// synchronizes the device) in that loop and makes the memory budget exact.
// Ranges are 256-byte aligned; freeing coalesces neighbouring free ranges.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace lem {

class Arena {
 public:
  Arena(char* base, size_t size) : base_(base), size_(size) {
    if (size_) free_[0] = size_;
  }

  void* alloc(size_t bytes) {
    const size_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      in_use_ += need;
      return base_ + off;
    }
    return nullptr;
  }

  bool release(void* p) {
    if (!p) return true;
    const size_t off = (size_t)((char*)p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
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
    return true;
  }

  size_t in_use() const { return in_use_; }
  size_t capacity() const { return size_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  bool owns(const void* p) const {
    return (const char*)p >= base_ && (const char*)p < base_ + size_;
  }

  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

 private:
  char* base_;
  size_t size_;
  size_t in_use_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;
};

}  // namespace lem
