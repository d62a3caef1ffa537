// arena.h -- host-side bookkeeping of the caller-owned device arena.
//
// The library never allocates device memory: graphs, per-query state and
// results are carved out of one caller-provided buffer.  First-fit over an
// address-ordered free map, 256-byte alignment, neighbours coalesced on free.
#pragma once
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace plc {

class Arena {
 public:
  static constexpr size_t kAlign = 256;

  void reset(void* base, size_t bytes) {
    base_ = static_cast<char*>(base);
    size_ = bytes & ~(kAlign - 1);
    free_.clear();
    used_.clear();
    if (size_ > 0) free_[0] = size_;
  }

  // Returns nullptr when no free block is large enough.
  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = kAlign;
    bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first;
        size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_[off] = bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }

  // Returns false for pointers this arena did not hand out.
  bool release(void* p) {
    if (!p) return true;
    size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return true;
      }
    }
    free_[off] = len;
    return true;
  }

  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  size_t capacity() const { return size_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
};

}  // namespace plc
