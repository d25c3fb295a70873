// arena.h -- host-side bookkeeping of one device memory arena: first-fit
// allocation of 256-byte aligned blocks with coalescing on free.  Only
// offsets are handled here (no device calls), so the server can take memory
// for records and workspaces without hipMalloc on the request path, and the
// logic is testable on the host.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace nk {

class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  static constexpr uint64_t kFail = ~0ull;

  explicit Arena(uint64_t bytes = 0) { reset(bytes); }

  void reset(uint64_t bytes) {
    free_.clear();
    used_.clear();
    cap_ = bytes / kAlign * kAlign;
    in_use_ = 0;
    peak_ = 0;
    if (cap_) free_[0] = cap_;
  }

  // Offset of a block of at least `bytes` (rounded up to kAlign), or kFail.
  uint64_t alloc(uint64_t bytes) {
    if (bytes == 0) bytes = 1;
    if (bytes > cap_) return kFail;
    const uint64_t need = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      in_use_ += need;
      if (in_use_ > peak_) peak_ = in_use_;
      return off;
    }
    return kFail;
  }

  // Like alloc, but from the top end of the highest free block that fits:
  // long-lived blocks taken this way stay clear of the short-lived ones taken
  // from the bottom, so releasing the latter leaves one contiguous region.
  uint64_t alloc_top(uint64_t bytes) {
    if (bytes == 0) bytes = 1;
    if (bytes > cap_) return kFail;
    const uint64_t need = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, len = it->second;
      const uint64_t blk = off + len - need;
      if (len > need) {
        free_[off] = len - need;
      } else {
        free_.erase(off);
      }
      used_[blk] = need;
      in_use_ += need;
      if (in_use_ > peak_) peak_ = in_use_;
      return blk;
    }
    return kFail;
  }

  // Releases a block returned by alloc or alloc_top; false if `off` is not one.
  bool release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    uint64_t start = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {  // merge with the right
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the left
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

  uint64_t capacity() const { return cap_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t free_blocks() const { return free_.size(); }
  size_t used_blocks() const { return used_.size(); }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length, disjoint, never adjacent
  std::map<uint64_t, uint64_t> used_;  // offset -> length
  uint64_t cap_ = 0, in_use_ = 0, peak_ = 0;
};

}  // namespace nk
