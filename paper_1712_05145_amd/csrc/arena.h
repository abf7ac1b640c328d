// First-fit free list over the byte offsets of a caller-owned device arena
// (host-side bookkeeping of the request server; no device calls).
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace ffth {

class FreeList {
 public:
  // The whole free space is [off, off + len).
  void reset(size_t off, size_t len) {
    free_.clear();
    if (len) free_[off] = len;
  }
  // Lowest-offset free range of at least `need` bytes; false if none.
  bool alloc(size_t need, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        *off = it->first;
        const size_t rest = it->second - need, at = it->first + need;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  // True when alloc(need) would succeed (nothing is taken).
  bool fits(size_t need) const {
    for (const auto& kv : free_)
      if (kv.second >= need) return true;
    return false;
  }
  // Give [off, off + len) back, merging with free neighbours.  A range that
  // overlaps free space was never handed out (or is returned twice): it is
  // refused, so that no byte can be handed out twice.
  bool release(size_t off, size_t len) {
    if (len == 0) return false;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first < off + len) return false;
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second > off) return false;
    }
    auto it = free_.emplace(off, len).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
    return true;
  }
  const std::map<size_t, size_t>& ranges() const { return free_; }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
};

}  // namespace ffth
