// First-fit sub-allocator over one device block, for the serving scheduler's
// workspace budget.  Pure host C++ (offsets only, no HIP), so it can be
// checked on a machine without a GPU.
//
// Every size is counted in 256-byte granules: capacity() is the budget
// rounded down to a granule and a request of n bytes takes need(n) =
// n rounded up.  A request with need(n) <= capacity() therefore always fits
// in an empty arena -- the property the scheduler's admission relies on.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace ftm_rt {

class Arena {
 public:
  static constexpr size_t kGranule = 256;
  static size_t need(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }

  void reset(size_t budget) {
    cap_ = budget / kGranule * kGranule;
    free_.clear();
    if (cap_) free_[0] = cap_;
    used_ = 0;
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }

  // Take need(bytes) bytes; false if no free block is large enough.
  bool alloc(size_t bytes, size_t* off) {
    bytes = need(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }

  // Return a block taken by alloc(bytes) at off; neighbouring free blocks merge.
  void release(size_t off, size_t bytes) {
    bytes = need(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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

  // Number of free blocks (1 when everything has been released).
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> length of each free block
  size_t cap_ = 0, used_ = 0;
};

}  // namespace ftm_rt
