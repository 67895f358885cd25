// Host-side bookkeeping of the serving runtime, free of HIP so that it also builds
// with the host compiler alone (the CPU tests compile it with AddressSanitizer): the
// first-fit allocator over one device allocation and the admission step for the
// request at the head of the queue.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace mapi {

constexpr size_t kPoolGranule = 256;

inline size_t pool_round(size_t x) { return (x + kPoolGranule - 1) / kPoolGranule * kPoolGranule; }

// First-fit allocator over [0, bytes) in 256-byte granules: free ranges keyed by
// offset, the lowest fitting range is split, released ranges merge with both
// neighbours, so the free list never holds two adjacent ranges.
class Pool {
 public:
  void reset(size_t bytes) {
    free_.clear();
    size_ = bytes / kPoolGranule * kPoolGranule;
    if (size_) free_[0] = size_;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = pool_round(bytes);
    if (bytes == 0) bytes = kPoolGranule;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  // Give back a range returned by alloc with the same size.
  void release(size_t off, size_t bytes) {
    bytes = pool_round(bytes);
    if (bytes == 0) bytes = kPoolGranule;
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
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t free_ranges() const { return free_.size(); }
  // The free list's invariants: ranges inside the pool, sorted, neither overlapping
  // nor adjacent, and together the complement of what is in use.
  bool consistent() const {
    size_t end = 0, total = 0;
    bool first = true;
    for (const auto& r : free_) {
      if (r.second == 0 || r.first % kPoolGranule || r.second % kPoolGranule) return false;
      if (!first && r.first <= end) return false;     // overlapping or adjacent
      if (r.first + r.second > size_) return false;
      end = r.first + r.second;
      total += r.second;
      first = false;
    }
    return total + used_ == size_;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

// Outcome of trying to admit the request at the head of the queue.
enum class Admission { kReject, kWait, kAdmit };

// Admission of one request: rejected at once if its device footprint alone exceeds
// the budget; otherwise it waits (nothing held) unless an instance slot is free, the
// queue has room for its work items, and both its device buffers and its result fit
// their pools, in which case both ranges are reserved.
inline Admission admit_request(Pool& dev, Pool& out, size_t budget, size_t dev_bytes, size_t out_bytes,
                               bool slot_free, uint64_t live_tiles, uint64_t tiles, uint64_t tile_cap,
                               size_t* dev_off, size_t* out_off) {
  if (dev_bytes > budget) return Admission::kReject;
  if (!slot_free || live_tiles + tiles > tile_cap) return Admission::kWait;
  if (!dev.alloc(dev_bytes, dev_off)) return Admission::kWait;
  if (!out.alloc(out_bytes, out_off)) {
    dev.release(*dev_off, dev_bytes);
    return Admission::kWait;
  }
  return Admission::kAdmit;
}

}  // namespace mapi
