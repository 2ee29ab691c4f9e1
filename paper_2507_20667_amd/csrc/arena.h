// Device arena of a context: first-fit allocation over one borrowed device
// range in 256-byte granules.  Plain C++ (no HIP): the serve scheduler's CPU
// tests use it over a fake range.
//
// Allocations are either transient (call workspaces, released when the call
// ends) or persistent (a plan's leaves and descriptors, subtree programs,
// captured graphs' workspaces: held until the plan is freed).  Admission asks
// how much any workspace could ever get: the range minus what is persistent.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>

namespace tn {

class Arena {
 public:
  void init(uint8_t *base, size_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    base_ = base;
    bytes_ = bytes;
    used_ = persistent_ = 0;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  // returns the offset, or -1 when no free block is large enough
  int64_t alloc(size_t bytes, bool persistent = false) {
    std::lock_guard<std::mutex> g(mu_);
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        int64_t off = it->first;
        size_t rem = it->second - bytes;
        free_.erase(it);
        if (rem) free_[off + (int64_t)bytes] = rem;
        used_ += bytes;
        if (persistent) persistent_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, size_t bytes, bool persistent = false) {
    if (off < 0) return;
    std::lock_guard<std::mutex> g(mu_);
    bytes = round(bytes);
    used_ -= bytes;
    if (persistent) persistent_ -= bytes;
    ++releases_;
    auto it = free_.emplace((int64_t)off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + (int64_t)it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + (int64_t)pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest_free() {
    std::lock_guard<std::mutex> g(mu_);
    size_t m = 0;
    for (auto &kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  size_t used() {
    std::lock_guard<std::mutex> g(mu_);
    return used_;
  }
  // bytes that transient allocations could ever hold at once
  size_t work_capacity() {
    std::lock_guard<std::mutex> g(mu_);
    return bytes_ - persistent_;
  }
  // counts releases: a waiter that saw one value knows memory came back when
  // the count moves
  uint64_t releases() {
    std::lock_guard<std::mutex> g(mu_);
    return releases_;
  }
  uint8_t *base() const { return base_; }
  size_t bytes() const { return bytes_; }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

 private:
  std::mutex mu_;
  uint8_t *base_ = nullptr;
  size_t bytes_ = 0;
  size_t used_ = 0;
  size_t persistent_ = 0;
  uint64_t releases_ = 0;
  std::map<int64_t, size_t> free_;
};

}  // namespace tn
