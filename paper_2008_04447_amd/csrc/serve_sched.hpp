// Host-only admission logic of the serving loop (no HIP): a first-fit arena
// over the HBM budget and a FIFO of waiting requests.  A request is admitted
// when a slot is free and a contiguous block of its footprint fits in the
// arena; the head of the queue is never bypassed, so admission order equals
// arrival order.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace rq {

class Arena {
 public:
  explicit Arena(size_t bytes) : size_(bytes) { free_[0] = bytes; }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  // First-fit allocation; returns false when no free block is large enough.
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {   // merge right
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {                                          // merge left
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
};

struct Pending {
  uint64_t id;
  size_t footprint;
};

struct Admission {
  uint64_t id;
  size_t offset;
};

class Admitter {
 public:
  explicit Admitter(size_t budget) : arena_(budget) {}
  // Returns false (and queues nothing) when the request can never fit.
  bool enqueue(uint64_t id, size_t footprint) {
    if (Arena::round(footprint) > arena_.size()) return false;
    queue_.push_back(Pending{id, footprint});
    return true;
  }
  // Admit from the head while slots and memory allow.
  std::vector<Admission> admit(int free_slots) {
    std::vector<Admission> out;
    while (free_slots > 0 && !queue_.empty()) {
      size_t off;
      if (!arena_.alloc(queue_.front().footprint, &off)) break;
      out.push_back(Admission{queue_.front().id, off});
      queue_.pop_front();
      --free_slots;
    }
    return out;
  }
  void finish(size_t offset, size_t footprint) { arena_.release(offset, footprint); }
  size_t queued() const { return queue_.size(); }
  size_t used() const { return arena_.used(); }
  const Arena& arena() const { return arena_; }

 private:
  Arena arena_;
  std::deque<Pending> queue_;
};

}  // namespace rq
