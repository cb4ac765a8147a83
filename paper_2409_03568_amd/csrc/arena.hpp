// Host-side bookkeeping of the serving runtime: an offset allocator over one device
// memory region and the admission rule that decides which queued job starts next.
// Plain C++17 with no HIP dependency, so the same code is unit-tested on the CPU.
#pragma once
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>

namespace ckks {
namespace rt {

// First-fit allocator of byte ranges inside [0, capacity), every range aligned to
// `align` bytes.  Freed ranges are merged with their free neighbours, so memory that
// is entirely free is always one range again.
class Arena {
 public:
  explicit Arena(uint64_t capacity = 0, uint64_t align = 256) { reset(capacity, align); }

  void reset(uint64_t capacity, uint64_t align = 256) {
    align_ = align ? align : 1;
    capacity_ = capacity / align_ * align_;
    free_.clear();
    used_.clear();
    used_bytes_ = 0;
    if (capacity_) free_[0] = capacity_;
  }

  uint64_t round(uint64_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

  // Reserves `bytes` (rounded up to the alignment); false when no free range is large
  // enough.  A request of 0 bytes reserves one aligned unit so every job owns a range.
  bool alloc(uint64_t bytes, uint64_t *offset) {
    const uint64_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, size = it->second;
      free_.erase(it);
      if (size > need) free_[off + need] = size - need;
      used_[off] = need;
      used_bytes_ += need;
      *offset = off;
      return true;
    }
    return false;
  }

  // Returns a range obtained from alloc(); false for an offset that is not allocated.
  bool release(uint64_t offset) {
    auto it = used_.find(offset);
    if (it == used_.end()) return false;
    uint64_t off = it->first, size = it->second;
    used_.erase(it);
    used_bytes_ -= size;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + size == next->first) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += size;
        return true;
      }
    }
    free_[off] = size;
    return true;
  }

  uint64_t capacity() const { return capacity_; }
  uint64_t used() const { return used_bytes_; }
  size_t free_ranges() const { return free_.size(); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  uint64_t align_ = 256, capacity_ = 0, used_bytes_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  std::map<uint64_t, uint64_t> used_;  // offset -> size
};

// Admission by arrival order with bounded backfilling: the oldest queued job starts as
// soon as a slot (a stream) is free and the arena holds a contiguous range for its bytes.
// While it does not fit, younger jobs that do fit may start ahead of it, but every queued
// job can be overtaken at most max_bypass times; after that nothing younger starts before
// it, so no job waits forever behind a stream of smaller ones.  max_bypass = 0 is strict
// arrival order.
struct Queued {
  uint64_t id;
  uint64_t bytes;
  uint32_t bypassed = 0;  // younger jobs started ahead of this one
};

struct Admitted {
  uint64_t id;
  uint64_t offset;
};

class Admission {
 public:
  Admission(uint64_t capacity, uint32_t slots, uint64_t align = 256, uint32_t max_bypass = 0)
      : arena_(capacity, align), free_slots_(slots), max_bypass_(max_bypass) {}

  // A job that could never fit is refused at submission.
  bool fits_ever(uint64_t bytes) const { return arena_.round(bytes ? bytes : 1) <= arena_.capacity(); }
  void push(uint64_t id, uint64_t bytes) { queue_.push_back({id, bytes, 0}); }

  // Starts queued jobs (appended to out) and returns how many: the oldest ones while they
  // fit, then younger ones that fit ahead of a waiting older one within its bypass budget.
  template <class Out>
  size_t admit(Out &out) {
    size_t started = 0;
    while (!queue_.empty() && free_slots_ > 0) {
      uint64_t off = 0;
      if (!arena_.alloc(queue_.front().bytes, &off)) break;
      out.push_back(Admitted{queue_.front().id, off});
      queue_.pop_front();
      free_slots_--;
      started++;
    }
    if (queue_.empty() || free_slots_ == 0 || max_bypass_ == 0) return started;
    // the head waits for arena space: try the younger jobs, oldest first
    uint32_t budget = UINT32_MAX;  // smallest remaining bypass budget of the older jobs
    for (auto it = queue_.begin(); it != queue_.end() && free_slots_ > 0;) {
      if (it != queue_.begin()) {
        uint64_t off = 0;
        if (budget > 0 && arena_.alloc(it->bytes, &off)) {
          for (auto j = queue_.begin(); j != it; ++j) j->bypassed++;
          budget--;
          out.push_back(Admitted{it->id, off});
          it = queue_.erase(it);
          free_slots_--;
          started++;
          backfilled_++;
          continue;
        }
      }
      const uint32_t left = it->bypassed < max_bypass_ ? max_bypass_ - it->bypassed : 0;
      budget = left < budget ? left : budget;
      if (budget == 0) break;
      ++it;
    }
    return started;
  }

  // A started job finished: its slot and range become free.
  bool finish(uint64_t offset) {
    if (!arena_.release(offset)) return false;
    free_slots_++;
    return true;
  }

  // Removes one queued job; false if it is not in the queue.
  bool cancel(uint64_t id) {
    for (auto it = queue_.begin(); it != queue_.end(); ++it)
      if (it->id == id) {
        queue_.erase(it);
        return true;
      }
    return false;
  }

  // Drops every job still queued (their ids are appended to out).
  template <class Out>
  void cancel_queued(Out &out) {
    for (const auto &q : queue_) out.push_back(q.id);
    queue_.clear();
  }

  size_t queued() const { return queue_.size(); }
  uint32_t free_slots() const { return free_slots_; }
  uint64_t backfilled() const { return backfilled_; }
  const Arena &arena() const { return arena_; }

 private:
  Arena arena_;
  uint32_t free_slots_;
  uint32_t max_bypass_;
  uint64_t backfilled_ = 0;
  std::deque<Queued> queue_;
};

}  // namespace rt
}  // namespace ckks
