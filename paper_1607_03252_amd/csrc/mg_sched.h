// Host-side admission scheduler of the serving form (no device code).
//
// Requests (level, seed) wait in one arrival-ordered queue.  Each MLMC level
// has a fixed pool of resident sample slots (sized by the caller from the HBM
// footprint of one sample of that level).  admit() walks the queue from its
// head and hands every request whose level has a free slot the lowest free
// slot of that level; a request whose pool is full keeps its place, so
// requests of one level are admitted in arrival order and a full level never
// blocks the others.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace mg {

struct Ticket {
  long long tag;     // caller's request id
  uint64_t seed;
  int level;
  int slot;          // assigned slot (-1 while queued)
  double t_arrival;  // caller's arrival time (seconds)
};

class Scheduler {
 public:
  // slots_per_level[l] >= 0 slots for level l; queue_capacity >= 1.
  Scheduler(const std::vector<int>& slots_per_level, int queue_capacity);

  // 0 on success, -1 for a bad level, -5 when the queue is full.
  int submit(int level, uint64_t seed, long long tag, double t_arrival);
  // Admit up to max_out queued requests; returns how many were written.
  // With open (one flag per level), only levels whose flag is set admit.
  int admit(Ticket* out, int max_out, const std::vector<char>* open = nullptr);
  // Free a busy slot; 0 on success, -1 if the slot is not busy.
  int release(int slot);

  int levels() const { return (int)first_.size() - 1; }
  int slots() const { return first_.back(); }
  int first_slot(int level) const { return first_[level]; }
  int slot_level(int slot) const { return slot_level_[slot]; }
  int queued() const { return (int)queue_.size(); }
  int busy() const { return busy_count_; }

 private:
  std::vector<int> first_;       // first slot of each level, plus the total
  std::vector<int> slot_level_;  // level of each slot
  std::vector<char> busy_;       // per slot
  std::vector<int> free_count_;  // per level
  int busy_count_ = 0;
  int capacity_;
  std::deque<Ticket> queue_;
};

}  // namespace mg
