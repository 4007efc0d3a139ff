// Host-side admission scheduler of the serving form (no device code).
//
// Requests (level, seed) wait in one arrival-ordered queue.  Resident samples
// live in lanes: a lane holds a fixed number of sample slots of one MLMC level
// and costs a fixed number of device bytes (its grids, state and staging).
// All lanes share one HBM budget.  A lane is opened when a request of its
// level finds no free slot and the budget (after evicting empty lanes) has
// room for it; empty lanes stay resident until their bytes are needed by
// another level.  admit() walks the queue from its head:
//  * a request takes the lowest free slot of the lowest idle lane of its
//    level that is not draining; if such lanes have free slots but are all
//    busy on the device, it waits for them;
//  * otherwise it opens a lane, evicting empty idle lanes when the budget is
//    short (one lane when one is large enough: the smallest such; otherwise
//    the largest first until the bytes suffice);
//  * a request that can open no lane and has no lane of its level reserves
//    the memory: while it waits, no other request opens a lane, and lanes of
//    other levels whose bytes cover the shortfall (empty ones first, then
//    those with the fewest resident samples) are drained, i.e. take no new
//    samples, until they are empty and can be evicted for it.
// Once a request waits, later requests of its level wait for the rest of
// that walk.  Requests of one level are admitted in arrival order, the
// budget is never exceeded, and every request is admitted once enough
// samples finish.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace mg {

struct Ticket {
  long long tag;     // caller's request id
  uint64_t seed;
  int level;
  int slot;          // assigned slot (-1 while queued)
  int lane;          // lane of that slot (-1 while queued)
  double t_arrival;  // caller's arrival time (seconds)
  long long seq;     // submission number (internal)
};

struct LaneEvent {
  enum Kind { kOpen = 1, kClose = 2 };
  int kind;
  int lane;
  int level;
  int first;   // first slot of the lane; its slots are first .. first + nslots - 1
  int nslots;
  size_t bytes;
};

class Scheduler {
 public:
  // lane_slots[l] in [0, kMaxLaneSlots] slots per lane of level l (0: the
  // level is not served); lane_bytes[l] device bytes of such a lane; budget
  // bytes for all lanes together; queue_capacity >= 1.
  Scheduler(const std::vector<int>& lane_slots, const std::vector<size_t>& lane_bytes,
            size_t budget, int queue_capacity);
  static constexpr int kMaxLaneSlots = 4096;

  // 0 on success; -1 for a bad level; -2 when a lane of that level cannot fit
  // the budget (or the level has no slots); -5 when the queue is full.
  int submit(int level, uint64_t seed, long long tag, double t_arrival);
  // Admit up to max_out queued requests; returns how many were written.  The
  // lanes it opens and evicts are queued as events (evictions first).
  int admit(Ticket* out, int max_out);
  // Take up to max_out pending lane events, oldest first.
  int take_events(LaneEvent* out, int max_out);
  // Mark a lane as running on the device (no admission, no eviction) or idle.
  int set_inflight(int lane, bool inflight);
  // Free a busy slot; 0 on success, -1 if the slot is not busy.
  int release(int slot);

  int levels() const { return (int)lane_slots_.size(); }
  int lane_slots(int level) const { return lane_slots_[level]; }
  size_t lane_bytes(int level) const { return lane_bytes_[level]; }
  int queued() const { return (int)queue_.size(); }
  int busy() const { return busy_count_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t budget() const { return budget_; }
  int lanes() const { return (int)lanes_.size(); }
  int slot_space() const { return (int)slot_lane_.size(); }
  bool reserved() const { return reserve_ >= 0; }

 private:
  struct Lane {
    int level, first, nslots, busy = 0;
    bool inflight = false, draining = false;
  };
  bool try_open(int level);
  int open_lane(int level);
  void close_lane(int id);
  void mark_drain(int level);
  void clear_reservation();
  bool evictable(const Lane& ln) const { return ln.busy == 0 && !ln.inflight; }

  std::vector<int> lane_slots_;
  std::vector<size_t> lane_bytes_;
  size_t budget_, used_ = 0, peak_ = 0;
  int capacity_;
  std::map<int, Lane> lanes_;     // by id (ascending: the admission order)
  int next_lane_ = 0;
  std::vector<int> slot_lane_;    // lane of each slot of the slot space, -1: none
  std::vector<char> slot_busy_;
  int busy_count_ = 0;
  std::deque<Ticket> queue_;
  long long next_seq_ = 0;
  long long reserve_ = -1;        // seq of the request holding the reservation
  std::deque<LaneEvent> events_;
};

}  // namespace mg
