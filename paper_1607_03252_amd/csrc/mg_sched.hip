// Admission scheduler of the serving form and its C ABI (host code only).
#include "mg_sched.h"

#include <algorithm>
#include <new>

#include "mlmcmg.h"

namespace mg {

Scheduler::Scheduler(const std::vector<int>& lane_slots, const std::vector<size_t>& lane_bytes,
                     size_t budget, int queue_capacity)
    : lane_slots_(lane_slots), lane_bytes_(lane_bytes), budget_(budget), capacity_(queue_capacity) {}

int Scheduler::submit(int level, uint64_t seed, long long tag, double t_arrival) {
  if (level < 0 || level >= levels()) return MG_EINVAL;
  if (lane_slots_[level] == 0 || lane_bytes_[level] > budget_) return MG_ENOMEM;
  if ((int)queue_.size() >= capacity_) return MG_EBUSY;
  queue_.push_back(Ticket{tag, seed, level, -1, -1, t_arrival, next_seq_++});
  return MG_OK;
}

int Scheduler::open_lane(int level) {
  const int k = lane_slots_[level];
  // the lowest run of k free slot numbers (the slot space grows at its end)
  int first = 0, run = 0;
  for (int s = 0; s < (int)slot_lane_.size() && run < k; ++s) {
    if (slot_lane_[s] >= 0) {
      run = 0;
      first = s + 1;
    } else {
      ++run;
    }
  }
  if ((int)slot_lane_.size() < first + k) {
    slot_lane_.resize(first + k, -1);
    slot_busy_.resize(first + k, 0);
  }
  const int id = next_lane_++;
  for (int s = first; s < first + k; ++s) slot_lane_[s] = id;
  lanes_.emplace(id, Lane{level, first, k});
  used_ += lane_bytes_[level];
  peak_ = std::max(peak_, used_);
  events_.push_back(LaneEvent{LaneEvent::kOpen, id, level, first, k, lane_bytes_[level]});
  return id;
}

void Scheduler::close_lane(int id) {
  const Lane ln = lanes_.at(id);
  for (int s = ln.first; s < ln.first + ln.nslots; ++s) slot_lane_[s] = -1;
  used_ -= lane_bytes_[ln.level];
  lanes_.erase(id);
  events_.push_back(LaneEvent{LaneEvent::kClose, id, ln.level, ln.first, ln.nslots,
                              lane_bytes_[ln.level]});
}

bool Scheduler::try_open(int level) {
  const size_t need = lane_bytes_[level];
  if (used_ + need > budget_) {
    size_t freeable = 0;
    for (const auto& kv : lanes_)
      if (evictable(kv.second)) freeable += lane_bytes_[kv.second.level];
    if (used_ - freeable + need > budget_) return false;
    const size_t deficit = used_ + need - budget_;
    // one victim when one is large enough (the smallest such), else the
    // largest first; ties go to the lower lane id
    int single = -1;
    for (const auto& kv : lanes_) {
      if (!evictable(kv.second)) continue;
      const size_t b = lane_bytes_[kv.second.level];
      if (b >= deficit && (single < 0 || b < lane_bytes_[lanes_.at(single).level])) single = kv.first;
    }
    std::vector<int> victims;
    if (single >= 0) {
      victims.push_back(single);
    } else {
      for (const auto& kv : lanes_)
        if (evictable(kv.second)) victims.push_back(kv.first);
      std::stable_sort(victims.begin(), victims.end(), [&](int a, int b) {
        return lane_bytes_[lanes_.at(a).level] > lane_bytes_[lanes_.at(b).level];
      });
      size_t got = 0, take = 0;
      while (got < deficit) got += lane_bytes_[lanes_.at(victims[take++]).level];
      victims.resize(take);
    }
    for (int v : victims) close_lane(v);
  }
  open_lane(level);
  return true;
}

void Scheduler::mark_drain(int level) {
  // bytes to set free beyond what the budget has left
  long long deficit = (long long)(used_ + lane_bytes_[level]) - (long long)budget_;
  for (auto& kv : lanes_)
    if (evictable(kv.second)) {
      kv.second.draining = true;
      deficit -= (long long)lane_bytes_[kv.second.level];
    }
  std::vector<int> cand;
  for (const auto& kv : lanes_)
    if (!kv.second.draining) cand.push_back(kv.first);
  // the fewest resident samples first (they empty soonest), then the larger
  // lane, then the lower id
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
    const Lane& x = lanes_.at(a);
    const Lane& y = lanes_.at(b);
    if (x.busy != y.busy) return x.busy < y.busy;
    return lane_bytes_[x.level] > lane_bytes_[y.level];
  });
  for (size_t i = 0; i < cand.size() && deficit > 0; ++i) {
    Lane& ln = lanes_.at(cand[i]);
    ln.draining = true;
    deficit -= (long long)lane_bytes_[ln.level];
  }
}

void Scheduler::clear_reservation() {
  reserve_ = -1;
  for (auto& kv : lanes_) kv.second.draining = false;
}

int Scheduler::admit(Ticket* out, int max_out) {
  int n = 0;
  // a level whose oldest queued request was passed over stays passed over
  // for the rest of the walk: what a later request of it finds (a drain
  // lifted, bytes set free by an eviction) its older requests find first in
  // the next walk, so each level keeps its arrival order
  std::vector<char> passed(levels(), 0);
  for (auto it = queue_.begin(); it != queue_.end() && n < max_out;) {
    const int l = it->level;
    if (passed[l]) {
      ++it;
      continue;
    }
    int lane = -1;
    bool waiting = false;  // free slots of its level exist in lanes on the device
    bool has_lane = false;
    for (const auto& kv : lanes_) {
      const Lane& ln = kv.second;
      if (ln.level != l) continue;
      has_lane = true;
      if (ln.draining || ln.busy == ln.nslots) continue;
      if (!ln.inflight) {
        lane = kv.first;
        break;
      }
      waiting = true;
    }
    if (lane < 0) {
      if (waiting || (reserve_ >= 0 && reserve_ != it->seq)) {
        passed[l] = 1;
        ++it;
        continue;
      }
      if (try_open(l)) {
        lane = next_lane_ - 1;
      } else {
        if (!has_lane && reserve_ < 0) {
          reserve_ = it->seq;
          mark_drain(l);
        }
        passed[l] = 1;
        ++it;
        continue;
      }
    }
    Lane& ln = lanes_.at(lane);
    int s = ln.first;
    while (slot_busy_[s]) ++s;  // lowest free slot of the lane
    slot_busy_[s] = 1;
    ++ln.busy;
    ++busy_count_;
    if (it->seq == reserve_) clear_reservation();
    Ticket t = *it;
    t.slot = s;
    t.lane = lane;
    out[n++] = t;
    it = queue_.erase(it);
  }
  return n;
}

int Scheduler::take_events(LaneEvent* out, int max_out) {
  int n = 0;
  while (n < max_out && !events_.empty()) {
    out[n++] = events_.front();
    events_.pop_front();
  }
  return n;
}

int Scheduler::set_inflight(int lane, bool inflight) {
  auto it = lanes_.find(lane);
  if (it == lanes_.end()) return MG_EINVAL;
  it->second.inflight = inflight;
  return MG_OK;
}

int Scheduler::release(int slot) {
  if (slot < 0 || slot >= (int)slot_busy_.size() || !slot_busy_[slot]) return MG_EINVAL;
  slot_busy_[slot] = 0;
  --busy_count_;
  --lanes_.at(slot_lane_[slot]).busy;
  return MG_OK;
}

}  // namespace mg

struct mg_sched_s {
  mg::Scheduler s;
};

extern "C" {

int mg_sched_create(int n_levels, const int* lane_slots, const size_t* lane_bytes, size_t budget,
                    int queue_capacity, mg_sched* out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (n_levels < 1 || !lane_slots || !lane_bytes || budget == 0 || queue_capacity < 1)
    return MG_EINVAL;
  std::vector<int> k(lane_slots, lane_slots + n_levels);
  std::vector<size_t> b(lane_bytes, lane_bytes + n_levels);
  for (int l = 0; l < n_levels; ++l)
    if (k[l] < 0 || k[l] > mg::Scheduler::kMaxLaneSlots || (k[l] > 0 && b[l] == 0)) return MG_EINVAL;
  auto* p = new (std::nothrow) mg_sched_s{mg::Scheduler(k, b, budget, queue_capacity)};
  if (!p) return MG_ENOMEM;
  *out = p;
  return MG_OK;
}

int mg_sched_destroy(mg_sched s) {
  delete s;
  return MG_OK;
}

int mg_sched_submit(mg_sched s, int level, uint64_t seed, long long tag, double t_arrival) {
  if (!s) return MG_EINVAL;
  return s->s.submit(level, seed, tag, t_arrival);
}

int mg_sched_admit(mg_sched s, mg_ticket* out, int max_out, int* n_out) {
  if (!s || !n_out || max_out < 0 || (max_out > 0 && !out)) return MG_EINVAL;
  std::vector<mg::Ticket> t(max_out);
  const int n = s->s.admit(t.data(), max_out);
  for (int i = 0; i < n; ++i)
    out[i] = mg_ticket{t[i].tag, t[i].seed, t[i].level, t[i].slot, t[i].lane, t[i].t_arrival};
  *n_out = n;
  return MG_OK;
}

int mg_sched_events(mg_sched s, mg_lane_event* out, int max_out, int* n_out) {
  if (!s || !n_out || max_out < 0 || (max_out > 0 && !out)) return MG_EINVAL;
  std::vector<mg::LaneEvent> e(max_out);
  const int n = s->s.take_events(e.data(), max_out);
  for (int i = 0; i < n; ++i)
    out[i] = mg_lane_event{e[i].kind, e[i].lane, e[i].level, e[i].first, e[i].nslots, e[i].bytes};
  *n_out = n;
  return MG_OK;
}

int mg_sched_set_inflight(mg_sched s, int lane, int inflight) {
  if (!s) return MG_EINVAL;
  return s->s.set_inflight(lane, inflight != 0);
}

int mg_sched_release(mg_sched s, int slot) {
  if (!s) return MG_EINVAL;
  return s->s.release(slot);
}

int mg_sched_counts(mg_sched s, int* queued, int* busy) {
  if (!s) return MG_EINVAL;
  if (queued) *queued = s->s.queued();
  if (busy) *busy = s->s.busy();
  return MG_OK;
}

int mg_sched_memory(mg_sched s, size_t* used, size_t* peak, int* lanes) {
  if (!s) return MG_EINVAL;
  if (used) *used = s->s.used();
  if (peak) *peak = s->s.peak();
  if (lanes) *lanes = s->s.lanes();
  return MG_OK;
}

}  // extern "C"
