// Admission scheduler of the serving form and its C ABI (host code only).
#include "mg_sched.h"

#include <algorithm>
#include <new>

#include "mlmcmg.h"

namespace mg {

Scheduler::Scheduler(const std::vector<int>& slots_per_level, int queue_capacity)
    : capacity_(queue_capacity) {
  first_.push_back(0);
  for (size_t l = 0; l < slots_per_level.size(); ++l) {
    first_.push_back(first_.back() + slots_per_level[l]);
    free_count_.push_back(slots_per_level[l]);
    for (int s = 0; s < slots_per_level[l]; ++s) slot_level_.push_back((int)l);
  }
  busy_.assign(first_.back(), 0);
}

int Scheduler::submit(int level, uint64_t seed, long long tag, double t_arrival) {
  if (level < 0 || level >= levels()) return MG_EINVAL;
  if ((int)queue_.size() >= capacity_) return MG_EBUSY;
  queue_.push_back(Ticket{tag, seed, level, -1, t_arrival});
  return MG_OK;
}

int Scheduler::admit(Ticket* out, int max_out, const std::vector<char>* open_levels) {
  auto usable = [&](int l) { return free_count_[l] > 0 && (!open_levels || (*open_levels)[l]); };
  int n = 0;
  int open = 0;  // levels that can still admit
  for (int l = 0; l < levels(); ++l) open += usable(l);
  for (auto it = queue_.begin(); it != queue_.end() && n < max_out && open > 0;) {
    const int l = it->level;
    if (!usable(l)) {
      ++it;
      continue;
    }
    int s = first_[l];
    while (busy_[s]) ++s;  // lowest free slot of the level
    busy_[s] = 1;
    ++busy_count_;
    if (--free_count_[l] == 0) --open;
    Ticket t = *it;
    t.slot = s;
    out[n++] = t;
    it = queue_.erase(it);
  }
  return n;
}

int Scheduler::release(int slot) {
  if (slot < 0 || slot >= slots() || !busy_[slot]) return MG_EINVAL;
  busy_[slot] = 0;
  --busy_count_;
  ++free_count_[slot_level_[slot]];
  return MG_OK;
}

}  // namespace mg

struct mg_sched_s {
  mg::Scheduler s;
};

extern "C" {

int mg_sched_create(int n_levels, const int* slots_per_level, int queue_capacity, mg_sched* out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (n_levels < 1 || !slots_per_level || queue_capacity < 1) return MG_EINVAL;
  std::vector<int> v(slots_per_level, slots_per_level + n_levels);
  for (int c : v)
    if (c < 0) return MG_EINVAL;
  auto* p = new (std::nothrow) mg_sched_s{mg::Scheduler(v, queue_capacity)};
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
    out[i] = mg_ticket{t[i].tag, t[i].seed, t[i].level, t[i].slot, t[i].t_arrival};
  *n_out = n;
  return MG_OK;
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

}  // extern "C"
