"""CPU tests of the serving form's admission scheduler (mg_sched_*, host only).

The policy: one queue in arrival order; samples live in lanes of a fixed
number of slots of one level, each costing fixed bytes, under one shared
budget.  A request takes a free slot of an idle, non-draining lane of its
level, else opens a lane (evicting empty idle lanes when the budget is
short), else, when its level has no lane at all, reserves memory: no other
request opens a lane until it is admitted, and lanes of other levels drain.
The tests drive the native scheduler with a fake executor (service times
drawn on the host), compare every admission and every lane event with a
plain Python model of that policy, and check the invariants that follow
from it: the budget is never exceeded, each level is admitted in arrival
order, every request is eventually admitted, and memory one level leaves
idle admits requests of another.
"""
import collections

import numpy as np
import pytest

import paper_1607_03252_amd as M

OPEN, CLOSE = M.MG_LANE_OPEN, M.MG_LANE_CLOSE


class Model:
    """The admission policy written out directly (independent of the C++)."""

    def __init__(self, slots, nbytes, budget, cap):
        self.k, self.b, self.budget, self.cap = list(slots), list(nbytes), budget, cap
        self.q = []          # [seq, tag, seed, level, t]
        self.seq = 0
        self.lanes = {}      # id -> dict(level, first, n, busy, inflight, draining)
        self.next_id = 0
        self.slot_lane = []  # lane id per slot number, or None
        self.slot_busy = []
        self.used = 0
        self.reserve = None
        self.events = []
        self.reservations = 0
        self.evictions = 0

    def bytes_of(self, lid):
        return self.b[self.lanes[lid]["level"]]

    def submit(self, level, seed, tag, t):
        if not 0 <= level < len(self.k):
            return M.MG_EINVAL
        if self.k[level] == 0 or self.b[level] > self.budget:
            return M.MG_ENOMEM
        if len(self.q) >= self.cap:
            return M.MG_EBUSY
        self.q.append([self.seq, tag, seed, level, t])
        self.seq += 1
        return M.MG_OK

    def _open(self, level):
        k = self.k[level]
        first = 0
        while any(x is not None for x in self.slot_lane[first:first + k]):
            first += 1
        while len(self.slot_lane) < first + k:
            self.slot_lane.append(None)
            self.slot_busy.append(False)
        lid = self.next_id
        self.next_id += 1
        for s in range(first, first + k):
            self.slot_lane[s] = lid
        self.lanes[lid] = dict(level=level, first=first, n=k, busy=0, inflight=False,
                               draining=False)
        self.used += self.b[level]
        self.events.append((OPEN, lid, level, first, k, self.b[level]))
        return lid

    def _close(self, lid):
        ln = self.lanes.pop(lid)
        for s in range(ln["first"], ln["first"] + ln["n"]):
            self.slot_lane[s] = None
        self.used -= self.b[ln["level"]]
        self.events.append((CLOSE, lid, ln["level"], ln["first"], ln["n"], self.b[ln["level"]]))

    def _empty(self):
        return [i for i in sorted(self.lanes)
                if self.lanes[i]["busy"] == 0 and not self.lanes[i]["inflight"]]

    def _try_open(self, level):
        need = self.b[level]
        if self.used + need > self.budget:
            empty = self._empty()
            if self.used - sum(self.bytes_of(i) for i in empty) + need > self.budget:
                return None
            short = self.used + need - self.budget
            big = [i for i in empty if self.bytes_of(i) >= short]
            if big:
                victims = [min(big, key=lambda i: (self.bytes_of(i), i))]
            else:
                victims, got = [], 0
                for i in sorted(empty, key=lambda i: (-self.bytes_of(i), i)):
                    if got >= short:
                        break
                    victims.append(i)
                    got += self.bytes_of(i)
            for i in victims:
                self._close(i)
                self.evictions += 1
        return self._open(level)

    def _drain(self, level):
        short = self.used + self.b[level] - self.budget
        for i in self._empty():
            self.lanes[i]["draining"] = True
            short -= self.bytes_of(i)
        rest = sorted((i for i in self.lanes if not self.lanes[i]["draining"]),
                      key=lambda i: (self.lanes[i]["busy"], -self.bytes_of(i), i))
        for i in rest:
            if short <= 0:
                break
            self.lanes[i]["draining"] = True
            short -= self.bytes_of(i)

    def admit(self, max_out):
        out, keep = [], []
        passed = set()  # levels with a request left waiting in this walk
        for idx, r in enumerate(self.q):
            if len(out) >= max_out:
                keep.extend(self.q[idx:])
                break
            seq, tag, seed, lv, t = r
            if lv in passed:
                keep.append(r)
                continue
            mine = [i for i in sorted(self.lanes) if self.lanes[i]["level"] == lv]
            free = [i for i in mine
                    if not self.lanes[i]["draining"] and self.lanes[i]["busy"] < self.lanes[i]["n"]]
            idle = [i for i in free if not self.lanes[i]["inflight"]]
            if idle:
                lid = idle[0]
            elif free or (self.reserve is not None and self.reserve != seq):
                passed.add(lv)
                keep.append(r)
                continue
            else:
                lid = self._try_open(lv)
                if lid is None:
                    if not mine and self.reserve is None:
                        self.reserve = seq
                        self.reservations += 1
                        self._drain(lv)
                    passed.add(lv)
                    keep.append(r)
                    continue
            ln = self.lanes[lid]
            s = ln["first"]
            while self.slot_busy[s]:
                s += 1
            self.slot_busy[s] = True
            ln["busy"] += 1
            if seq == self.reserve:
                self.reserve = None
                for x in self.lanes.values():
                    x["draining"] = False
            out.append((tag, seed, lv, s, lid, t))
        self.q = keep
        return out

    def take_events(self):
        e, self.events = self.events, []
        return e

    def set_inflight(self, lid, flag):
        if lid not in self.lanes:
            return M.MG_EINVAL
        self.lanes[lid]["inflight"] = bool(flag)
        return M.MG_OK

    def release(self, slot):
        if not (0 <= slot < len(self.slot_busy)) or not self.slot_busy[slot]:
            return M.MG_EINVAL
        self.slot_busy[slot] = False
        self.lanes[self.slot_lane[slot]]["busy"] -= 1
        return M.MG_OK


class Executor:
    """Fake executor: lanes from the scheduler's events, every lane that holds
    samples runs one step per round (its launch in flight), service times
    drawn on the host.  Checks the events against the lanes it holds."""

    def __init__(self, s, budget):
        self.s, self.budget = s, budget
        self.lanes = {}      # lane -> (level, first, n, bytes)
        self.run = {}        # slot -> [tag, steps left, lane]
        self.used = 0
        self.peak = 0

    def apply(self, events):
        for kind, lid, lv, first, n, nb in events:
            if kind == CLOSE:
                assert lid in self.lanes and self.lanes[lid] == (lv, first, n, nb)
                assert not any(v[2] == lid for v in self.run.values()), "evicted a lane in use"
                del self.lanes[lid]
                self.used -= nb
            else:
                assert kind == OPEN and lid not in self.lanes
                for other in self.lanes.values():  # slot ranges are disjoint
                    assert first + n <= other[1] or other[1] + other[2] <= first
                self.lanes[lid] = (lv, first, n, nb)
                self.used += nb
            # the budget holds after every event (evictions come first)
            assert self.used <= self.budget
            self.peak = max(self.peak, self.used)

    def place(self, tickets, service):
        for tag, _, lv, slot, lid, _ in tickets:
            assert slot not in self.run
            l2, first, n, _ = self.lanes[lid]
            assert l2 == lv and first <= slot < first + n
            self.run[slot] = [tag, service[tag], lid]

    def step(self, m=None):
        """One round: launch every lane with samples, then finish them."""
        active = {v[2] for v in self.run.values()}
        for lid in active:
            assert self.s.set_inflight(lid, 1) == M.MG_OK
            if m:
                assert m.set_inflight(lid, 1) == M.MG_OK
        done = []
        for slot, v in list(self.run.items()):
            v[1] -= 1
            if v[1] == 0:
                done.append((slot, v[0]))
        for lid in active:
            assert self.s.set_inflight(lid, 0) == M.MG_OK
            if m:
                m.set_inflight(lid, 0)
        for slot, tag in done:
            assert self.s.release(slot) == M.MG_OK
            if m:
                assert m.release(slot) == M.MG_OK
            del self.run[slot]
        return [t for _, t in done]


def _mix(rng, n):
    return [int(x) for x in rng.choice(4, size=n, p=np.array([64, 16, 4, 1]) / 85)]


def test_open_on_demand_and_shared_budget():
    # budget 40: one level-1 lane (30) and one level-0 lane (10), or four level-0 lanes
    s = M.Sched([2, 1], [10, 30], 40, 16)
    for i, lv in enumerate([1, 0, 0, 0, 1]):
        assert s.submit(lv, 100 + i, i, float(i)) == M.MG_OK
    got = s.admit(8)
    assert [(t[0], t[3], t[4]) for t in got] == [(0, 0, 0), (1, 1, 1), (2, 2, 1)]
    assert s.events() == [(OPEN, 0, 1, 0, 1, 30), (OPEN, 1, 0, 1, 2, 10)]
    assert s.memory() == (40, 40, 2)
    # request 3 (level 0) waits for a level-0 slot; request 4 (level 1) for a level-1 slot
    assert s.admit(8) == [] and s.counts() == (2, 3)
    # the level-1 sample finishes: its lane is empty, but request 3 (level 0)
    # is first in the queue and takes its bytes for a second level-0 lane
    # (slots 3-4: the lowest free run of two)
    assert s.release(0) == M.MG_OK
    got = s.admit(8)
    assert [(t[0], t[3], t[4]) for t in got] == [(3, 3, 2)]
    assert s.events() == [(CLOSE, 0, 1, 0, 1, 30), (OPEN, 2, 0, 3, 2, 10)]
    # request 4 (level 1, no lane) reserves: the lane with the fewest samples
    # (lane 2) drains and takes no new sample, and nothing opens a lane
    assert s.admit(8) == [] and s.memory()[0] == 20
    assert s.submit(0, 105, 5) == M.MG_OK
    assert s.admit(8) == []
    assert s.release(3) == M.MG_OK
    got = s.admit(8)
    assert [(t[0], t[3], t[4]) for t in got] == [(4, 0, 3)]
    assert s.events() == [(CLOSE, 2, 0, 3, 2, 10), (OPEN, 3, 1, 0, 1, 30)]
    assert s.memory() == (40, 40, 2) and s.counts() == (1, 3)
    # the reservation is over: request 5 takes the next free level-0 slot
    assert s.release(1) == M.MG_OK
    assert [(t[0], t[3]) for t in s.admit(8)] == [(5, 1)]


def test_burst_at_one_level_takes_the_whole_budget():
    # memory another level leaves idle admits this level: eight level-0 lanes
    # of 2 slots fit 80 bytes, which two level-1 lanes would otherwise hold
    s = M.Sched([2, 1], [10, 40], 80, 64)
    for i in range(2):
        s.submit(1, i, i)
    assert len(s.admit(64)) == 2 and s.memory()[0] == 80
    for sl in (0, 1):
        s.release(sl)
    for i in range(16):
        s.submit(0, i, 100 + i)
    got = s.admit(64)
    assert len(got) == 16 and len({t[4] for t in got}) == 8
    assert s.memory() == (80, 80, 8)
    ev = s.events()
    assert sum(e[0] == CLOSE for e in ev) == 2 and sum(e[0] == OPEN for e in ev) == 10


def test_inflight_lanes_neither_admit_nor_evict():
    s = M.Sched([2, 1], [10, 20], 20, 16)
    s.submit(0, 0, 0)
    (t,) = s.admit(4)
    lane = t[4]
    s.set_inflight(lane, 1)
    s.submit(0, 1, 1)
    assert s.admit(4) == []      # a free slot, but the lane runs: wait
    s.set_inflight(lane, 0)
    assert [x[0] for x in s.admit(4)] == [1]
    s.release(t[3])
    s.release(t[3] + 1)
    s.set_inflight(lane, 1)      # empty, yet running: not evicted
    s.submit(1, 2, 2)
    assert s.admit(4) == []
    s.set_inflight(lane, 0)
    assert [x[0] for x in s.admit(4)] == [2]
    assert s.set_inflight(999, 1) == M.MG_EINVAL


def test_errors_and_capacity():
    s = M.Sched([2, 0, 1], [10, 0, 50], 40, 3)
    assert s.submit(3, 0, 0) == M.MG_EINVAL
    assert s.submit(-1, 0, 0) == M.MG_EINVAL
    assert s.submit(1, 0, 0) == M.MG_ENOMEM   # level not served
    assert s.submit(2, 0, 0) == M.MG_ENOMEM   # a lane larger than the budget
    for i in range(3):
        assert s.submit(0, i, i) == M.MG_OK
    assert s.submit(0, 9, 9) == M.MG_EBUSY
    assert s.release(0) == M.MG_EINVAL        # not busy
    assert s.release(99) == M.MG_EINVAL
    assert s.release(-1) == M.MG_EINVAL
    for bad in (([1, -1], [1, 1], 10, 4), ([1], [1], 10, 0), ([1], [0], 10, 4),
                ([1], [1], 0, 4), ([5000], [1], 10, 4)):
        with pytest.raises(M.MGError):
            M.Sched(*bad)
    assert len(s.admit(0)) == 0 and len(s.admit(2)) == 2   # max_out bounds one pass


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fake_executor_matches_policy_model(seed):
    rng = np.random.default_rng(seed)
    slots = [6, 3, 2, 1]
    nbytes = [6, 24, 96, 200]
    budget = [220, 240, 260, 300][seed]
    cap = 60
    s, m = M.Sched(slots, nbytes, budget, cap), Model(slots, nbytes, budget, cap)
    ex = Executor(s, budget)
    service, arrival, admitted = {}, collections.defaultdict(list), collections.defaultdict(list)
    finished, tag = set(), 0
    for step in range(600):
        for lv in _mix(rng, rng.poisson(1.5)):
            st = s.submit(lv, 1000 + tag, tag, float(step))
            assert st == m.submit(lv, 1000 + tag, tag, float(step))
            if st == M.MG_OK:
                arrival[lv].append(tag)
                service[tag] = int(rng.integers(1, 6)) * (1 + lv)
            tag += 1
        k = int(rng.integers(1, 12))
        got = s.admit(k)
        assert got == m.admit(k)
        ev = s.events()
        assert ev == m.take_events()
        ex.apply(ev)
        ex.place(got, service)
        for t in got:
            admitted[t[2]].append(t[0])
        finished.update(ex.step(m))
        assert s.counts() == (len(m.q), len(ex.run))
        assert s.memory()[:2] == (m.used, ex.peak) and m.used == ex.used
    for _ in range(10000):
        if not (ex.run or s.counts()[0]):
            break
        got = s.admit(64)
        assert got == m.admit(64)
        ev = s.events()
        assert ev == m.take_events()
        ex.apply(ev)
        ex.place(got, service)
        for t in got:
            admitted[t[2]].append(t[0])
        finished.update(ex.step(m))
    for lv in range(4):
        assert admitted[lv] == arrival[lv]  # arrival order within a level
    assert finished == set(service)          # every request was served
    assert ex.peak <= budget
    # the run went through evictions and reservations
    assert m.evictions > 0 and m.reservations > 0, (m.evictions, m.reservations)


def test_no_starvation_of_a_large_request():
    # a steady stream of small requests keeps level-0 lanes busy; a level-3
    # request (a lane that needs the whole budget) is still admitted, within
    # the service time of the samples resident when it arrived
    s = M.Sched([4, 1], [25, 100], 100, 1000)
    ex = Executor(s, 100)
    service, tag = {}, 0
    big = None
    for step in range(200):
        for _ in range(3):
            s.submit(0, tag, tag)
            service[tag] = 4
            tag += 1
        if step == 20:
            s.submit(1, 0, -1)
            service[-1] = 3
        got = s.admit(1000)
        ex.apply(s.events())
        ex.place(got, service)
        if any(t[0] == -1 for t in got):
            big = step
        ex.step()
    assert big is not None and 20 <= big <= 20 + 4 + 1


def test_work_conserving_with_room():
    # with room in the budget, an unbounded pass admits every queued request
    # whose level's lanes are not all in flight
    rng = np.random.default_rng(7)
    s = M.Sched([2, 2, 1], [1, 2, 4], 10 ** 6, 1000)
    busy = []
    for step in range(200):
        for _ in range(int(rng.integers(0, 4))):
            assert s.submit(int(rng.integers(0, 3)), 0, step) == M.MG_OK
        q = s.counts()[0]
        got = s.admit(1000)
        assert len(got) == q and s.counts()[0] == 0
        busy += [t[3] for t in got]
        for sl in list(busy):
            if rng.random() < 0.3:
                assert s.release(sl) == M.MG_OK
                busy.remove(sl)
    assert s.events()[0][0] == OPEN


# ---- property test: arbitrary operation sequences against the model -----------
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@st.composite
def _scenario(draw):
    levels = draw(st.integers(1, 4))
    slots = [draw(st.integers(0, 4)) for _ in range(levels)]
    nbytes = [draw(st.integers(1, 60)) for _ in range(levels)]
    budget = draw(st.integers(1, 150))
    cap = draw(st.integers(1, 12))
    ops = draw(st.lists(st.tuples(st.integers(0, 4), st.integers(0, 9), st.integers(0, 9)),
                        min_size=1, max_size=80))
    return slots, nbytes, budget, cap, ops


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(_scenario())
def test_random_operations_match_the_model(sc):
    slots, nbytes, budget, cap, ops = sc
    s, m = M.Sched(slots, nbytes, budget, cap), Model(slots, nbytes, budget, cap)
    busy, tag = [], 0
    for op, a, b in ops:
        if op == 0:    # submit (level a mod levels + 1 probes the bad-level error)
            lv = a % (len(slots) + 1)
            assert s.submit(lv, a, tag, 0.0) == m.submit(lv, a, tag, 0.0)
            tag += 1
        elif op == 1:  # admit
            got = s.admit(b)
            assert got == m.admit(b)
            busy += [t[3] for t in got]
        elif op == 2 and busy:  # release one busy slot
            sl = busy.pop(a % len(busy))
            assert s.release(sl) == M.MG_OK and m.release(sl) == M.MG_OK
        elif op == 3:  # toggle a lane in flight (only lanes the model knows)
            ids = sorted(m.lanes)
            if ids:
                lid = ids[a % len(ids)]
                flag = b & 1
                assert s.set_inflight(lid, flag) == m.set_inflight(lid, flag) == M.MG_OK
        else:          # release a slot that is not busy: refused by both
            free = [q for q in range(len(m.slot_busy)) if not m.slot_busy[q]]
            if free:
                sl = free[a % len(free)]
                assert s.release(sl) == m.release(sl) == M.MG_EINVAL
        assert s.events() == m.take_events()
        used, peak, lanes = s.memory()
        assert used == m.used <= budget and peak <= budget and lanes == len(m.lanes)
        assert s.counts() == (len(m.q), sum(m.slot_busy))
    # liveness: with every lane idle and every admitted sample finishing at
    # once, each round admits at least one request (a drain takes one round
    # to empty its lanes), so the queue empties within twice its length
    for lid in list(m.lanes):
        s.set_inflight(lid, 0)
    queued = s.counts()[0]
    for _ in range(2 * queued + 2):
        if s.counts()[0] == 0:
            break
        busy += [t[3] for t in s.admit(1000)]
        s.events()
        for sl in busy:
            assert s.release(sl) == M.MG_OK
        busy = []
    assert s.counts()[0] == 0
