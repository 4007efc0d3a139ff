"""CPU tests of the serving form's admission scheduler (mg_sched_*, host only).

The policy: one queue in arrival order; level l owns a fixed pool of slots;
each admission pass walks the queue from its head and gives every request
whose level has a free slot the lowest free slot of that level.  The tests
drive the native scheduler with a fake executor (service times drawn on the
host) and compare every admission against a plain Python model of that
policy, and check the invariants that follow from it.
"""
import collections

import numpy as np
import pytest

import paper_1607_03252_amd as M


class Model:
    """The admission policy written out directly (independent of the C++)."""

    def __init__(self, slots, cap):
        self.first = np.concatenate([[0], np.cumsum(slots)]).astype(int)
        self.busy = [False] * int(self.first[-1])
        self.cap = cap
        self.q = []

    def submit(self, level, seed, tag, t):
        if level < 0 or level >= len(self.first) - 1:
            return M.MG_EINVAL
        if len(self.q) >= self.cap:
            return M.MG_EBUSY
        self.q.append((tag, seed, level, -1, t))
        return M.MG_OK

    def admit(self, max_out):
        out, keep = [], []
        for r in self.q:
            lv = r[2]
            free = [s for s in range(self.first[lv], self.first[lv + 1]) if not self.busy[s]]
            if free and len(out) < max_out:
                self.busy[free[0]] = True
                out.append((r[0], r[1], lv, free[0], r[4]))
            else:
                keep.append(r)
        self.q = keep
        return out

    def release(self, slot):
        if not (0 <= slot < len(self.busy)) or not self.busy[slot]:
            return M.MG_EINVAL
        self.busy[slot] = False
        return M.MG_OK


def test_fifo_within_level_and_no_head_of_line_blocking():
    s = M.Sched([1, 1], 16)
    for i, lv in enumerate([1, 1, 0, 1, 0]):
        assert s.submit(lv, 100 + i, i, float(i)) == M.MG_OK
    got = s.admit(8)
    # level 1 takes request 0 (slot 1); request 1 (level 1) waits but does not
    # hold back request 2 (level 0, slot 0)
    assert [(t[0], t[3]) for t in got] == [(0, 1), (2, 0)]
    assert s.counts() == (3, 2)
    assert s.release(1) == M.MG_OK
    assert [(t[0], t[3]) for t in s.admit(8)] == [(1, 1)]
    assert s.release(0) == M.MG_OK
    assert [(t[0], t[3]) for t in s.admit(8)] == [(4, 0)]
    assert s.counts() == (1, 2)


def test_errors_and_capacity():
    s = M.Sched([2, 0, 1], 3)
    assert s.submit(3, 0, 0) == M.MG_EINVAL
    assert s.submit(-1, 0, 0) == M.MG_EINVAL
    for i in range(3):
        assert s.submit(1, i, i) == M.MG_OK  # level 1 has no slots: they wait
    assert s.submit(0, 9, 9) == M.MG_EBUSY
    assert s.admit(8) == []
    assert s.release(0) == M.MG_EINVAL  # not busy
    assert s.release(99) == M.MG_EINVAL
    assert s.release(-1) == M.MG_EINVAL
    with pytest.raises(M.MGError):
        M.Sched([1, -1], 4)
    with pytest.raises(M.MGError):
        M.Sched([1], 0)


def test_lowest_free_slot_and_ranges():
    s = M.Sched([3, 2], 64)
    for i in range(5):
        s.submit(0 if i < 3 else 1, i, i)
    got = s.admit(16)
    assert [t[3] for t in got] == [0, 1, 2, 3, 4]
    assert s.release(1) == M.MG_OK and s.release(0) == M.MG_OK
    s.submit(0, 7, 7)
    s.submit(0, 8, 8)
    assert [t[3] for t in s.admit(16)] == [0, 1]
    # max_out bounds one pass
    s2 = M.Sched([4], 64)
    for i in range(4):
        s2.submit(0, i, i)
    assert len(s2.admit(3)) == 3 and len(s2.admit(3)) == 1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fake_executor_matches_policy_model(seed):
    rng = np.random.default_rng(seed)
    slots = [5, 3, 2, 1]
    cap = 40
    s, m = M.Sched(slots, cap), Model(slots, cap)
    service = {}            # tag -> steps still to run
    running = {}            # slot -> tag
    arrival_order = collections.defaultdict(list)
    admit_order = collections.defaultdict(list)
    finished = set()
    tag = 0
    for step in range(400):
        for _ in range(rng.poisson(1.2)):
            lv = int(rng.choice(4, p=[64 / 85, 16 / 85, 4 / 85, 1 / 85]))
            st = s.submit(lv, 1000 + tag, tag, float(step))
            assert st == m.submit(lv, 1000 + tag, tag, float(step))
            if st == M.MG_OK:
                arrival_order[lv].append(tag)
                service[tag] = int(rng.integers(1, 6)) * (1 + lv)
            tag += 1
        k = int(rng.integers(1, 12))
        got = s.admit(k)
        assert got == m.admit(k)
        for t in got:
            assert t[3] not in running
            lo = sum(slots[:t[2]])
            assert lo <= t[3] < lo + slots[t[2]]
            running[t[3]] = t[0]
            admit_order[t[2]].append(t[0])
        # the fake executor: every resident request runs one step
        for sl, tg in list(running.items()):
            service[tg] -= 1
            if service[tg] == 0:
                assert s.release(sl) == M.MG_OK and m.release(sl) == M.MG_OK
                del running[sl]
                finished.add(tg)
        q, b = s.counts()
        assert b == len(running) and q == len(m.q)
    # drain
    while running or s.counts()[0]:
        got = s.admit(64)
        assert got == m.admit(64)
        for t in got:
            running[t[3]] = t[0]
            admit_order[t[2]].append(t[0])
        for sl, tg in list(running.items()):
            service[tg] -= 1
            if service[tg] == 0:
                s.release(sl)
                m.release(sl)
                del running[sl]
                finished.add(tg)
    for lv in range(4):
        assert admit_order[lv] == arrival_order[lv]  # arrival order within a level
    assert finished == set(service)


def test_work_conserving():
    # an unbounded pass admits, per level, min(requests of that level queued,
    # free slots of that level)
    rng = np.random.default_rng(7)
    pools = [2, 2, 1]
    s = M.Sched(pools, 1000)
    queued = [0, 0, 0]
    busy = {}  # slot -> level
    for step in range(300):
        for _ in range(int(rng.integers(0, 4))):
            lv = int(rng.integers(0, 3))
            assert s.submit(lv, 0, step) == M.MG_OK
            queued[lv] += 1
        free = [pools[lv] - sum(1 for v in busy.values() if v == lv) for lv in range(3)]
        got = s.admit(1000)
        per = collections.Counter(t[2] for t in got)
        for lv in range(3):
            assert per[lv] == min(queued[lv], free[lv])
            queued[lv] -= per[lv]
        for t in got:
            busy[t[3]] = t[2]
        assert s.counts() == (sum(queued), len(busy))
        for sl in list(busy):
            if rng.random() < 0.3:
                assert s.release(sl) == M.MG_OK
                del busy[sl]
