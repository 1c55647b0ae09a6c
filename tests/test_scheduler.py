"""Serving scheduler logic with a scripted executor (CPU only): admission by
output footprint, the budget is never exceeded, oversize requests are
rejected, FIFO progress, every admitted request completes."""
import itertools

import numpy as np
import pytest

from paper_2408_14302_amd.serve import Request, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4       # every look at the clock advances it a little
        return self.t


class FakeExecutor:
    """Completes a batch after a fixed number of polls; records what ran together."""

    def __init__(self, polls=3):
        self.polls = polls
        self.launched = []
        self.live = {}
        self.ids = itertools.count()

    def launch(self, slot, batch):
        h = next(self.ids)
        self.live[h] = self.polls
        self.launched.append((slot, [r.rid for r in batch]))
        return h

    def done(self, h):
        self.live[h] -= 1
        return self.live[h] <= 0

    def release(self, slot, batch):
        pass


def make_reqs(n, seed=0, keys=(64, 128), big=None):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(1e-3)
        k = int(rng.choice(keys))
        fp = int(rng.integers(1, 50)) * 1000
        if big is not None and i in big:
            fp = 10 ** 12
        out.append(Request(rid=i, arrival=t, n=fp // 4, scale_key=k, hop=1, footprint=fp))
    return out


class BudgetWatch(Scheduler):
    def admit(self, now):
        r = super().admit(now)
        assert self.inflight_bytes <= self.budget
        return r


def test_all_complete_and_budget_respected():
    ex = FakeExecutor()
    sch = BudgetWatch(ex, budget_bytes=120_000, slots=3, max_batch=8, clock=FakeClock())
    reqs = make_reqs(300)
    st = sch.run(reqs, t0=0.0)
    assert st.admitted == 300 and st.rejected == 0
    assert len(st.latencies_ms) == 300
    assert st.max_inflight_bytes <= 120_000
    assert all(r.completed is not None for r in reqs)
    # batches are homogeneous in scale set and within max_batch
    by = {r.rid: r for r in reqs}
    for slot, ids in ex.launched:
        assert 1 <= len(ids) <= 8
        assert len({by[i].scale_key for i in ids}) == 1
        assert 0 <= slot < 3


def test_oversize_rejected_without_blocking():
    ex = FakeExecutor()
    sch = Scheduler(ex, budget_bytes=100_000, slots=2, max_batch=4, clock=FakeClock())
    reqs = make_reqs(50, seed=1, big={3, 17})
    st = sch.run(reqs, t0=0.0)
    assert st.rejected == 2 and st.admitted == 48
    assert reqs[3].rejected and reqs[17].rejected and reqs[3].completed is None


def test_fifo_within_scale_set():
    """Requests of one scale set are admitted in arrival order."""
    ex = FakeExecutor(polls=5)
    sch = Scheduler(ex, budget_bytes=60_000, slots=2, max_batch=3, clock=FakeClock())
    reqs = make_reqs(120, seed=2)
    sch.run(reqs, t0=0.0)
    for key in (64, 128):
        adm = [r.admitted for r in sorted(reqs, key=lambda r: r.rid) if r.scale_key == key]
        assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_overlap_uses_several_slots():
    ex = FakeExecutor(polls=50)
    sch = Scheduler(ex, budget_bytes=10 ** 9, slots=4, max_batch=2, clock=FakeClock())
    reqs = make_reqs(100, seed=3)
    st = sch.run(reqs, t0=0.0)
    assert st.busy_slots_max > 1


def test_rejects_bad_parameters():
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(), budget_bytes=0)
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(), budget_bytes=10, slots=0)
