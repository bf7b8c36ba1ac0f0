"""Serving loop on the CPU with a fake executor: admission by footprint in arrival order, the
budget is never exceeded, every study runs exactly its sweeps in consecutive ticks starting at
the tick after its admission, finished studies free their memory."""
import time

import pytest

from paper_1803_10045_amd import serve


class FakeRequest(serve.Request):
    def __init__(self, rid, arrival, n_sweeps, nbytes):
        self.rid, self.arrival, self.n_sweeps, self._nbytes = rid, arrival, n_sweeps, nbytes

    def footprint(self):
        return self._nbytes


class FakeExecutor:
    """Records every tick; time advances by a fixed amount per tick."""

    def __init__(self, tick_s=0.001):
        self.tick_s = tick_s
        self.ticks = []  # list of [(rid, sweep)]
        self.loaded = []
        self.released = []
        self.resident = {}
        self.max_resident = 0
        self.clock = 0.0

    def start(self):
        self.clock = 0.0

    def load(self, slot):
        self.loaded.append(slot.req.rid)
        self.resident[slot.req.rid] = slot.nbytes
        slot.state = "state"

    def run_tick(self, slots, lane=0):
        self.ticks.append([(s.req.rid, s.sweep) for s in slots])
        self.max_resident = max(self.max_resident, sum(self.resident.values()))
        self.clock += self.tick_s

    def mark(self, lane=0):
        return self.clock

    def done(self, token):
        return True

    def wait(self, token):
        return token

    def release(self, slot, keep):
        self.released.append(slot.req.rid)
        del self.resident[slot.req.rid]
        return ("result", slot.req.rid) if keep else None

    def collect_retired(self, force=True):
        pass

    def finish(self):
        pass


def run(reqs, budget):
    ex = FakeExecutor()
    comp, results, makespan, ticks = serve.serve(reqs, budget, ex, keep_results=True)
    return ex, comp, results, ticks


def test_every_study_runs_its_sweeps_in_consecutive_ticks():
    reqs = [FakeRequest(i, 0.002 * i, n_sweeps=3 + i % 4, nbytes=10) for i in range(12)]
    ex, comp, results, ticks = run(reqs, budget=1000)
    assert sorted(c.rid for c in comp) == list(range(12))
    assert set(results) == set(range(12))
    for r in reqs:
        seen = [(t, sw) for t, tick in enumerate(ex.ticks) for rid, sw in tick if rid == r.rid]
        assert [sw for _, sw in seen] == list(range(r.n_sweeps))
        ts = [t for t, _ in seen]
        assert ts == list(range(ts[0], ts[0] + r.n_sweeps))  # consecutive ticks, no gaps
    assert ticks == len(ex.ticks)


def test_admission_respects_budget_and_arrival_order():
    sizes = [60, 30, 50, 20, 70, 10, 40]
    reqs = [FakeRequest(i, 0.0, n_sweeps=2 + i % 3, nbytes=s) for i, s in enumerate(sizes)]
    ex, comp, _, _ = run(reqs, budget=100)
    assert ex.max_resident <= 100
    assert ex.loaded == list(range(len(sizes)))  # first come, first served
    assert sorted(ex.released) == list(range(len(sizes)))
    # studies overlap on the device: some tick holds more than one study
    assert max(len(t) for t in ex.ticks) > 1


def test_late_arrivals_join_running_ticks():
    reqs = [FakeRequest(0, 0.0, n_sweeps=400, nbytes=10), FakeRequest(1, 0.05, n_sweeps=3, nbytes=10)]
    ex = FakeExecutor()
    # slow ticks so that study 0 is still running when study 1 arrives
    orig = ex.run_tick

    def slow(slots, lane=0):
        time.sleep(0.0005)
        orig(slots, lane)

    ex.run_tick = slow
    comp, _, _, _ = serve.serve(reqs, 100, ex)
    both = [t for t in ex.ticks if {rid for rid, _ in t} == {0, 1}]
    assert len(both) == 3  # study 1 ran all its sweeps next to study 0
    done = {c.rid: c for c in comp}
    assert done[1].finished < done[0].finished


def test_request_larger_than_budget_is_rejected():
    with pytest.raises(ValueError, match="more than the whole budget"):
        run([FakeRequest(0, 0.0, 1, 500)], budget=100)


def test_latency_summary():
    comp = [serve.Completion(i, 0.0, 0.0, float(i + 1)) for i in range(100)]
    s = serve.latency_summary(comp)
    assert s["p50_s"] == pytest.approx(50.5)
    assert s["p99_s"] == pytest.approx(99.01)
    assert s["max_s"] == 100.0


class TwoLaneExecutor(FakeExecutor):
    lanes = [None, None]


def test_lanes_run_independently():
    """Large studies (lane 1) never share a tick with small ones (lane 0), and a small study that
    arrives after a large one finishes first."""
    reqs = [FakeRequest(0, 0.0, n_sweeps=300, nbytes=50), FakeRequest(1, 0.02, n_sweeps=3, nbytes=10),
            FakeRequest(2, 0.02, n_sweeps=4, nbytes=10)]
    ex = TwoLaneExecutor()
    orig = ex.run_tick

    def slow(slots, lane=0):
        time.sleep(0.0002 if lane == 0 else 0.0005)
        orig(slots, lane)

    ex.run_tick = slow
    comp, _, _, _ = serve.serve(reqs, 100, ex, lane_of=lambda r: 1 if r.rid == 0 else 0,
                                small_in_flight_beside_large=1)
    for t in ex.ticks:
        rids = {rid for rid, _ in t}
        assert rids == {0} or 0 not in rids
    done = {c.rid: c for c in comp}
    assert done[1].finished < done[0].finished and done[2].finished < done[0].finished


class TimedTwoLaneExecutor(FakeExecutor):
    """Ticks run asynchronously: a tick takes `dur[lane]` seconds of a simulated GPU per lane and
    is in flight until then (done() polls the wall clock)."""
    lanes = [None, None]

    def __init__(self, dur):
        super().__init__()
        self.dur = dur
        self.busy_until = [0.0, 0.0]
        self.spans = []  # (lane, start, end)

    def start(self):
        self.t0 = time.perf_counter()

    def run_tick(self, slots, lane=0):
        super().run_tick(slots, lane)
        now = time.perf_counter() - self.t0
        start = max(now, self.busy_until[lane])
        self.busy_until[lane] = start + self.dur[lane]
        self.spans.append((lane, start, self.busy_until[lane]))

    def mark(self, lane=0):
        return self.busy_until[lane]

    def done(self, token):
        return time.perf_counter() - self.t0 >= token

    def wait(self, token):
        while not self.done(token):
            time.sleep(0.0001)
        return token


def test_small_lane_yields_to_a_large_study():
    """With small_in_flight_beside_large = 0 no small tick is enqueued while a large tick is in
    flight, so a small study that arrives during a large one starts after it; with 1 it runs
    beside it and finishes first."""
    def run_cap(cap):
        reqs = [FakeRequest(0, 0.0, n_sweeps=5, nbytes=50), FakeRequest(1, 0.005, n_sweeps=2, nbytes=10)]
        ex = TimedTwoLaneExecutor(dur=[0.001, 0.01])
        comp, _, _, _ = serve.serve(reqs, 100, ex, lane_of=lambda r: 1 if r.rid == 0 else 0,
                                    small_in_flight_beside_large=cap)
        return ex, {c.rid: c for c in comp}

    ex, done = run_cap(0)
    large_end = max(e for lane, _, e in ex.spans if lane == 1)
    assert min(st for lane, st, _ in ex.spans if lane == 0) >= large_end
    assert done[0].finished <= done[1].finished
    ex, done = run_cap(1)
    assert done[1].finished < done[0].finished


def test_lane_batch_runs_oldest_first():
    reqs = [FakeRequest(i, 0.0, n_sweeps=3, nbytes=10) for i in range(3)]
    ex = TwoLaneExecutor()
    comp, _, _, _ = serve.serve(reqs, 100, ex, lane_of=lambda r: 1, lane_batch=[0, 1])
    assert all(len(t) == 1 for t in ex.ticks)
    assert [t[0][0] for t in ex.ticks] == [0, 0, 0, 1, 1, 1, 2, 2, 2]


def test_small_studies_wait_before_running_beside_a_large_one():
    """With small_wait_beside_large = W a small tick starts beside a large tick only once the
    oldest small study has waited W since its arrival; without a large tick it starts at once."""
    def run_wait(wait):
        reqs = [FakeRequest(0, 0.0, n_sweeps=8, nbytes=50), FakeRequest(1, 0.005, n_sweeps=2, nbytes=10)]
        ex = TimedTwoLaneExecutor(dur=[0.001, 0.01])
        comp, _, _, _ = serve.serve(reqs, 100, ex, lane_of=lambda r: 1 if r.rid == 0 else 0,
                                    small_in_flight_beside_large=1, small_wait_beside_large=wait)
        return ex, {c.rid: c for c in comp}

    ex, done = run_wait(0.03)
    first_small = min(st for lane, st, _ in ex.spans if lane == 0)
    assert first_small >= 0.005 + 0.03 - 1e-3  # waited, although a large tick was in flight
    assert first_small < max(e for lane, _, e in ex.spans if lane == 1)  # but ran beside the large study
    ex, done = run_wait(0.0)
    assert min(st for lane, st, _ in ex.spans if lane == 0) < 0.005 + 0.01


def test_lane_resident_cap_holds_requests_in_order_and_lets_other_lanes_pass():
    """With at most one resident study in lane 1, a second lane-1 request is held (in order)
    while later lane-0 requests are admitted; it is admitted once the first has finished."""
    reqs = [FakeRequest(0, 0.0, 2, 10), FakeRequest(1, 0.0, 2, 10), FakeRequest(2, 0.0, 1, 1),
            FakeRequest(3, 0.0, 1, 10), FakeRequest(4, 0.0, 1, 1)]
    lane = {0: 1, 1: 1, 2: 0, 3: 1, 4: 0}
    sched = serve.Scheduler(100, lambda r: lane[r.rid], 2, lane_resident=[0, 1])
    for r in reqs:
        sched.arrive(r)
    assert [s.req.rid for s in sched.admit(0.0)] == [0, 2, 4]
    assert [r.rid for r in sched.queue] == [1, 3]
    first = sched.tick(1)
    assert [s.req.rid for s in first] == [0]
    sched.advance(first)
    assert sched.admit(0.0) == []  # study 0 still has a sweep to run
    for s in sched.advance(sched.tick(1)):
        sched.release(s)
    assert [s.req.rid for s in sched.admit(0.0)] == [1]
    assert [r.rid for r in sched.queue] == [3]


def test_lane_resident_cap_reserves_the_budget_of_held_requests():
    """A held request keeps its place in memory: a later request of another lane passes it only
    if the budget also has room for the held one."""
    reqs = [FakeRequest(0, 0.0, 1, 40), FakeRequest(1, 0.0, 1, 40), FakeRequest(2, 0.0, 1, 30),
            FakeRequest(3, 0.0, 1, 10)]
    lane = {0: 1, 1: 1, 2: 0, 3: 0}
    sched = serve.Scheduler(100, lambda r: lane[r.rid], 2, lane_resident=[0, 1])
    for r in reqs:
        sched.arrive(r)
    # 40 used; request 1 (40) held; request 2 (30) would leave no room for it: it waits, and so
    # does request 3 behind it (first come, first served)
    assert [s.req.rid for s in sched.admit(0.0)] == [0]
    assert [r.rid for r in sched.queue] == [1, 2, 3]
    for s in sched.advance(sched.tick(1)):
        sched.release(s)
    assert [s.req.rid for s in sched.admit(0.0)] == [1, 2, 3]
    assert sched.used == 80


def test_served_with_large_resident_cap_runs_every_study():
    """The serving loop with one resident large study at a time: every study runs its sweeps,
    and at most one lane-1 study is resident at any tick."""
    reqs = [FakeRequest(i, 0.0, 3, 10 if i % 3 == 0 else 1) for i in range(9)]
    ex = FakeExecutor()
    ex.lanes = [None, None]
    resident_large = []
    run_tick = ex.run_tick

    def tick(slots, lane=0):
        resident_large.append(sum(1 for rid in ex.resident if rid % 3 == 0))
        run_tick(slots, lane)

    ex.run_tick = tick
    comp, _, _, _ = serve.serve(reqs, 1000, ex, lane_of=lambda r: 1 if r.rid % 3 == 0 else 0, large_resident=1)
    assert sorted(c.rid for c in comp) == list(range(9))
    assert max(resident_large) == 1
    for rid in range(9):
        assert sum(1 for t in ex.ticks for r, _ in t if r == rid) == 3
