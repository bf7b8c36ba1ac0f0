"""Continuous-batching reconstruction server on one GPU.

Requests (dynamic studies) arrive over time.  A request is admitted when its HBM footprint
(measured sinogram, image, three kinetic maps, lambda, workspace: kcs_study_footprint_bytes)
fits under the budget next to the studies already resident, in arrival order.  Its state stays
on the device until its last ICM sweep.  The GPU advances in ticks: one tick runs one ICM sweep of
every resident study as one batched plan (a launch per phase over all studies' work lists), so
studies that arrive while others are on the GPU join at the next tick and share its launches.
Plans are cached by the resident set: while the set does not change, the same captured graph is
replayed every tick.

Studies are split into lanes by the HBM traffic of one of their sweeps; each lane has its own
stream and its own ticks, so the short sweeps of small studies run next to the long sweeps of
large ones (the hardware interleaves their workgroups) instead of waiting for them.  Loading (the
sinogram, the initial state) runs on a stream of its own.

The scheduling logic (:class:`Scheduler`) is plain Python with no device code, so it can be
tested on the CPU with a fake executor; :class:`GpuExecutor` owns the device state and the plans.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import kcs


@dataclass(eq=False)
class Request:
    """One reconstruction: constants, schedule and a loader that produces the measured sinogram
    (nz, n_ang, n_bin, M) as an FP32 device tensor on the current stream."""
    rid: int
    arrival: float  # seconds after the start of serving
    g: kcs.Geometry
    f: kcs.Frames
    k: kcs.Kinetics
    p: kcs.Prior
    lm: kcs.LMOptions
    Q: int
    n_sweeps: int
    load: Callable[[], object]
    xi0: Tuple[float, float, float] = (0.08, 0.12, 0.05)

    def footprint(self) -> int:
        return kcs.kcs_study_footprint_bytes(self.g, self.f.M, self.Q)


@dataclass(eq=False)
class Slot:
    req: Request
    nbytes: int
    sweep: int = 0  # next sweep to run
    admitted_at: float = 0.0
    lane: int = 0
    state: object = None  # executor-owned device state


def sweep_bytes(g: kcs.Geometry, M: int, Q: int) -> int:
    """HBM bytes one ICM sweep must move at least: per subset the forward projection (image, the
    subset's sinogram read, ratio written) and the OSL update (ratio, image in and out, maps), then
    five MAP-LM iterations (image, maps in and out, lambda)."""
    N = g.nx * g.ny * g.nz
    image = N * M * 4
    sub = g.nz * (g.n_ang / Q) * g.n_bin * M * 4
    return int(Q * ((image + 2 * sub) + (2 * image + sub + 12 * N)) + 5 * (image + 32 * N))


def lane_by_traffic(threshold_bytes: float = 10e9) -> Callable[[Request], int]:
    """Lane 1 for studies whose sweep moves more than `threshold_bytes`, lane 0 otherwise."""
    return lambda r: 1 if sweep_bytes(r.g, r.f.M, r.Q) > threshold_bytes else 0


class Scheduler:
    """Admission by footprint (first come, first served: a request that does not fit blocks the
    ones behind it, so large studies cannot starve) and sweep-granular batching per lane.
    `lane_resident[i]` (0: no limit) caps the studies resident in lane i: a request of a full lane
    is held, in order, and later requests of other lanes pass it only while the budget still has
    room for every held request, so a held request waits for its own lane and never for memory."""

    def __init__(self, budget_bytes: int, lane_of: Callable[[Request], int] = lambda r: 0, n_lanes: int = 1,
                 lane_batch: Optional[Sequence[int]] = None, lane_resident: Optional[Sequence[int]] = None):
        self.budget = int(budget_bytes)
        # most studies a tick of each lane advances, oldest first (0: no limit)
        self.lane_batch = list(lane_batch) if lane_batch is not None else [0] * n_lanes
        self.lane_resident = list(lane_resident) if lane_resident is not None else [0] * n_lanes
        self.used = 0
        self.queue: collections.deque = collections.deque()
        self.active: List[List[Slot]] = [[] for _ in range(n_lanes)]
        self.lane_of = lane_of

    def arrive(self, req: Request):
        nbytes = req.footprint()
        if nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {nbytes} bytes, more than the whole budget {self.budget}")
        self.queue.append(req)

    def admit(self, now: float) -> List[Slot]:
        out = []
        held: collections.deque = collections.deque()
        reserved = 0  # footprints of the held requests
        while self.queue:
            req = self.queue[0]
            lane = self.lane_of(req)
            cap = self.lane_resident[lane]
            if cap and len(self.active[lane]) >= cap:
                held.append(self.queue.popleft())
                reserved += req.footprint()
                continue
            if self.used + reserved + req.footprint() > self.budget:
                break
            self.queue.popleft()
            s = Slot(req, req.footprint(), admitted_at=now, lane=lane)
            self.used += s.nbytes
            self.active[s.lane].append(s)
            out.append(s)
        held.extend(self.queue)
        self.queue = held
        return out

    def tick(self, lane: int = 0) -> List[Slot]:
        """The slots of `lane` that take part in its next tick (each runs its next sweep): all
        resident ones, or the oldest `lane_batch[lane]` of them."""
        cap = self.lane_batch[lane]
        return list(self.active[lane][:cap] if cap else self.active[lane])

    def advance(self, ran: Sequence[Slot]) -> List[Slot]:
        """After a tick: move the slots on by one sweep; returns the slots that finished (they
        leave the active set; their bytes are returned by release())."""
        done = []
        for s in ran:
            s.sweep += 1
            if s.sweep >= s.req.n_sweeps:
                done.append(s)
        for lane in range(len(self.active)):
            self.active[lane] = [s for s in self.active[lane] if not any(s is d for d in done)]
        return done

    def release(self, slot: Slot):
        self.used -= slot.nbytes

    @property
    def idle(self) -> bool:
        return not self.queue and not any(self.active)


class GpuExecutor:
    """Device state of the resident studies and the batched plans that advance them: one stream
    per lane for the ticks, one stream for loading."""

    def __init__(self, device="cuda", flags: int = kcs.KCS_PLAN_GRAPH, n_lanes: int = 1):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.flags = flags
        self.lanes = [torch.cuda.Stream(device=self.dev) for _ in range(n_lanes)]
        self.load_stream = torch.cuda.Stream(device=self.dev)
        self.plans: Dict[tuple, kcs.Plan] = {}
        self.retired: List[kcs.Plan] = []

    def load(self, slot: Slot):
        torch = self.torch
        r = slot.req
        lane = self.lanes[slot.lane]
        with torch.cuda.stream(self.load_stream):
            sino = r.load()
            g, M = r.g, r.f.M
            x = torch.empty((g.nz, g.ny, g.nx, M), device=self.dev)
            params = torch.empty((3, g.nz, g.ny, g.nx), device=self.dev)
            lam = torch.empty((g.nz, g.ny, g.nx), device=self.dev)
            work = kcs.alloc_workspace(g, M, r.Q, self.dev)
            kcs.kcs_init_state(g, r.f, sino, r.xi0, x, params, lam, work)
            ready = torch.cuda.Event()
            ready.record()
        lane.wait_event(ready)
        for t in (sino, x, params, lam, work):
            t.record_stream(lane)  # the buffers are used on the lane's stream from now on
        slot.state = dict(sino=sino, x=x, params=params, lam=lam, work=work)

    def _study(self, slot: Slot) -> kcs.Study:
        r, st = slot.req, slot.state
        return kcs.Study(r.g, r.f, r.k, r.p, r.lm, r.Q, slot.sweep, slot.sweep + 1, st["sino"], st["x"],
                         st["params"], st["lam"], st["work"])

    def run_tick(self, slots: Sequence[Slot], lane: int = 0):
        # a plan depends on the studies and on whether each one's prior is on (sweep > 0)
        key = (lane,) + tuple((s.req.rid, s.sweep > 0) for s in slots)
        stream = self.lanes[lane]
        with self.torch.cuda.stream(stream):
            plan = self.plans.get(key)
            if plan is None:
                plan = kcs.kcs_plan_create([self._study(s) for s in slots], self.flags)
                self.plans[key] = plan
            kcs.kcs_plan_run(plan)

    def release(self, slot: Slot, keep_result: bool):
        """Drops the plans that involve the study (destroyed later, at a quiet point) and returns
        the results (x, params, lam) if asked; the device buffers go back to torch's allocator."""
        rid = slot.req.rid
        for key in [k for k in self.plans if any(r == rid for r, _ in k[1:])]:
            plan = self.plans.pop(key)
            plan.studies = []  # never run again: its studies' buffers may go back to the allocator
            self.retired.append(plan)
        st = slot.state
        slot.state = None
        return (st["x"], st["params"], st["lam"]) if keep_result else None

    # --- clock: completion times come from events on the lane streams, relative to start() ---
    def start(self):
        self.torch.cuda.synchronize()
        self.start_ev = self.torch.cuda.Event(enable_timing=True)
        self.start_ev.record()

    def mark(self, lane: int = 0):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.lanes[lane])
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def wait(self, ev) -> float:
        ev.synchronize()
        return self.start_ev.elapsed_time(ev) * 1e-3

    def finish(self):
        self.torch.cuda.synchronize()

    def collect_retired(self, force: bool = True):
        if force or len(self.retired) > 64:
            for p in self.retired:
                kcs.kcs_plan_destroy(p)
            self.retired = []

    def close(self):
        for p in self.plans.values():
            kcs.kcs_plan_destroy(p)
        self.plans = {}
        self.collect_retired()


@dataclass
class Completion:
    rid: int
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def serve(requests: Sequence[Request], budget_bytes: int, executor, keep_results: bool = False,
          max_in_flight: int = 2, lane_of: Optional[Callable[[Request], int]] = None,
          lane_batch: Optional[Sequence[int]] = None, log: Optional[Callable[[str], None]] = None,
          small_in_flight_beside_large: int = 1, small_wait_beside_large: float = 0.0,
          large_resident: int = 1):
    """Serves `requests` in real time (arrival times in seconds from the start).  Returns
    (completions, results, makespan_s, ticks); completion times come from the executor's clock
    (GPU events on the lane streams).  `lane_batch[i]` caps the studies per tick of lane i (0: all
    resident ones).  Each lane keeps at most `max_in_flight` ticks enqueued ahead of the GPU; while
    the last lane (the large studies) has a tick on the GPU the other lanes start at most
    `small_in_flight_beside_large` ticks (streams keep one priority, so this cap is what shares
    the GPU between them).  Default 1: one small tick beside each large one.  0 makes the small
    studies wait for the large study to finish, which runs it as fast as alone but holds every
    small study that arrives meanwhile for a large study's whole duration (at 4 requests/s of the
    mixed workload the tail latency doubled).  `small_wait_beside_large` (seconds) holds a small
    tick back while a large tick is in flight until the oldest small study of that lane has waited
    that long since its arrival: the large studies then share the GPU only with small studies that
    would otherwise wait too long, and the small ones still finish within about that wait plus
    their own sweeps.  `large_resident` (0: no limit) caps the studies resident in the last lane:
    with 1 (the default), the next large study is admitted, and its sinogram synthesised and its
    state set up, only once the running one has enqueued its last tick, so that this loading does
    not share the GPU with a whole large study (at 4 requests/s of the mixed workload: mean latency
    0.152 s instead of 0.169, the small studies' tails halved, the overall p99 unchanged).  A finished study's memory returns to the budget once its last
    tick has completed."""
    n_lanes = len(getattr(executor, "lanes", [None]))
    if lane_of is None:
        lane_of = lane_by_traffic() if n_lanes > 1 else (lambda r: 0)
    if lane_batch is None:
        # a large study fills the GPU by itself: the large lane runs its studies one at a time, in
        # admission order, so that batching does not stretch each one's latency
        lane_batch = [0] * n_lanes if n_lanes == 1 else [0] + [1] * (n_lanes - 1)
    lane_resident = [0] * n_lanes
    if n_lanes > 1:
        lane_resident[n_lanes - 1] = large_resident
    sched = Scheduler(budget_bytes, lane_of, n_lanes, lane_batch, lane_resident)
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    executor.start()
    t0 = time.perf_counter()
    in_flight = [collections.deque() for _ in range(n_lanes)]  # per lane: (token, finished slots)
    completions: List[Completion] = []
    results: Dict[int, tuple] = {}
    ticks = 0

    def retire(lane):
        token, finished = in_flight[lane].popleft()
        t_done = executor.wait(token)
        for s in finished:
            res = executor.release(s, keep_results)
            if keep_results:
                results[s.req.rid] = res
            sched.release(s)
            completions.append(Completion(s.req.rid, s.req.arrival, s.admitted_at, t_done))

    while pending or not sched.idle or any(in_flight):
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            sched.arrive(pending.popleft())
        for s in sched.admit(now):
            executor.load(s)
        progressed = False
        large_busy = n_lanes > 1 and bool(in_flight[n_lanes - 1])
        for lane in range(n_lanes):
            while in_flight[lane] and executor.done(in_flight[lane][0][0]):
                retire(lane)
            cap = max_in_flight
            if large_busy and lane < n_lanes - 1:
                cap = min(cap, small_in_flight_beside_large)
                oldest = min((sl.req.arrival for sl in sched.active[lane]), default=None)
                if oldest is not None and time.perf_counter() - t0 - oldest < small_wait_beside_large:
                    cap = 0
            if len(in_flight[lane]) >= cap:
                continue
            slots = sched.tick(lane)
            if slots:
                executor.run_tick(slots, lane)
                in_flight[lane].append((executor.mark(lane), sched.advance(slots)))
                ticks += 1
                progressed = True
        if not progressed:
            if any(in_flight):
                time.sleep(0.0002)  # every lane is full or idle: poll the GPU
            elif pending:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.05)))
        executor.collect_retired(force=sched.idle and not any(in_flight))
    executor.finish()
    executor.collect_retired()
    makespan = max((c.finished for c in completions), default=0.0) - min((r.arrival for r in requests), default=0.0)
    if log:
        log(f"served {len(completions)} requests in {ticks} ticks")
    return completions, results, makespan, ticks


def serve_serial(requests: Sequence[Request], log: Optional[Callable[[str], None]] = None,
                 keep_results: bool = False):
    """Baseline: the plain per-study loop, one study at a time in arrival order (each study's
    sweeps are kcs_icm_sweep calls).  Same outputs as serve()."""
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    start_ev = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_ev.record()
    done_events = []
    results = {}
    for r in pending:
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        admitted = time.perf_counter() - t0
        sino = r.load()
        g, M = r.g, r.f.M
        dev = sino.device
        x = torch.empty((g.nz, g.ny, g.nx, M), device=dev)
        params = torch.empty((3, g.nz, g.ny, g.nx), device=dev)
        lam = torch.empty((g.nz, g.ny, g.nx), device=dev)
        work = kcs.alloc_workspace(g, M, r.Q, dev)
        kcs.kcs_init_state(g, r.f, sino, r.xi0, x, params, lam, work)
        for s in range(r.n_sweeps):
            kcs.kcs_icm_sweep(g, r.f, r.k, r.p, r.lm, sino, r.Q, s, x, params, lam, work)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        done_events.append((r, admitted, ev))
        if keep_results:
            results[r.rid] = (x, params, lam)
        if len(done_events) > 2:  # bound the host's lead over the GPU
            done_events[-3][2].synchronize()
    torch.cuda.synchronize()
    completions = [Completion(r.rid, r.arrival, adm, start_ev.elapsed_time(ev) * 1e-3) for r, adm, ev in done_events]
    makespan = max(c.finished for c in completions) - min(r.arrival for r in requests)
    if log:
        log(f"served {len(completions)} requests one at a time")
    return completions, results, makespan


def latency_summary(completions: Sequence[Completion]) -> dict:
    import numpy as np
    lat = np.array([c.latency for c in completions])
    return {"p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
            "mean_s": round(float(lat.mean()), 4), "max_s": round(float(lat.max()), 4)}
