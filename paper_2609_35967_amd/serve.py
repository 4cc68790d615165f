"""Serving: simulation runs that arrive over time share the GPU.

A run is (params, state, seed, intervals).  Runs wait in arrival order until
the HBM budget has room for them (their state, neighbourhoods and workspace,
sized from the library's own workspace size).  An admitted run joins the
tier of its size (by particle count); each tier has its own stream and
advances on its own:

    a tier round = one interval of every run of the tier, as one launch per
    stage over all of them (gd_many_interval: sort, tree, search, rates and
    plan, sampling with one pass over the deferred particles of the tier,
    audit, push).

Tiers are not in lock-step: a tier whose round has finished starts its next
one at once, so small runs do not wait for the intervals of large ones, and
the host keeps up to `depth` rounds of a tier queued so that the GPU does
not idle between them.  A tier whose live runs hold more than `round_cap`
particles splits them into groups under the cap and steps the groups in
turn, so that one round never holds the intervals of every large run.  A
tier's launch tables are built again only when its set of live runs changes
(a run joins or queues its last interval); tables a tier no longer uses are
released once the rounds that read them have finished.

A run that has done its intervals retires and frees its budget; runs waiting
for memory are admitted at the next poll.  Runs share nothing, and each
run's kernels and their inputs are those of the run stepped alone, so its
result does not depend on what else is served.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

from .binding import CuStream, Engine, ManyRuns, check, load

import numpy as np


@dataclass
class Run:
    rid: int
    params: dict
    state: dict
    seed: int
    intervals: int
    arrival: float = 0.0
    engine: Engine | None = None
    done: int = 0       # intervals enqueued
    finished: int = 0   # intervals completed
    bytes: int = 0
    latencies_ms: list = field(default_factory=list)   # GPU time of each interval's round
    ends_ms: list = field(default_factory=list)        # completion of each interval (server clock)


class _Tier:
    def __init__(self, torch, device, cap: int, cus=None, stream=None):
        self.torch = torch
        self.cu = CuStream(cus[0], cus[1], device=device) if cus else None
        self.stream = self.cu.stream if cus else (stream or torch.cuda.Stream(device=device))
        self.cap = int(cap)
        self.runs: list[Run] = []
        self.groups: list[tuple[list[Run], ManyRuns]] = []
        self.plan: list[int] = []  # rids the current groups step
        self.next = 0        # group of the next round
        self.inflight = []   # (start event, end event, runs of the round)
        self.stale = []      # (tables, event after which they are unused)

    def live(self) -> list[Run]:
        """The runs the next rounds step: those with intervals left to queue."""
        return [r for r in self.runs if r.done < r.intervals]

    def _regroup(self, live):
        """Largest first, each run into the first group with room for it under
        the particle cap (a run above the cap has a group of its own)."""
        if self.groups:
            done = self.torch.cuda.Event()
            done.record(self.stream)
            self.stale += [(many, done) for _, many in self.groups]
        bins: list[list[Run]] = []
        load: list[int] = []
        for r in sorted(live, key=lambda x: -x.engine.n):
            for g in range(len(bins)):
                if load[g] + r.engine.n <= self.cap:
                    bins[g].append(r)
                    load[g] += r.engine.n
                    break
            else:
                bins.append([r])
                load.append(r.engine.n)
        self.groups = [(b, ManyRuns([r.engine for r in b])) for b in bins]
        self.next = 0

    def launch(self) -> bool:
        torch = self.torch
        live = self.live()
        if not live:
            return False
        ids = sorted(r.rid for r in live)
        if ids != self.plan:
            self._regroup(live)
            self.plan = ids
        runs, many = self.groups[self.next % len(self.groups)]
        self.next += 1
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(self.stream)
        many.interval(self.stream)
        t1.record(self.stream)
        for r in runs:
            r.done += 1
        self.inflight.append((t0, t1, runs))
        return True

    def reap(self, ref, block: bool = False):
        """Completed rounds: (ms, end on the server clock, runs) for each, oldest first."""
        out = []
        while self.inflight and (block or self.inflight[0][1].query()):
            t0, t1, runs = self.inflight.pop(0)
            t1.synchronize()
            out.append((t0.elapsed_time(t1), ref.elapsed_time(t1), runs))
            block = False
        keep = []
        for many, ev in self.stale:
            if ev.query():
                many.close()
            else:
                keep.append((many, ev))
        self.stale = keep
        return out


class Server:
    def __init__(self, budget_bytes: float, tiers=(1 << 14, 1 << 17), depth: int = 2, max_runs: int = 1024,
                 device: str = "cuda", keep_results: bool = True, round_cap: int = 1 << 19, cus=None,
                 exclusive: bool = False):
        """tiers: particle-count limits of the tiers but the last (a run goes
        to the first tier whose limit it does not exceed); depth: rounds a
        tier keeps queued; round_cap: particles one round of a tier steps at
        most (a tier with more live runs takes them in groups, round after
        round, so that a long round does not hold every run's interval);
        cus: None, or per tier (first CU, CU count) of the compute units its
        stream may use (a stream per tier restricted to them); exclusive:
        the tiers take turns on one stream (at most `depth` rounds queued in
        all), so that no round shares the device with another: the lowest
        interval latency, at the price of capacity."""
        import torch
        self.keep_results = bool(keep_results)
        self.torch = torch
        self.lib = load()
        self.budget = float(budget_bytes)
        self.used = 0.0
        self.device = device
        self.limits = list(tiers)
        nt = len(self.limits) + 1
        if cus is not None and len(cus) != nt:
            raise ValueError(f"cus needs one (first, count) per tier ({nt})")
        self.exclusive = bool(exclusive)
        if self.exclusive and cus is not None:
            raise ValueError("exclusive tiers share one stream: no per-tier compute units")
        shared = torch.cuda.Stream(device=device) if self.exclusive else None
        self.tiers = [_Tier(torch, device, round_cap, cus[i] if cus else None, shared) for i in range(nt)]
        self.turn = 0
        self.ref = torch.cuda.Event(enable_timing=True)  # the server clock's origin
        self.ref.record(torch.cuda.current_stream())
        self.depth = max(1, int(depth))
        self.max_runs = int(max_runs)
        self.waiting: list[Run] = []
        self.finished: list[Run] = []
        self.rounds = 0  # tier rounds queued

    @staticmethod
    def run_bytes(lib, params: dict, n: int) -> int:
        """HBM a run holds: two state copies, neighbour rows, per-particle
        vectors and the workspace."""
        from .binding import make_problem
        P = make_problem(params, n)
        sz = C.c_size_t()
        check(lib.gd_workspace_size(C.byref(P), C.byref(sz)))
        state = 2 * 16 * 8 * n           # two copies of up to 16 eight-byte arrays
        rows = n * P.k * 4 + n * (4 + 8 + 8 + 4)
        return int(sz.value + state + rows)

    @property
    def active(self) -> list[Run]:
        return [r for t in self.tiers for r in t.runs]

    def submit(self, run: Run):
        run.bytes = self.run_bytes(self.lib, run.params, len(run.state["x"]))
        if run.bytes > self.budget:
            raise ValueError(f"run {run.rid} needs {run.bytes} B, above the budget")
        self.waiting.append(run)

    def _tier_of(self, n: int) -> _Tier:
        for lim, t in zip(self.limits, self.tiers):
            if n <= lim:
                return t
        return self.tiers[-1]

    def admit(self):
        admitted = False
        while (self.waiting and len(self.active) < self.max_runs
               and self.used + self.waiting[0].bytes <= self.budget):
            r = self.waiting.pop(0)
            r.engine = Engine(r.params, r.state, seed=r.seed, device=self.device, device_interval=True)
            self.used += r.bytes
            self._tier_of(r.engine.n).runs.append(r)
            admitted = True
        if admitted:  # the new engines' uploads ran on torch's stream
            self.torch.cuda.current_stream().synchronize()

    def _collect(self, tier: _Tier, block: bool = False) -> list[Run]:
        out = []
        for ms, end, runs in tier.reap(self.ref, block):
            for r in runs:
                r.finished += 1
                r.latencies_ms.append(ms)
                r.ends_ms.append(end)
        for r in list(tier.runs):
            if r.finished >= r.intervals:
                tier.runs.remove(r)
                self.used -= r.bytes
                if not self.keep_results:
                    r.engine = None  # its memory goes back to the allocator
                self.finished.append(r)
                out.append(r)
        return out

    def poll(self) -> tuple[list[Run], bool]:
        """Collect finished rounds, retire finished runs, and queue the next
        round of every tier that has room.  Returns (runs retired, whether a
        round was queued).  Never waits for the GPU."""
        out, launched = [], False
        for t in self.tiers:
            out += self._collect(t)
        if self.exclusive:
            # tiers in turn while the shared stream has room
            nt = len(self.tiers)
            for d in range(nt):
                if sum(len(x.inflight) for x in self.tiers) >= self.depth:
                    break
                t = self.tiers[(self.turn + d) % nt]
                if t.launch():
                    self.rounds += 1
                    launched = True
                    self.turn = (self.turn + d + 1) % nt
                    break
            return out, launched
        for t in self.tiers:
            if len(t.inflight) < self.depth and t.launch():
                self.rounds += 1
                launched = True
        return out, launched

    def wait(self) -> list[Run]:
        """Block until the oldest queued round of any tier finishes."""
        busy = [t for t in self.tiers if t.inflight]
        if not busy:
            return []
        t = min(busy, key=lambda x: len(x.inflight))
        return self._collect(t, block=True)

    def round(self) -> list[Run]:
        """One round of every tier with runs, then wait for all of them (the
        blocking form, for tests and simple drivers)."""
        for t in self.tiers:
            if t.launch():
                self.rounds += 1
        out = []
        for t in self.tiers:
            while t.inflight:
                out += self._collect(t, block=True)
            out += self._collect(t)
        return out

    def idle(self) -> bool:
        return not self.active and not self.waiting

    def close(self):
        for t in self.tiers:
            while t.inflight:
                self._collect(t, block=True)
            for many, ev in t.stale:
                ev.synchronize()
                many.close()
            t.stale = []
            for _, many in t.groups:
                many.close()
            t.groups = []
            t.plan = []
            if t.cu is not None:
                t.cu.close()
                t.cu = None


def drive(server: Server, arrivals, clock) -> None:
    """Serve `arrivals` [(time, Run)] (ascending) to completion: submit each
    run at its time on `clock()`, admit, queue rounds, and wait for the GPU
    only when nothing can be queued."""
    import time
    pending = list(arrivals)
    while pending or not server.idle():
        now = clock()
        while pending and pending[0][0] <= now:
            server.submit(pending.pop(0)[1])
        server.admit()
        _, launched = server.poll()
        if launched:
            continue
        if any(t.inflight for t in server.tiers):
            server.wait()
        elif pending:
            time.sleep(max(0.0, pending[0][0] - clock()))


def latency_percentiles(runs, q=(50, 99)):
    """Percentiles of the GPU time of the rounds that held each run's intervals."""
    lat = np.concatenate([np.asarray(r.latencies_ms) for r in runs]) if runs else np.zeros(1)
    return [float(np.percentile(lat, x)) for x in q]


def gap_percentiles(runs, q=(50, 99)):
    """Percentiles of the time between successive interval completions of a
    run (what its owner waits per interval once it is running)."""
    gaps = [np.diff(np.asarray(r.ends_ms)) for r in runs if len(r.ends_ms) > 1]
    g = np.concatenate(gaps) if gaps else np.zeros(1)
    return [float(np.percentile(g, x)) for x in q]
