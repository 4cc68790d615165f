"""Serving: simulation runs that arrive over time share the GPU.

A run is (params, state, seed, intervals).  Runs wait in arrival order until
the HBM budget has room for them (their state, neighbourhoods and workspace,
sized from the library's own workspace size); then each round advances every
admitted run by one interval:

    per run, on one of a few streams: neighbour search, rates, the per-lane
    sampling pass (its arguments into slot r of a shared table);
    one launch: the deferred particles of every run (gd_sample_table_run);
    per run: the audit, the push.

A run that has done its intervals retires and frees its budget, and runs
waiting for memory are admitted at the next round.  Runs share nothing, and
each run's kernels and their inputs are those of the run stepped alone, so
its result does not depend on what else is served.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

from .binding import Engine, check, load

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
    done: int = 0
    bytes: int = 0
    latencies_ms: list = field(default_factory=list)


class Server:
    def __init__(self, budget_bytes: float, streams: int = 8, max_runs: int = 1024, device: str = "cuda",
                 keep_results: bool = True):
        import torch
        self.keep_results = bool(keep_results)
        self.torch = torch
        self.lib = load()
        self.budget = float(budget_bytes)
        self.used = 0.0
        self.device = device
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(streams)))]
        self.max_runs = int(max_runs)
        sz = C.c_size_t()
        check(self.lib.gd_sample_table_size(self.max_runs, C.byref(sz)))
        self.table = torch.empty(sz.value, dtype=torch.uint8, device=device)
        self.table_bytes = sz.value
        self.waiting: list[Run] = []
        self.active: list[Run] = []
        self.finished: list[Run] = []

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

    def submit(self, run: Run):
        run.bytes = self.run_bytes(self.lib, run.params, len(run.state["x"]))
        if run.bytes > self.budget:
            raise ValueError(f"run {run.rid} needs {run.bytes} B, above the budget")
        self.waiting.append(run)

    def admit(self):
        while self.waiting and len(self.active) < self.max_runs and self.used + self.waiting[0].bytes <= self.budget:
            r = self.waiting.pop(0)
            r.engine = Engine(r.params, r.state, seed=r.seed, device=self.device)
            self.used += r.bytes
            self.active.append(r)

    def round(self):
        """One interval of every active run; returns the runs that finished."""
        torch = self.torch
        lib = self.lib
        if not self.active:
            return []
        act = self.active
        ks = {r.engine.P.k <= 32 for r in act}
        fp = {int(r.engine.P.rates_fp32) for r in act}
        if len(ks) != 1 or len(fp) != 1:
            raise ValueError("served runs need one k class and one rates form")
        cs = torch.cuda.current_stream()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(cs)
        for st in self.streams:
            st.wait_stream(cs)
        order = sorted(range(len(act)), key=lambda i: -act[i].engine.n)
        load_of = [0] * len(self.streams)
        tp = self.table.data_ptr()
        for slot, i in enumerate(order):
            s = min(range(len(self.streams)), key=lambda t: load_of[t])
            load_of[s] += act[i].engine.n
            e = act[i].engine
            e.stream = self.streams[s]
            e.build_neighbors()
            e.collision_rates()
            e.sample_deferred(tp, self.table_bytes, slot)
        for st in self.streams:
            cs.wait_stream(st)
        check(lib.gd_sample_table_run(C.c_void_p(tp), self.table_bytes, len(act), act[0].engine.P.k, fp.pop(),
                                      C.c_void_p(cs.cuda_stream)))
        for st in self.streams:
            st.wait_stream(cs)
        for r in act:
            r.engine.sample_audit()
            if r.engine.P.push != 0:
                r.engine.push()
        for st in self.streams:
            cs.wait_stream(st)
        t1.record(cs)
        t1.synchronize()
        ms = t0.elapsed_time(t1)
        out = []
        for r in act:
            r.engine.stream = None
            r.done += 1
            r.latencies_ms.append(ms)
        for r in list(act):
            if r.done >= r.intervals:
                act.remove(r)
                self.used -= r.bytes
                if not self.keep_results:
                    r.engine = None  # its memory goes back to the allocator
                self.finished.append(r)
                out.append(r)
        return out

    def idle(self) -> bool:
        return not self.active and not self.waiting


def latency_percentiles(runs, q=(50, 99)):
    lat = np.concatenate([np.asarray(r.latencies_ms) for r in runs]) if runs else np.zeros(1)
    return [float(np.percentile(lat, x)) for x in q]
