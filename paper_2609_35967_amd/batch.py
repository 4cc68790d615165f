"""Many independent runs ("boxes") stepped together on one GPU.

Each box is an Engine with its own state, neighbourhoods, interval state and
workspace, and its own adaptive interval.  Three forms step every box:

* ``step_plain`` -- the plain per-box loop: one interval of each box after the
  other, launched eagerly on the current stream;
* ``step_many`` -- one launch per stage over every box (gd_many_interval):
  the boxes' blocks follow one another in each grid and find their box's
  arguments through tables in device memory, so an interval is about forty
  launches whatever the number of boxes.  ``tune`` picks its launch shapes
  by timing candidates on the batch itself (from a saved device state, so
  every candidate runs the same intervals) and records what it measured;
* ``replay`` -- one HIP graph holding two intervals of every box.  Per
  interval: each box's neighbour search, rates and per-lane sampling pass on
  its stream (boxes dealt to a few streams, largest first, each to the stream
  with the least work so far, so that the small launches of different boxes
  overlap), its sampling arguments written to a slot of a shared table; then
  one launch samples the particles that outlast the per-lane pass in every
  box (gd_sample_table_run), and each box's audit follows on its stream.
  Two intervals per graph: the Morton permutation alternates between a box's
  two state buffers and the sampling between its two mass buffers, so after
  two intervals every buffer is back in its place and the graph can be
  replayed.  The sampling calls take their interval index from the device
  interval state, so each replay draws fresh numbers.

A box's result does not depend on the form or on the other boxes: the kernels
and their inputs are the same, and nothing is shared between boxes.
"""
from __future__ import annotations

from .binding import MANY_DEFAULTS, PROF, Engine, ManyRuns, check, load

import ctypes as C
import time


class BoxBatch:
    def __init__(self, boxes, streams: int = 4, device: str = "cuda"):
        """boxes: [(params, state, seed)]; streams: streams the graph spreads boxes over."""
        import torch
        self.torch = torch
        self.boxes = boxes
        self.device = device
        self.engines = [Engine(p, s, seed=sd, device=device, device_interval=True) for p, s, sd in boxes]
        self.nstreams = max(1, int(streams))
        self.graph = None
        self.streams = None

    @property
    def n_particles(self) -> int:
        return sum(e.n for e in self.engines)

    def many(self, tuning: dict | None = None) -> list:
        """The one-launch-per-stage form over every box (built on first use,
        or again when `tuning` is given).  tuning["sets"] = S splits the boxes
        into S sets of about equal particle count (largest first, each to the
        lightest set), each stepped as one on a stream of its own: a set whose
        interval ends in one particle's long chain of events (one wavefront
        busy) then overlaps the other sets' work.  The other keys are the
        launch shapes of gd_many_create."""
        torch = self.torch
        if tuning is not None or getattr(self, "_many", None) is None:
            for m in getattr(self, "_many", None) or []:
                m.close()
            t = dict(tuning if tuning is not None else (getattr(self, "tuned", None) or {}))
            sets = max(1, min(int(t.pop("sets", 1)), len(self.engines)))
            load_of = [0] * sets
            members = [[] for _ in range(sets)]
            for i in sorted(range(len(self.engines)), key=lambda i: -self.engines[i].n):
                k = min(range(sets), key=lambda j: load_of[j])
                members[k].append(self.engines[i])
                load_of[k] += self.engines[i].n
            self._many = [ManyRuns(mem, t) for mem in members if mem]
            if len(getattr(self, "_many_streams", [])) < len(self._many):
                self._many_streams = [torch.cuda.Stream() for _ in range(len(self._many))]
        return self._many

    def step_many(self):
        """One interval of every box, one launch per stage (per set of boxes)."""
        sets = self.many()
        if len(sets) == 1:
            sets[0].interval()
            return
        torch = self.torch
        cs = torch.cuda.current_stream()
        for m, st in zip(sets, self._many_streams):
            st.wait_stream(cs)
            m.interval(st)
        for st in self._many_streams[:len(sets)]:
            cs.wait_stream(st)

    # ---- the project's autotuner for the launch shapes of step_many ---------------
    def _save(self):
        torch = self.torch
        torch.cuda.synchronize()
        out = []
        for e in self.engines:
            out.append(dict(A={k: v.clone() for k, v in e.A.t.items()}, B={k: v.clone() for k, v in e.B.t.items()},
                            Acur=e.A.cur, Bcur=e.B.cur, Aobj=e.A, Bobj=e.B,
                            t={k: getattr(e, k).clone() for k in ("nbr", "cnt", "dmax", "n_active", "lam", "events", "iv")},
                            interval=e.interval, moved=e.moved))
        return out

    def _load(self, saved):
        torch = self.torch
        torch.cuda.synchronize()
        for e, s in zip(self.engines, saved):
            e.A, e.B = s["Aobj"], s["Bobj"]
            for k, v in s["A"].items():
                e.A.t[k].copy_(v)
            for k, v in s["B"].items():
                e.B.t[k].copy_(v)
            e.A.cur, e.B.cur = s["Acur"], s["Bcur"]
            for k, v in s["t"].items():
                getattr(e, k).copy_(v)
            e.interval, e.moved = s["interval"], s["moved"]
        torch.cuda.synchronize()

    SPACE = dict(sets=(1, 2, 4, 8), knn_tile=(1, 0), heavy_blocks=(256, 512, 768, 1024, 1536),
                 event_div=(256, 512, 1024, 2048),
                 fallback_div=(64, 256, 1024), red_div=(512, 2048, 8192))

    def tune(self, intervals: int = 2, space: dict | None = None) -> dict:
        """Coordinate search over the launch shapes of step_many: each knob in
        turn takes every value of `space` with the others at their best so far;
        every trial runs the same `intervals` intervals from the same saved
        state (results do not depend on the shapes, only times do).  Keeps the
        fastest and returns {"choice", "trials": [(setting, ms per interval)]}."""
        torch = self.torch
        space = space or self.SPACE
        saved = self._save()
        best = dict(MANY_DEFAULTS, sets=1)
        trials = []
        cache = {}

        def trial(setting):
            key = tuple(sorted(setting.items()))
            if key in cache:
                return cache[key]
            self._load(saved)
            self.many(dict(setting))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(intervals):
                self.step_many()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / intervals
            cache[key] = ms
            trials.append((dict(setting), round(ms, 3)))
            return ms

        best_ms = trial(best)
        for knob, values in space.items():
            for v in values:
                cand = dict(best, **{knob: v})
                ms = trial(cand)
                if ms < best_ms:
                    best, best_ms = cand, ms
        self._load(saved)
        self.tuned = best
        self.many(best)
        self.tuning_record = dict(choice=best, ms_per_interval=round(best_ms, 3), trials=trials)
        return self.tuning_record

    def step_plain(self):
        """One interval of every box, one box after the other on the current stream."""
        for e in self.engines:
            e.stream = None
            e.step()

    def capture(self):
        """Record two intervals of every box into one graph (nothing runs yet)."""
        torch = self.torch
        lib = load()
        for w in PROF.values():  # no timing events inside the graph
            check(lib.gd_profile_events(w, None, None))
        # a throwaway copy of the smallest box runs two intervals eagerly, so
        # that every kernel of the path is loaded before the recording
        p, s, sd = min(self.boxes, key=lambda b: len(b[1]["x"]))
        w = Engine(p, s, seed=sd, device=self.device, device_interval=True)
        w.step()
        w.step()
        torch.cuda.synchronize()
        del w
        self.streams = [torch.cuda.Stream() for _ in range(self.nstreams)]
        load_of = [0] * self.nstreams
        assign = [0] * len(self.engines)
        for i in sorted(range(len(self.engines)), key=lambda i: -self.engines[i].n):
            s = min(range(self.nstreams), key=lambda t: load_of[t])
            assign[i] = s
            load_of[s] += self.engines[i].n
        ks = {e.P.k <= 32 for e in self.engines}
        fp = {int(e.P.rates_fp32) for e in self.engines}
        if len(ks) != 1 or len(fp) != 1:
            raise ValueError("batched boxes need one k class (k <= 32 or not) and one rates form")
        nb = len(self.engines)
        sz = C.c_size_t()
        check(lib.gd_sample_table_size(nb, C.byref(sz)))
        self.table = torch.empty(sz.value, dtype=torch.uint8, device=self.device)
        tp, tb = self.table.data_ptr(), sz.value
        k, f32 = self.engines[0].P.k, fp.pop()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cs = torch.cuda.current_stream()
            for st in self.streams:
                st.wait_stream(cs)
            for _ in range(2):
                for i, e in enumerate(self.engines):
                    e.stream = self.streams[assign[i]]
                    e.build_neighbors()
                    e.collision_rates()
                    e.sample_deferred(tp, tb, i)
                for st in self.streams:
                    cs.wait_stream(st)
                check(lib.gd_sample_table_run(C.c_void_p(tp), tb, nb, k, f32, C.c_void_p(cs.cuda_stream)))
                for st in self.streams:
                    st.wait_stream(cs)
                for e in self.engines:
                    e.sample_audit()
                    if e.P.push != 0:
                        e.push()
            for st in self.streams:
                cs.wait_stream(st)
        for e in self.engines:
            e.stream = None
        self.graph = g

    def replay(self):
        """Two intervals of every box (the recorded graph)."""
        if self.graph is None:
            self.capture()
        self.graph.replay()
