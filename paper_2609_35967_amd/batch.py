"""Many independent runs ("boxes") stepped together on one GPU.

Each box is an Engine with its own state, neighbourhoods, interval state and
workspace, and its own adaptive interval.  Two forms step every box:

* ``step_plain`` -- the plain per-box loop: one interval of each box after the
  other, launched eagerly on the current stream;
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

from .binding import PROF, Engine, check, load

import ctypes as C


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
