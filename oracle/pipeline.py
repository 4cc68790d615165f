"""One frozen-neighbour interval of the hot path, on the CPU oracle, and the
symmetric operator sequence of a transport step.

Test infrastructure only.  The order of steps follows Sect. 2.5.3:
Morton order and neighbours (Sect. 2.5.1), snapshot of the neighbourhood,
rates and controller moments, interval plan, Monte Carlo sampling against the
frozen neighbourhood, broadcast (the new masses become the next snapshot),
audit of the safety factor, then the push over the executed interval
(Sect. 2.3.3).

strang_step follows Sect. 2.6: C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2), where a
collision operator C runs intervals until its collision step of dt/2 is
complete, the neighbour lists are rebuilt only after the positions changed
(so the last C of a step and the first C of the next share them), D is the
diffusion step of Sect. 2.4 and T the push over the whole transport step.
"""
from __future__ import annotations

import numpy as np

from . import (audit, diffuse, knn, make_problem, mc, morton_keys, plan, push_global, push_local, rates,
               sort_perm)

T_TICKS = 1 << 30


class OracleRun:
    def __init__(self, params: dict, state: dict, seed: int = 0):
        self.params = params
        self.P = make_problem(params)
        self.st = {k: np.array(v, copy=True) for k, v in state.items()}
        self.seed = int(seed)
        self.C = 1.0
        self.ticks = 0
        self.interval = 0
        self.time = 0.0
        self.nb = None
        self.last = {}
        self.moved = True        # positions changed since the neighbour lists were built
        self.diff_step = 0       # draws of the next diffusion step

    def build_neighbors(self):
        st = self.st
        keys = morton_keys(st["x"], st["y"], st["z"], st["M"])
        perm = sort_perm(keys)
        self.st = {k: v[perm] for k, v in st.items()}
        st = self.st
        self.nb = knn(self.P, st["x"], st["y"], st["z"], st["M"])
        self.moved = False
        return perm

    def step(self, rebuild: bool = True, log_cap: int = 0, push: bool = True):
        P = self.P
        if rebuild or self.nb is None:
            self.build_neighbors()
        st = self.st
        nbr, cnt, dmax = self.nb
        lam, a, b, _ = rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"])
        pl = plan(P, st["m"], st["M"], a, b, self.params["dt_coll"], self.ticks, self.C)
        res = mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"],
                 pl["dt_exe"], self.seed, self.interval, log_cap=log_cap)
        au = audit(P, st["m"], res["m"], st["M"], pl["group_of"], pl["gM"], self.C)
        m_old = st["m"]
        st["m"] = res["m"]
        self.C = au["C"]
        self.ticks += pl["exe_ticks"]
        if self.ticks >= T_TICKS:
            self.ticks = 0
        self.time += pl["dt_exe"]
        self.interval += 1
        if push:
            self.transport(pl["dt_exe"])
        self.last = dict(lam=lam, a=a, b=b, plan=pl, mc=res, audit=au, m_old=m_old)
        return self.last

    def transport(self, dt: float):
        st = self.st
        kind = self.params.get("push", "none")
        if kind == "local":
            st["z"], st["vz"] = push_local(st["z"], st["vz"], st["st_mid"], st["M"], dt)
            self.moved = True
        elif kind == "global":
            new = push_global(self.P, st, dt)
            for k2 in ("r", "th", "ph", "vr", "lth", "lph", "x", "y", "z", "M"):
                st[k2] = new[k2]
            self.moved = True

    def diffusion(self, dt: float):
        if self.params.get("diffusion", "none") == "none":
            return
        new = diffuse(self.P, self.st, dt, self.seed, self.diff_step)
        self.diff_step += 1
        for k2 in ("r", "th", "ph", "vr", "lth", "lph", "x", "y", "z", "M"):
            self.st[k2] = new[k2]
        self.moved = True

    def collide(self, log_cap: int = 0):
        """Intervals without transport until the collision step of dt_coll is complete."""
        out = []
        while True:
            out.append(self.step(rebuild=self.moved or self.nb is None, log_cap=log_cap, push=False))
            if self.ticks == 0:
                return out

    def strang_step(self, log_cap: int = 0):
        """C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2) with dt/2 = dt_coll."""
        h = float(self.params["dt_coll"])
        out = self.collide(log_cap)
        self.diffusion(h)
        self.transport(2.0 * h)
        self.diffusion(h)
        return out + self.collide(log_cap)
