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
               sort_perm, transport_dt)

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
        self.dt_coll = float(params["dt_coll"])

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
        pl = plan(P, st["m"], st["M"], a, b, self.dt_coll, self.ticks, self.C)
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

    def step_dt(self, limits: dict) -> float:
        """The transport step of Sect. 2.6 chosen from the local constraints
        (reading R36), with the neighbourhood radii of the current lists (zero
        before the first search)."""
        d = self.nb[2] if self.nb is not None else np.zeros(len(self.st["M"]))
        kw = dict(limits)
        return transport_dt(self.P, self.params.get("push", "none"), self.st, d, **kw)

    def strang_step(self, log_cap: int = 0, limits: dict | None = None):
        """C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2) with dt/2 = dt_coll; with
        `limits`, dt is chosen at the start of the step (step_dt) and the
        collision steps of this transport step take dt_coll = dt/2."""
        if limits is not None:
            assert self.ticks == 0
            self.dt_coll = 0.5 * self.step_dt(limits)
        h = self.dt_coll
        out = self.collide(log_cap)
        self.diffusion(h)
        self.transport(2.0 * h)
        self.diffusion(h)
        return out + self.collide(log_cap)


class GroupedRun(OracleRun):
    """Collision steps with spatial groups (Sect. 2.5.3), on the oracle.

    Groups are n_groups contiguous ranges of the active particles in Morton
    order, g*N//G .. (g+1)*N//G.  Two groups interact when a particle of one
    keeps a neighbour in the other.  Every group has its own safety factor C
    and clock.  Within a collision step of 2^30 ticks the groups are processed
    instant by instant:

      1. at instant tau the groups whose interval ends there broadcast: their
         particles' masses at the end of the interval become the masses every
         later snapshot sees;
      2. the groups starting at tau (all of them at tau = 0) then plan one by
         one in ascending order.  A group's dyadic request (the plan of
         Sect. 2.5.3 over its own controller bins) is kept within 1/16 and 16
         times the interval of every interacting group that already has one
         scheduled; where the two limits conflict the lower one wins (a
         scheduled interval is never cut, so the refinement waits); the size is
         then halved until it starts on a multiple of itself and ends by 2^30;
      3. the group samples its whole interval at once against the broadcast
         masses of tau (nothing it does is visible to others before its end),
         and its C is audited.

    Group intervals are numbered in the order they are planned; that number
    keys the random numbers of the interval.
    """

    def __init__(self, params: dict, state: dict, seed: int = 0, n_groups: int = 1):
        super().__init__(params, state, seed)
        self.n_groups = int(n_groups)
        self.gC = [1.0] * self.n_groups
        self.bounds = None
        self.links = None
        self.log = []

    def collide(self, log_cap: int = 0):
        """The collision operator of strang_step: the grouped one."""
        start = len(self.log)
        self.collide_groups()
        return [dict(mc=dict(near_tie=np.array([e["near_tie"]]))) for e in self.log[start:]]

    def _layout(self):
        n_act = int(np.count_nonzero(self.st["M"] > 0))
        G = self.n_groups
        self.bounds = [g * n_act // G for g in range(G + 1)]
        owner = np.full(len(self.st["M"]), -1, np.int64)
        for g in range(G):
            owner[self.bounds[g]:self.bounds[g + 1]] = g
        nbr, cnt, _ = self.nb
        links = [set() for _ in range(G)]
        for i in range(n_act):
            for j in nbr[i, 1:cnt[i]]:
                if j >= 0 and owner[j] >= 0 and owner[j] != owner[i]:
                    links[owner[i]].add(int(owner[j]))
                    links[owner[j]].add(owner[i])
        self.links = links

    def collide_groups(self):
        P = self.P
        T = T_TICKS
        if self.moved or self.nb is None:
            self.build_neighbors()
            self._layout()
        elif self.bounds is None:
            self._layout()
        st = self.st
        nbr, cnt, dmax = self.nb
        G = self.n_groups
        m_pub = st["m"].copy()             # what the snapshots see
        m_end = st["m"].copy()             # each group's masses at the end of its interval
        size = [0] * G
        end = [0] * G
        start_at = [0] * G
        tau, starting, done = 0, list(range(G)), []
        tick = np.ldexp(self.dt_coll, -30)
        while True:
            for g in starting:
                a0, a1 = self.bounds[g], self.bounds[g + 1]
                q = np.arange(a0, a1)
                lam, a, b, _ = rates(P, nbr, cnt, dmax, m_pub, st["M"], st["x"], st["y"], st["z"], queries=q)
                pl = plan(P, m_pub[a0:a1], st["M"][a0:a1], a, b, self.dt_coll, tau, self.gC[g])
                want = pl["exe_ticks"]
                others = [size[h] for h in self.links[g] if size[h]]
                lo_lim = max([1] + [z // 16 for z in others])
                hi_lim = min([T] + [16 * z for z in others])
                z = max(min(want, hi_lim), lo_lim)
                while z > 1 and (tau % z != 0 or tau + z > T):
                    z //= 2
                res = mc(P, st["id"], nbr, cnt, dmax, m_pub, st["M"], st["x"], st["y"], st["z"], z * tick,
                         self.seed, self.interval, queries=q)
                self.interval += 1
                au = audit(P, m_pub[a0:a1], res["m"], st["M"][a0:a1], pl["group_of"], pl["gM"], self.gC[g])
                self.gC[g] = au["C"]
                m_end[a0:a1] = res["m"]
                size[g], end[g], start_at[g] = z, tau + z, tau
                done.append((g, tau, z))
                self.log.append(dict(group=g, start=tau, ticks=z, requested=want, lo=lo_lim, hi=hi_lim,
                                     near_tie=bool(res["near_tie"].any())))
            tau = min(end)
            starting = [g for g in range(G) if end[g] == tau]
            for g in starting:
                a0, a1 = self.bounds[g], self.bounds[g + 1]
                m_pub[a0:a1] = m_end[a0:a1]
                size[g] = 0
            if tau == T:
                st["m"] = m_pub
                return done
