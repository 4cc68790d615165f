"""Thin ctypes binding of libgd.so (include/gd.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  The library must
be built (``paper_2609_35967_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgd.so")

GD_OK = 0
KERNELS = {"const": 0, "additive": 1, "product": 2, "physical": 3}
PUSH = {"none": 0, "local": 1, "global": 2}
DIFFUSION = {"none": 0, "concentration": 1, "density": 2}
DEV_BITS = {"nonfinite": 0x1, "log_overflow": 0x2, "knn_fallback": 0x4, "tick_floor": 0x8, "mass_range": 0x10,
            "internal": 0x20, "event_cap": 0x40}
T_TICKS = 1 << 30


class GdProblem(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("k", C.c_int32), ("kernel", C.c_int32), ("push", C.c_int32), ("nbin_min", C.c_int32),
        ("erosion", C.c_int32), ("grouping", C.c_int32), ("periodic", C.c_int32 * 3), ("L", C.c_double * 3),
        ("rmax", C.c_double), ("t0", C.c_double), ("m0", C.c_double), ("eps", C.c_double), ("dt_fn_max", C.c_double),
        ("rho_s", C.c_double), ("s_min", C.c_double), ("v_frag", C.c_double), ("GM", C.c_double),
        ("Sigma_g0", C.c_double), ("R0", C.c_double), ("p", C.c_double), ("q", C.c_double), ("h_g0", C.c_double),
        ("alpha", C.c_double), ("mu_mH", C.c_double), ("sigma_H2", C.c_double), ("s0", C.c_double),
        ("St0", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double), ("drag", C.c_int32),
        ("brownian", C.c_int32), ("turbulence", C.c_int32), ("caps", C.c_int32), ("rates_fp32", C.c_int32),
        ("diffusion", C.c_int32), ("vint", C.c_int32), ("axisym", C.c_int32), ("pad_", C.c_int32),
        ("Sc", C.c_double * 3), ("St_diff", C.c_double),
    ]


class GdParticles(C.Structure):
    _fields_ = [
        ("id", C.c_void_p), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
        ("r", C.c_void_p), ("th", C.c_void_p), ("ph", C.c_void_p),
        ("vr", C.c_void_p), ("lth", C.c_void_p), ("lph", C.c_void_p),
        ("vz", C.c_void_p), ("st_mid", C.c_void_p), ("M", C.c_void_p),
        ("m", C.c_void_p * 2), ("cur", C.c_int32),
    ]


class GdNeighbors(C.Structure):
    _fields_ = [("nbr", C.c_void_p), ("cnt", C.c_void_p), ("dmax", C.c_void_p), ("n_active", C.c_void_p)]


class GdInterval(C.Structure):
    _fields_ = [
        ("dt_coll", C.c_double), ("dt_req", C.c_double), ("dt_exe", C.c_double), ("C", C.c_double),
        ("time", C.c_double), ("ticks", C.c_int64), ("exe_ticks", C.c_int64), ("n_intervals", C.c_int64),
        ("n_events", C.c_int64), ("audit_worst", C.c_double), ("n_groups", C.c_int32), ("pad", C.c_int32),
    ]


class GdRun(C.Structure):
    _fields_ = [
        ("p", C.POINTER(GdProblem)), ("a", C.POINTER(GdParticles)), ("b", C.POINTER(GdParticles)),
        ("nb", C.POINTER(GdNeighbors)), ("iv", C.c_void_p), ("lam_i", C.c_void_p), ("n_events", C.c_void_p),
        ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("seed", C.c_uint64),
    ]


class GdStepLimits(C.Structure):
    _fields_ = [("dt_max", C.c_double), ("dt_out", C.c_double), ("c_orb", C.c_double), ("c_adv", C.c_double),
                ("c_diff", C.c_double)]


STEP_DEFAULTS = dict(dt_out=math.inf, c_orb=0.05, c_adv=0.5, c_diff=0.5)


class GdManyTuning(C.Structure):
    _fields_ = [("knn_tile", C.c_int32), ("fallback_div", C.c_int32), ("event_div", C.c_int32),
                ("red_div", C.c_int32), ("heavy_blocks", C.c_int32)]


MANY_DEFAULTS = dict(knn_tile=1, fallback_div=256, event_div=512, red_div=2048, heavy_blocks=768)

EXPORTS = ("gd_workspace_size", "gd_workspace_init", "gd_interval_init", "gd_build_neighbors", "gd_collision_rates",
           "gd_sample_collisions", "gd_push", "gd_profile_events", "gd_status_read", "gd_last_error", "gd_version",
           "gd_sample_table_size", "gd_sample_collisions_deferred", "gd_sample_table_run", "gd_sample_audit",
           "gd_reshuffle_neighbors", "gd_diffuse", "gd_group_interactions", "gd_collision_rates_group",
           "gd_sample_collisions_group", "gd_publish_group", "gd_reshuffle_neighbors_static",
           "gd_many_create", "gd_many_interval", "gd_many_parity", "gd_many_destroy", "gd_stream_create_cu_mask",
           "gd_stream_destroy", "gd_transport_dt",
           "gd_group_sched_create", "gd_group_sched_begin", "gd_group_sched_instants", "gd_group_sched_read",
           "gd_group_sched_destroy")
PROF = {"sort": 0, "tree": 1, "knn_query": 2, "rates": 3, "mc": 4, "audit": 5, "push": 6, "diffuse": 7}
GD_INTERVAL_ON_DEVICE = (1 << 64) - 1

_lib = None


class GdError(RuntimeError):
    pass


def load(path: str | None = None):
    """Load libgd.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise GdError(f"{p} is missing: build it with `python -m paper_2609_35967_amd.build` "
                      "(no CPU fallback exists)")
    L = C.CDLL(p)
    vp = C.c_void_p
    L.gd_workspace_size.argtypes = [C.POINTER(GdProblem), C.POINTER(C.c_size_t)]
    L.gd_interval_init.argtypes = [vp, C.c_double, vp]
    L.gd_workspace_init.argtypes = [C.POINTER(GdProblem), vp, C.c_size_t, vp]
    L.gd_build_neighbors.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdParticles),
                                     C.POINTER(GdNeighbors), vp, C.c_size_t, vp]
    L.gd_collision_rates.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors), vp, vp,
                                     vp, vp, vp, C.c_size_t, vp]
    L.gd_sample_collisions.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors), vp, vp,
                                       C.c_uint64, C.c_uint64, vp, vp, C.c_int32, vp, C.c_size_t, vp]
    L.gd_push.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), vp, C.c_double, vp, C.c_size_t, vp]
    L.gd_sample_table_size.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    L.gd_sample_collisions_deferred.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors),
                                                vp, vp, C.c_uint64, C.c_uint64, vp, vp, C.c_int32, vp, C.c_size_t,
                                                vp, C.c_size_t, C.c_int32, vp]
    L.gd_sample_table_run.argtypes = [vp, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, vp]
    L.gd_sample_audit.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), vp, vp, C.c_size_t, vp]
    L.gd_reshuffle_neighbors.argtypes = [C.POINTER(GdProblem), C.POINTER(GdNeighbors), C.c_uint64, C.c_uint32, vp,
                                         C.c_size_t, vp]
    L.gd_reshuffle_neighbors_static.argtypes = [C.POINTER(GdProblem), C.POINTER(GdNeighbors), C.c_uint64,
                                                C.c_uint32, vp]
    L.gd_diffuse.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.c_double, C.c_uint64, C.c_uint32, vp]
    L.gd_group_interactions.argtypes = [C.POINTER(GdProblem), C.POINTER(GdNeighbors), vp, C.c_int32, vp, vp]
    L.gd_collision_rates_group.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors), vp,
                                           vp, C.c_int64, C.c_int64, C.c_int32, C.c_int32, vp, vp, C.c_int32, vp,
                                           C.c_size_t, vp]
    L.gd_sample_collisions_group.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors),
                                             vp, vp, C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, vp, vp,
                                             C.c_size_t, vp]
    L.gd_publish_group.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.c_int64, C.c_int64, vp, C.c_int32,
                                   vp]
    L.gd_many_create.argtypes = [C.POINTER(GdRun), C.c_int32, C.POINTER(GdManyTuning), C.POINTER(vp)]
    L.gd_many_interval.argtypes = [vp, vp]
    L.gd_many_parity.argtypes = [vp, C.POINTER(C.c_int32)]
    L.gd_many_destroy.argtypes = [vp]
    L.gd_stream_create_cu_mask.argtypes = [C.POINTER(C.c_uint32), C.c_int32, C.POINTER(vp)]
    L.gd_stream_destroy.argtypes = [vp]
    L.gd_group_sched_create.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors), vp,
                                        C.c_int32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, C.c_uint64, C.POINTER(vp)]
    L.gd_group_sched_begin.argtypes = [vp, C.c_int64, vp]
    L.gd_group_sched_instants.argtypes = [vp, C.c_int32, vp]
    L.gd_group_sched_read.argtypes = [vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32), vp,
                                      C.c_int32]
    L.gd_group_sched_destroy.argtypes = [vp]
    L.gd_transport_dt.argtypes = [C.POINTER(GdProblem), C.POINTER(GdParticles), C.POINTER(GdNeighbors),
                                  C.POINTER(GdStepLimits), vp, vp, vp, C.c_size_t, vp]
    L.gd_status_read.argtypes = [vp, vp, C.POINTER(C.c_int32)]
    L.gd_profile_events.argtypes = [C.c_int32, vp, vp]
    L.gd_last_error.restype = C.c_char_p
    L.gd_version.restype = C.c_char_p
    for name in ("gd_workspace_size", "gd_workspace_init", "gd_interval_init", "gd_build_neighbors", "gd_collision_rates",
                 "gd_sample_collisions", "gd_push", "gd_status_read", "gd_profile_events", "gd_sample_table_size",
                 "gd_sample_collisions_deferred", "gd_sample_table_run", "gd_sample_audit",
                 "gd_reshuffle_neighbors", "gd_diffuse", "gd_group_interactions", "gd_collision_rates_group",
                 "gd_sample_collisions_group", "gd_publish_group", "gd_reshuffle_neighbors_static",
                 "gd_many_create", "gd_many_interval", "gd_many_parity", "gd_many_destroy",
                 "gd_stream_create_cu_mask", "gd_stream_destroy", "gd_transport_dt", "gd_group_sched_create",
                 "gd_group_sched_begin", "gd_group_sched_instants", "gd_group_sched_read", "gd_group_sched_destroy"):
        getattr(L, name).restype = C.c_int32
    if path is None:
        _lib = L
    return L


def check(rc: int):
    if rc != GD_OK:
        msg = load().gd_last_error().decode()
        raise GdError(f"gd status {rc}: {msg}")


def make_problem(cfg: dict, n: int | None = None) -> GdProblem:
    """gd_problem from a workload parameter dict."""
    P = GdProblem()
    P.n = int(cfg["n"] if n is None else n)
    P.k = int(cfg["k"])
    P.kernel = KERNELS[cfg["kernel"]]
    P.push = PUSH[cfg.get("push", "none")]
    P.nbin_min = int(cfg.get("nbin_min", 0))
    P.erosion = int(cfg.get("erosion", 1))
    P.grouping = int(cfg.get("grouping", 1))
    per = cfg.get("periodic", (0, 0, 0))
    Ls = cfg.get("L", (1.0, 1.0, 1.0))
    for a in range(3):
        P.periodic[a] = int(per[a])
        P.L[a] = float(Ls[a])
    P.rmax = float(cfg.get("rmax", math.inf))
    for name in ("t0", "m0", "eps", "dt_fn_max", "rho_s", "s_min", "v_frag", "GM", "Sigma_g0", "R0", "p", "q",
                 "h_g0", "alpha", "mu_mH", "sigma_H2", "s0", "St0", "r_in", "r_out"):
        setattr(P, name, float(cfg.get(name, 0.0)))
    for name in ("drag", "brownian", "turbulence", "caps", "rates_fp32", "vint", "axisym"):
        setattr(P, name, int(cfg.get(name, 0)))
    P.diffusion = DIFFUSION[cfg.get("diffusion", "none")]
    Sc = cfg.get("Sc", (1.0, 1.0, 1.0))
    for a in range(3):
        P.Sc[a] = float(Sc[a])
    P.St_diff = float(cfg.get("St_diff", 0.0))
    return P


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


STATE_ARRAYS = ("x", "y", "z", "r", "th", "ph", "vr", "lth", "lph", "vz", "st_mid", "M")


class DeviceState:
    """One set of particle arrays on the GPU (torch tensors) and its gd_particles view."""

    def __init__(self, torch, arrays: dict, n: int, device):
        self.torch = torch
        self.n = n
        self.t = {}
        for k in STATE_ARRAYS:
            if k in arrays and arrays[k] is not None:
                self.t[k] = torch.as_tensor(np.ascontiguousarray(arrays[k], np.float64), device=device).clone()
        self.t["id"] = torch.as_tensor(np.ascontiguousarray(arrays["id"]).astype(np.int32), device=device).clone()
        m = torch.as_tensor(np.ascontiguousarray(arrays["m"], np.float64), device=device)
        self.t["m0"] = m.clone()
        self.t["m1"] = torch.empty_like(m)
        self.cur = 0

    @classmethod
    def like(cls, other: "DeviceState"):
        self = cls.__new__(cls)
        self.torch = other.torch
        self.n = other.n
        self.t = {k: other.torch.empty_like(v) for k, v in other.t.items()}
        self.cur = other.cur
        return self

    def struct(self) -> GdParticles:
        s = GdParticles()
        s.id = self.t["id"].data_ptr()
        for k in STATE_ARRAYS:
            setattr(s, k, self.t[k].data_ptr() if k in self.t else None)
        s.m[0] = self.t["m0"].data_ptr()
        s.m[1] = self.t["m1"].data_ptr()
        s.cur = self.cur
        return s

    def m(self):
        return self.t["m0"] if self.cur == 0 else self.t["m1"]

    def to_numpy(self) -> dict:
        out = {k: v.cpu().numpy() for k, v in self.t.items() if k not in ("m0", "m1", "id")}
        out["id"] = self.t["id"].cpu().numpy().view(np.uint32)
        out["m"] = self.m().cpu().numpy()
        return out


class Engine:
    """A run of the hot path on one GPU: state (double-buffered for the Morton
    permutation), neighbourhoods, interval state and workspace, all resident in HBM."""

    def __init__(self, params: dict, state: dict, seed: int = 0, device: str = "cuda", stream=None,
                 device_interval: bool = False):
        import torch
        self.torch = torch
        self.lib = load()
        self.params = params
        n = len(state["x"])
        self.n = n
        self.P = make_problem(params, n)
        self.device = torch.device(device)
        self.stream = stream
        self.seed = int(seed)
        self.interval = 0
        # sampling takes its interval index from the device interval state
        # (GD_INTERVAL_ON_DEVICE), as a call recorded in a graph must
        self.device_interval = bool(device_interval)
        k = self.P.k
        self.A = DeviceState(torch, state, n, self.device)
        self.B = DeviceState.like(self.A)
        i32 = dict(dtype=torch.int32, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.nbr = torch.empty((n, k), **i32)
        self.cnt = torch.empty(n, **i32)
        self.dmax = torch.zeros(n, **f64)  # read back as the next search's hint
        self.n_active = torch.zeros(1, **i32)
        self.lam = torch.empty(n, **f64)
        self.events = torch.zeros(n, **i32)
        self.iv = torch.zeros(C.sizeof(GdInterval), dtype=torch.uint8, device=self.device)
        sz = C.c_size_t()
        check(self.lib.gd_workspace_size(C.byref(self.P), C.byref(sz)))
        self.ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.ws_bytes = sz.value
        self.nb = GdNeighbors(self.nbr.data_ptr(), self.cnt.data_ptr(), self.dmax.data_ptr(), self.n_active.data_ptr())
        self.moved = True       # positions changed since the neighbour lists were built
        self.diff_step = 0      # draws of the next diffusion step of strang_step
        if self.stream is not None:  # the uploads ran on torch's stream, the library runs on ours
            torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.gd_workspace_init(C.byref(self.P), C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))
        check(self.lib.gd_interval_init(C.c_void_p(self.iv.data_ptr()), float(params["dt_coll"]), self._s()))

    def _s(self):
        st = self.stream if self.stream is not None else self.torch.cuda.current_stream()
        return C.c_void_p(st.cuda_stream)

    # ---- the four calls --------------------------------------------------------
    def build_neighbors(self):
        sa, sb = self.A.struct(), self.B.struct()
        check(self.lib.gd_build_neighbors(C.byref(self.P), C.byref(sa), C.byref(sb), C.byref(self.nb),
                                          C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))
        self.A, self.B = self.B, self.A
        self.A.cur = sb.cur
        self.moved = False

    def collision_rates(self, lam_pair=None, ab=None):
        s = self.A.struct()
        check(self.lib.gd_collision_rates(C.byref(self.P), C.byref(s), C.byref(self.nb),
                                          C.c_void_p(self.iv.data_ptr()), _ptr(self.lam), _ptr(lam_pair), _ptr(ab),
                                          C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))

    def sample_collisions(self, log=None, log_cap=0, flip=True):
        s = self.A.struct()
        check(self.lib.gd_sample_collisions(C.byref(self.P), C.byref(s), C.byref(self.nb),
                                            C.c_void_p(self.iv.data_ptr()), _ptr(self.lam), self.seed,
                                            GD_INTERVAL_ON_DEVICE if self.device_interval else self.interval,
                                            _ptr(self.events), _ptr(log), int(log_cap),
                                            C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))
        self.interval += 1
        if flip:
            self.A.cur ^= 1

    def reshuffle_neighbors(self, refresh: int):
        """Random relabelling of the cached neighbours (product-kernel test), in place."""
        check(self.lib.gd_reshuffle_neighbors(C.byref(self.P), C.byref(self.nb), self.seed, int(refresh),
                                              C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))

    def reshuffle_neighbors_static(self, refresh: int):
        """The same relabelling through the allocation-free entry point (its
        table is the library's fixed per-GPU array, not the workspace)."""
        check(self.lib.gd_reshuffle_neighbors_static(C.byref(self.P), C.byref(self.nb), self.seed, int(refresh),
                                                     self._s()))

    def sample_deferred(self, table, table_bytes: int, slot: int):
        """The per-lane pass of sampling; the run's arguments go to table slot `slot`
        (the rest runs in gd_sample_table_run, then sample_audit)."""
        s = self.A.struct()
        check(self.lib.gd_sample_collisions_deferred(
            C.byref(self.P), C.byref(s), C.byref(self.nb), C.c_void_p(self.iv.data_ptr()), _ptr(self.lam),
            self.seed, GD_INTERVAL_ON_DEVICE if self.device_interval else self.interval, _ptr(self.events), None, 0,
            C.c_void_p(self.ws_ptr), self.ws_bytes, C.c_void_p(table), int(table_bytes), int(slot), self._s()))

    def sample_audit(self, flip: bool = True):
        s = self.A.struct()
        check(self.lib.gd_sample_audit(C.byref(self.P), C.byref(s), C.c_void_p(self.iv.data_ptr()),
                                       C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))
        self.interval += 1
        if flip:
            self.A.cur ^= 1

    def push(self, dt: float | None = None):
        s = self.A.struct()
        ivp = None if dt is not None else C.c_void_p(self.iv.data_ptr())
        check(self.lib.gd_push(C.byref(self.P), C.byref(s), ivp, 0.0 if dt is None else float(dt),
                               C.c_void_p(self.ws_ptr), self.ws_bytes, self._s()))
        if self.P.push != 0:
            self.moved = True

    def diffuse(self, dt: float, step: int):
        """One diffusion step of length dt (Sect. 2.4) on the current state, in place;
        `step` numbers the draws (each call of a run needs its own)."""
        s = self.A.struct()
        check(self.lib.gd_diffuse(C.byref(self.P), C.byref(s), float(dt), self.seed, int(step), self._s()))
        if self.P.diffusion != 0:
            self.moved = True

    def collide(self, max_intervals: int = 1 << 24) -> int:
        """Collision operator C(dt_coll): frozen-neighbour intervals without
        transport until the collision step is complete (its ticks wrap to 0).
        The neighbour lists are rebuilt only if the positions changed since they
        were built.  Reads the interval state after each interval (synchronises).
        Returns the number of intervals run."""
        for it in range(1, max_intervals + 1):
            if self.moved:
                self.build_neighbors()
            self.collision_rates()
            self.sample_collisions()
            if self.interval_state()["ticks"] == 0:
                return it
        raise GdError(f"collision step not complete after {max_intervals} intervals")

    # ---- spatial groups (Sect. 2.5.3) ---------------------------------------------
    def set_groups(self, n_groups: int, concurrent: bool = False, device: bool = False):
        """Split the active particles into `n_groups` contiguous Morton ranges, each
        with its own interval state; collide_groups() then schedules them.  With
        `concurrent`, every group also gets its own workspace and stream, so that
        the sampling of the groups starting at one instant overlaps (their plans
        still run one after another, as the ratio rule orders them).  With
        `device`, every group gets its own workspace and the scheduler runs on
        the device (gd_group_sched_*): one launch per stage over the groups at
        each instant, one host read per few instants."""
        torch = self.torch
        if not 1 <= n_groups <= 64:
            raise GdError("n_groups must be 1..64")
        self.n_groups = int(n_groups)
        self.gws = None
        self.gdev = bool(device)
        self._close_gsched()
        if device:
            self.gdws = []
            for _ in range(self.n_groups):
                buf = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
                self.gdws.append((buf, (buf.data_ptr() + 255) & ~255))
        if concurrent and not device:
            self.gws, self.gstreams = [], []
            for _ in range(self.n_groups):
                buf = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
                ptr = (buf.data_ptr() + 255) & ~255
                self.gws.append((buf, ptr))
                self.gstreams.append(torch.cuda.Stream(device=self.device))
        isz = C.sizeof(GdInterval)
        self.ivg = torch.zeros((self.n_groups, isz), dtype=torch.uint8, device=self.device)
        for g in range(self.n_groups):
            check(self.lib.gd_interval_init(C.c_void_p(self.ivg[g].data_ptr()), float(self.params["dt_coll"]),
                                            self._s()))
        self.gmask = torch.zeros(self.n_groups, dtype=torch.int64, device=self.device)
        self.gsched = torch.zeros(self.n_groups, dtype=torch.int64, device=self.device)  # scheduled ticks, 0: none
        self.group_lo = None
        if self.stream is not None or concurrent:  # the fills ran on torch's stream
            torch.cuda.current_stream(self.device).synchronize()
        if concurrent and not device:
            for _, ptr in self.gws:
                check(self.lib.gd_workspace_init(C.byref(self.P), C.c_void_p(ptr), self.ws_bytes, self._s()))
            self._sync_own()
        if device:
            for _, ptr in self.gdws:
                check(self.lib.gd_workspace_init(C.byref(self.P), C.c_void_p(ptr), self.ws_bytes, self._s()))
            self._sync_own()

    def _close_gsched(self):
        h = getattr(self, "gsched_h", None)
        if h:
            self._sync_own()
            check(self.lib.gd_group_sched_destroy(h))
        self.gsched_h = None

    def _collide_groups_device(self) -> list:
        """collide_groups() with the scheduler on the device."""
        if self.moved or self.group_lo is None or self.gsched_h is None or self.gsched_state != id(self.A):
            if self.moved or self.group_lo is None:
                if self.moved:
                    self.build_neighbors()
                self._group_layout()
            self._close_gsched()
            G = self.n_groups
            sa = self.A.struct()
            lo = (C.c_int32 * (G + 1))(*self.group_lo)
            wsa = (C.c_void_p * G)(*[ptr for _, ptr in self.gdws])
            h = C.c_void_p()
            check(self.lib.gd_group_sched_create(C.byref(self.P), C.byref(sa), C.byref(self.nb), lo, G,
                                                 C.c_void_p(self.ivg.data_ptr()), C.c_void_p(self.gmask.data_ptr()),
                                                 C.c_void_p(self.gsched.data_ptr()), _ptr(self.lam), _ptr(self.events),
                                                 wsa, self.ws_bytes, C.c_void_p(self.ws_ptr), self.seed, C.byref(h)))
            self.gsched_h = h
            self.gsched_state = id(self.A)
        st = self._s()
        check(self.lib.gd_group_sched_begin(self.gsched_h, self.interval, st))
        done, nxt, nlog = C.c_int32(), C.c_int64(), C.c_int32()
        batch = 2
        while True:
            check(self.lib.gd_group_sched_instants(self.gsched_h, batch, st))
            check(self.lib.gd_group_sched_read(self.gsched_h, st, C.byref(done), C.byref(nxt), C.byref(nlog), None, 0))
            if done.value:
                break
            batch = min(2 * batch, 16)
        n = nlog.value
        if n < 0:
            raise GdError("more group intervals in one collision step than the scheduler's log holds")
        log = (C.c_int64 * (3 * max(n, 1)))()
        check(self.lib.gd_group_sched_read(self.gsched_h, st, C.byref(done), C.byref(nxt), C.byref(nlog), log, n))
        self.interval = int(nxt.value)
        return [(int(log[3 * i]), int(log[3 * i + 1]), int(log[3 * i + 2])) for i in range(n)]

    def _group_layout(self):
        """Ranges over the active slots after a build, and the interaction rows (synchronises)."""
        if self.stream is not None:
            self.stream.synchronize()
        na = int(self.n_active.item())
        G = self.n_groups
        if na < G:
            raise GdError(f"{na} active particles cannot fill {G} groups")
        lo = (C.c_int32 * (G + 1))(*[g * na // G for g in range(G + 1)])
        check(self.lib.gd_group_interactions(C.byref(self.P), C.byref(self.nb), lo, G,
                                             C.c_void_p(self.gmask.data_ptr()), self._s()))
        self._sync_own()  # the rows are read below on torch's stream
        self.group_lo = [int(v) for v in lo]
        self.group_rows = [int(v) & ((1 << 64) - 1) for v in self.gmask.cpu().tolist()]

    def _sync_own(self):
        if self.stream is not None:
            self.stream.synchronize()
        else:
            self.torch.cuda.current_stream(self.device).synchronize()

    def _own_stream(self):
        return self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)

    def group_interval_state(self, g: int) -> dict:
        if self.stream is not None:
            self.stream.synchronize()
        s = GdInterval.from_buffer_copy(self.ivg[g].cpu().numpy().tobytes())
        return {name: getattr(s, name) for name, _ in GdInterval._fields_}

    def collide_groups(self) -> list:
        """Collision operator C(dt_coll) with spatial groups: each group runs its
        own frozen-neighbour intervals; at each instant the groups whose interval
        ends broadcast their masses, then the groups starting there plan in
        ascending order, each interval held within 1/16 .. 16 times the intervals
        already scheduled for the groups it interacts with (the lower limit wins
        when the two conflict; the limits are applied on the device).  A group's
        interval is sampled when it starts, against one snapshot per instant;
        its masses are broadcast when it ends.  Returns the executed intervals
        as (group, start tick, ticks).  Synchronises once per instant."""
        if getattr(self, "gdev", False):
            return self._collide_groups_device()
        T = 1 << 30
        if self.moved or self.group_lo is None:
            if self.moved:
                self.build_neighbors()
            self._group_layout()
        G, lo = self.n_groups, self.group_lo
        end = [0] * G
        tau, starting, done = 0, list(range(G)), []
        sa = self.A.struct()
        rows = C.c_void_p(self.gmask.data_ptr())
        sched = C.c_void_p(self.gsched.data_ptr())
        while True:
            if self.gws is None:
                for idx, g in enumerate(starting):
                    self._plan_and_sample(g, lo, rows, sched, idx == 0, C.c_void_p(self.ws_ptr), self._s())
            else:
                # group g's plan waits for the plan of the group before it (the
                # ratio limits read its scheduled size); its sampling runs on
                # its own stream and overlaps the next groups' work
                torch = self.torch
                own = self._own_stream()
                prev = torch.cuda.Event()
                prev.record(own)
                for g in starting:
                    sg = self.gstreams[g]
                    sg.wait_event(prev)
                    ws_g = C.c_void_p(self.gws[g][1])
                    self._rates_group(g, lo, rows, sched, True, ws_g, C.c_void_p(sg.cuda_stream))
                    prev = torch.cuda.Event()
                    prev.record(sg)
                    self._sample_group(g, lo, ws_g, C.c_void_p(sg.cuda_stream))
                for g in starting:
                    own.wait_stream(self.gstreams[g])
            if self.stream is not None:
                self.stream.synchronize()
            sizes = self.gsched.cpu().tolist()
            for g in starting:
                end[g] = tau + int(sizes[g])
                done.append((g, tau, int(sizes[g])))
            tau = min(end)
            starting = [g for g in range(G) if end[g] == tau]
            for g in starting:
                check(self.lib.gd_publish_group(C.byref(self.P), C.byref(sa), lo[g], lo[g + 1], sched, g, self._s()))
            if tau == T:
                return done

    def _rates_group(self, g, lo, rows, sched, snapshot, ws, stream):
        sa = self.A.struct()
        check(self.lib.gd_collision_rates_group(C.byref(self.P), C.byref(sa), C.byref(self.nb),
                                                C.c_void_p(self.ivg[g].data_ptr()), _ptr(self.lam), lo[g], lo[g + 1],
                                                g, self.n_groups, rows, sched, 1 if snapshot else 0, ws, self.ws_bytes,
                                                stream))

    def _sample_group(self, g, lo, ws, stream):
        sa = self.A.struct()
        check(self.lib.gd_sample_collisions_group(C.byref(self.P), C.byref(sa), C.byref(self.nb),
                                                  C.c_void_p(self.ivg[g].data_ptr()), _ptr(self.lam), self.seed,
                                                  self.interval, lo[g], lo[g + 1], _ptr(self.events), ws,
                                                  self.ws_bytes, stream))
        self.interval += 1

    def _plan_and_sample(self, g, lo, rows, sched, snapshot, ws, stream):
        self._rates_group(g, lo, rows, sched, snapshot, ws, stream)
        self._sample_group(g, lo, ws, stream)

    def transport_dt(self, limits: dict, set_step: bool = False) -> float:
        """The shared transport step of Sect. 2.6 from the particles' local
        constraints (gd_transport_dt; `limits`: dt_max and optionally the keys
        of STEP_DEFAULTS), read back to the host.  set_step: the interval
        state takes dt_coll = dt / 2 (at a collision-step boundary)."""
        lim = GdStepLimits(**dict(STEP_DEFAULTS, **limits))
        if not hasattr(self, "dt_dev"):
            self.dt_dev = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        s = self.A.struct()
        check(self.lib.gd_transport_dt(C.byref(self.P), C.byref(s), C.byref(self.nb), C.byref(lim),
                                       C.c_void_p(self.iv.data_ptr()) if set_step else None,
                                       C.c_void_p(self.dt_dev.data_ptr()), C.c_void_p(self.ws_ptr), self.ws_bytes,
                                       self._s()))
        self._sync_own()
        return float(self.dt_dev.item())

    def strang_step(self, limits: dict | None = None) -> int:
        """One transport step in the symmetric sequence of Sect. 2.6:
        C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2).  dt is 2 dt_coll of the run,
        or, with `limits`, chosen at the start of the step from the local
        constraints (transport_dt; one host read per step).  The last
        collision operator of a step and the first of the next share their
        neighbour lists.  With groups set (set_groups), the collision
        operators are the grouped ones (fixed dt only).  Returns the number of
        (group) intervals run."""
        if limits is not None:
            if getattr(self, "n_groups", 0):
                raise ValueError("steps chosen from local constraints run with a single group")
            h = 0.5 * self.transport_dt(limits, set_step=True)
        else:
            h = float(self.params["dt_coll"])
        self.last_dt = 2.0 * h
        collide = (lambda: len(self.collide_groups())) if getattr(self, "n_groups", 0) else self.collide
        n = collide()
        if self.P.diffusion != 0:
            self.diffuse(h, self.diff_step)
            self.diff_step += 1
        self.push(dt=2.0 * h)
        if self.P.diffusion != 0:
            self.diffuse(h, self.diff_step)
            self.diff_step += 1
        return n + collide()

    def step(self, rebuild: bool = True):
        """One frozen-neighbour interval: kNN, rates + plan, sampling, push."""
        if rebuild:
            self.build_neighbors()
        self.collision_rates()
        self.sample_collisions()
        if self.P.push != 0:
            self.push()

    # ---- inspection (synchronising) -----------------------------------------------
    def interval_state(self) -> dict:
        if self.stream is not None:
            self.stream.synchronize()
        raw = self.iv.cpu().numpy().tobytes()
        s = GdInterval.from_buffer_copy(raw)
        return {name: getattr(s, name) for name, _ in GdInterval._fields_}

    def status(self) -> int:
        """Device status bits of the engine's workspace, ORed with those of the
        per-group workspaces when groups run concurrently (synchronises)."""
        v = C.c_int32()
        check(self.lib.gd_status_read(C.c_void_p(self.ws_ptr), self._s(), C.byref(v)))
        out = v.value
        for g, (_, ptr) in enumerate(getattr(self, "gws", None) or []):
            check(self.lib.gd_status_read(C.c_void_p(ptr), C.c_void_p(self.gstreams[g].cuda_stream), C.byref(v)))
            out |= v.value
        if getattr(self, "gdev", False):
            for _, ptr in self.gdws:
                check(self.lib.gd_status_read(C.c_void_p(ptr), self._s(), C.byref(v)))
                out |= v.value
        return out

    def state_numpy(self) -> dict:
        return self.A.to_numpy()

    # ---- checkpoint / resume ------------------------------------------------------
    def checkpoint(self) -> dict:
        """Host copy of everything the run needs to continue as if uninterrupted:
        the particle state in its current order, the device interval state (C,
        clock, counters), the next interval index and diffusion step, and the
        seed.  The previous search's neighbour distances go along as well; they
        only seed the next search's radius.  Synchronises."""
        self._sync_own()
        return dict(state=self.A.to_numpy(), iv=self.iv.cpu().numpy().copy(), interval=int(self.interval),
                    diff_step=int(self.diff_step), seed=int(self.seed), dmax=self.dmax.cpu().numpy().copy())

    @classmethod
    def restore(cls, params: dict, ckpt: dict, **kw) -> "Engine":
        """A new engine that continues the run saved by checkpoint()."""
        eng = cls(params, ckpt["state"], seed=int(ckpt["seed"]), **kw)
        torch = eng.torch
        eng._sync_own()  # the interval state's initialisation has run
        eng.iv.copy_(torch.as_tensor(np.asarray(ckpt["iv"], np.uint8)))
        eng.dmax.copy_(torch.as_tensor(np.asarray(ckpt["dmax"], np.float64)))
        eng.interval = int(ckpt["interval"])
        eng.diff_step = int(ckpt["diff_step"])
        torch.cuda.current_stream(eng.device).synchronize()  # the copies ran on torch's stream
        return eng


class ManyRuns:
    """Engines stepped as one (gd_many_*): every stage of an interval is one
    launch over all of them.  The engines keep their own buffers; after each
    interval their bookkeeping (state buffers, cur, interval count) is
    updated as their own step() would.  `tuning` takes the keys of
    MANY_DEFAULTS (launch shapes only; results do not depend on them)."""

    def __init__(self, engines, tuning: dict | None = None):
        self.lib = load()
        self.engines = list(engines)
        self.tuning = dict(MANY_DEFAULTS, **(tuning or {}))
        n = len(self.engines)
        runs = (GdRun * n)()
        keep = []
        for i, e in enumerate(self.engines):
            e._sync_own()
            sa, sb = e.A.struct(), e.B.struct()
            sb.cur = sa.cur
            keep += [sa, sb]
            r = runs[i]
            r.p = C.pointer(e.P)
            r.a = C.pointer(sa)
            r.b = C.pointer(sb)
            r.nb = C.pointer(e.nb)
            r.iv = e.iv.data_ptr()
            r.lam_i = e.lam.data_ptr()
            r.n_events = e.events.data_ptr()
            r.ws = e.ws_ptr
            r.ws_bytes = e.ws_bytes
            r.seed = e.seed
        t = GdManyTuning(**{k: int(v) for k, v in self.tuning.items()})
        self.handle = C.c_void_p()
        check(self.lib.gd_many_create(runs, n, C.byref(t), C.byref(self.handle)))

    def interval(self, stream=None):
        """One interval of every run, enqueued on `stream` (torch's current one by default)."""
        torch = self.engines[0].torch
        st = stream if stream is not None else torch.cuda.current_stream()
        check(self.lib.gd_many_interval(self.handle, C.c_void_p(st.cuda_stream)))
        for e in self.engines:
            cur = e.A.cur
            e.A, e.B = e.B, e.A
            e.A.cur = cur ^ 1
            e.interval += 1
            if e.P.push != 0:
                e.moved = True

    def close(self):
        if self.handle:
            check(self.lib.gd_many_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CuStream:
    """A torch stream over a library stream restricted to the compute units
    [first, first + count) (gd_stream_create_cu_mask); `stream` is the torch
    object to launch and record events on.  close() releases it."""

    def __init__(self, first: int, count: int, device=None):
        import torch
        self.lib = load()
        words = (int(first) + int(count) + 31) // 32
        mask = (C.c_uint32 * max(1, words))()
        for cu in range(int(first), int(first) + int(count)):
            mask[cu // 32] |= 1 << (cu % 32)
        self.handle = C.c_void_p()
        check(self.lib.gd_stream_create_cu_mask(mask, len(mask), C.byref(self.handle)))
        self.stream = torch.cuda.ExternalStream(self.handle.value, device=device)

    def close(self):
        if self.handle:
            self.stream.synchronize()
            check(self.lib.gd_stream_destroy(self.handle))
            self.handle = C.c_void_p()
