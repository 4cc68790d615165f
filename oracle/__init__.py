"""Plain FP64 CPU oracle for the collision hot path of arXiv 2609.35967.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library: the C file ``gd_oracle.c`` restates every step of the
method from the paper, and this module only marshals numpy arrays into it.

Steps and the passages they follow (section numbers of the paper):
  morton_keys / sort_perm   Morton order of the neighbour search (Sect. 2.5.1)
  knn                       N_K nearest neighbours incl. self (Sect. 2.5.1)
  rates                     eq:rate / App. A kernels, channels (Sect. 2.5.1-2.5.2)
  plan                      controller bins, dt_fn,req, halving (Sect. 2.5.3)
  mc                        Gillespie sampling on the frozen neighbourhood (Sect. 2.5.3)
  audit                     safety-factor audit (Sect. 2.5.3)
  push_local, push_global   staggered semi-analytic push (Sect. 2.3.3)
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math
import os
import subprocess
import tempfile
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

KERNELS = {"const": 0, "additive": 1, "product": 2, "physical": 3}
DIFFUSION = {"none": 0, "concentration": 1, "density": 2}
NBIN = 128


def build(force: bool = False) -> str:
    """Compile gd_oracle.c into liboracle.so (gcc, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32), ("k", C.c_int32), ("nbin_min", C.c_int32),
        ("erosion", C.c_int32), ("grouping", C.c_int32),
        ("periodic", C.c_int32 * 3), ("L", C.c_double * 3), ("rmax", C.c_double),
        ("t0", C.c_double), ("m0", C.c_double),
        ("eps", C.c_double), ("dt_fn_max", C.c_double),
        ("rho_s", C.c_double), ("s_min", C.c_double), ("v_frag", C.c_double),
        ("GM", C.c_double), ("Sigma_g0", C.c_double), ("R0", C.c_double), ("p", C.c_double),
        ("q", C.c_double), ("h_g0", C.c_double), ("alpha", C.c_double), ("mu_mH", C.c_double),
        ("sigma_H2", C.c_double), ("s0", C.c_double), ("St0", C.c_double),
        ("r_in", C.c_double), ("r_out", C.c_double),
        ("drag", C.c_int32), ("brownian", C.c_int32), ("turbulence", C.c_int32), ("caps", C.c_int32),
        ("diffusion", C.c_int32), ("vint", C.c_int32), ("axisym", C.c_int32), ("pad_", C.c_int32),
        ("Sc", C.c_double * 3), ("St_diff", C.c_double),
    ]


def make_problem(cfg: dict) -> Problem:
    """Oracle problem struct from a workload parameter dict (see workloads)."""
    P = Problem()
    P.kernel = KERNELS[cfg["kernel"]]
    P.k = int(cfg["k"])
    P.nbin_min = int(cfg.get("nbin_min", max(2 * int(cfg["k"]), 64)))
    P.erosion = int(cfg.get("erosion", 1))
    P.grouping = int(cfg.get("grouping", 1))
    per = cfg.get("periodic", (0, 0, 0))
    L = cfg.get("L", (1.0, 1.0, 1.0))
    for a in range(3):
        P.periodic[a] = int(per[a])
        P.L[a] = float(L[a])
    P.rmax = float(cfg.get("rmax", np.inf))
    for name in ("t0", "m0", "eps", "dt_fn_max", "rho_s", "s_min", "v_frag", "GM", "Sigma_g0", "R0",
                 "p", "q", "h_g0", "alpha", "mu_mH", "sigma_H2", "s0", "St0", "r_in", "r_out"):
        setattr(P, name, float(cfg.get(name, 0.0)))
    for name in ("drag", "brownian", "turbulence", "caps", "vint", "axisym"):
        setattr(P, name, int(cfg.get(name, 0)))
    P.diffusion = DIFFUSION[cfg.get("diffusion", "none")]
    Sc = cfg.get("Sc", (1.0, 1.0, 1.0))
    for a in range(3):
        P.Sc[a] = float(Sc[a])
    P.St_diff = float(cfg.get("St_diff", 0.0))
    return P


def _declare(L):
    """Argument and result types of the oracle's exported functions."""
    vp = C.c_void_p
    i64 = C.c_int64
    d = C.c_double
    L.orc_philox4x32_10.argtypes = [vp, vp, vp]
    L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, vp]
    L.orc_morton3_10.argtypes = [C.c_uint32] * 3
    L.orc_morton3_10.restype = C.c_uint32
    L.orc_morton_keys.argtypes = [i64, vp, vp, vp, vp, vp]
    L.orc_knn.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp]
    L.orc_frag_moments.argtypes = [d, d, vp, vp]
    L.orc_rates.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.orc_bin_of.argtypes = [d]
    L.orc_bin_of.restype = C.c_int32
    L.orc_plan.argtypes = [vp, i64, vp, vp, vp, vp, d, i64, d, vp, vp, vp, vp]
    L.orc_mc.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, C.c_uint64,
                         C.c_uint32, vp, vp, vp, C.c_int32, vp, vp, vp]
    L.orc_audit.argtypes = [vp, i64, vp, vp, vp, vp, vp, d, vp]
    L.orc_push_local.argtypes = [i64, vp, vp, vp, vp, d]
    L.orc_push_global.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d]
    L.orc_pair_rate.argtypes = [vp, d, d, d, d, d, d, d, vp]
    L.orc_gas_at.argtypes = [vp, d, d, vp]
    L.orc_oc07.argtypes = [d, d, d, d]
    L.orc_oc07.restype = d
    L.orc_reshuffle_index.argtypes = [i64, C.c_uint64, C.c_uint32, i64]
    L.orc_reshuffle_index.restype = i64
    L.orc_reshuffle.argtypes = [i64, C.c_int32, vp, vp, i64, C.c_uint64, C.c_uint32]
    L.orc_diff_coeffs.argtypes = [vp, d, d, d, vp]
    L.orc_diff_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, vp]
    L.orc_diffuse.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, C.c_uint64,
                              C.c_uint32]
    L.orc_transport_dt.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, d, d, d, d]
    L.orc_transport_dt.restype = d
    L.orc_fsum.argtypes = [i64, vp]
    L.orc_fsum.restype = d
    L.orc_num_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _declare(C.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def planted(*edits):
    """Swap in a copy of the oracle with each (old, new) text edit applied to
    gd_oracle.c, built in a temporary folder: a test that plants a mistake in
    the oracle checks that its pins reject it.  Every `old` must occur in the
    source exactly once."""
    global _lib
    src = open(_SRC).read()
    for old, new in edits:
        if src.count(old) != 1:
            raise ValueError(f"planted edit does not match exactly once: {old!r}")
        src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as tmp:
        c_path = os.path.join(tmp, "gd_oracle_planted.c")
        so_path = os.path.join(tmp, "liboracle_planted.so")
        with open(c_path, "w") as f:
            f.write(src)
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", so_path, c_path, "-lm"])
        saved = lib()
        with _lock:
            _lib = _declare(C.CDLL(so_path))
        try:
            yield
        finally:
            with _lock:
                _lib = saved


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------- #
def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def uniforms(seed: int, pid: int, interval: int, event: int):
    u = np.zeros(4, np.float64)
    lib().orc_uniforms(C.c_uint64(seed), pid, interval, event, _p(u))
    return u


def morton3_10(qx, qy, qz) -> int:
    return int(lib().orc_morton3_10(qx, qy, qz))


def morton_keys(x, y, z, M):
    x, y, z, M = (_c(a, np.float64) for a in (x, y, z, M))
    keys = np.zeros(len(x), np.uint32)
    lib().orc_morton_keys(len(x), _p(x), _p(y), _p(z), _p(M), _p(keys))
    return keys


def sort_perm(keys):
    """Stable ascending order of the Morton keys (library sort as a step)."""
    return np.argsort(np.asarray(keys), kind="stable").astype(np.int64)


def knn(P: Problem, x, y, z, M, queries=None):
    x, y, z, M = (_c(a, np.float64) for a in (x, y, z, M))
    n = len(x)
    q = None if queries is None else _c(queries, np.int64)
    nq = n if q is None else len(q)
    nbr = np.full((nq, P.k), -1, np.int32)
    cnt = np.zeros(nq, np.int32)
    dmax = np.zeros(nq, np.float64)
    lib().orc_knn(C.byref(P), n, _p(x), _p(y), _p(z), _p(M), nq, _p(q), _p(nbr), _p(cnt), _p(dmax))
    return nbr, cnt, dmax


def frag_moments(s_i: float, s_min: float):
    a = C.c_double()
    b = C.c_double()
    lib().orc_frag_moments(s_i, s_min, C.byref(a), C.byref(b))
    return a.value, b.value


def rates(P: Problem, nbr, cnt, dmax, m_snap, M, x, y, z, want_pairs=False, queries=None):
    """Rates of every slot, or of the slots in `queries` (outputs in query order)."""
    n = len(cnt)
    nbr = _c(nbr, np.int32)
    cnt = _c(cnt, np.int32)
    dmax, m_snap, M, x, y, z = (_c(a, np.float64) for a in (dmax, m_snap, M, x, y, z))
    q = None if queries is None else _c(queries, np.int64)
    nq = n if q is None else len(q)
    lam = np.zeros(nq)
    a = np.zeros(nq)
    b = np.zeros(nq)
    pairs = np.zeros((nq, P.k)) if want_pairs else None
    lib().orc_rates(C.byref(P), n, nq, _p(q), _p(nbr), _p(cnt), _p(dmax), _p(m_snap), _p(M), _p(x), _p(y),
                    _p(z), _p(lam), _p(a), _p(b), _p(pairs))
    return lam, a, b, pairs


def bin_of(m: float) -> int:
    return int(lib().orc_bin_of(m))


def plan(P: Problem, m_snap, M, a, b, dt_coll: float, ticks: int, Cfac: float):
    """Returns dict(dt_req, dt_exe, margin, exe_ticks, group_of, gM)."""
    m_snap, M, a, b = (_c(v, np.float64) for v in (m_snap, M, a, b))
    out = np.zeros(3)
    et = np.zeros(1, np.int64)
    group_of = np.zeros(NBIN, np.int32)
    gM = np.zeros(NBIN)
    lib().orc_plan(C.byref(P), len(M), _p(m_snap), _p(M), _p(a), _p(b), dt_coll, int(ticks), Cfac,
                   _p(out), _p(et), _p(group_of), _p(gM))
    return dict(dt_req=out[0], dt_exe=out[1], margin=out[2], exe_ticks=int(et[0]),
                group_of=group_of, gM=gM)


def mc(P: Problem, ids, nbr, cnt, dmax, m_snap, M, x, y, z, dt_exe, seed, interval, log_cap=0, queries=None):
    """Sampling of every slot, or of the slots in `queries` (outputs in query order)."""
    n_all = len(cnt)
    q = None if queries is None else _c(queries, np.int64)
    n = n_all if q is None else len(q)
    ids = _c(ids, np.uint32)
    nbr = _c(nbr, np.int32)
    cnt = _c(cnt, np.int32)
    dmax, m_snap, M, x, y, z = (_c(v, np.float64) for v in (dmax, m_snap, M, x, y, z))
    m_out = np.zeros(n)
    ev = np.zeros(n, np.int32)
    tie = np.zeros(n, np.uint8)
    ls = lc = lt = None
    if log_cap > 0:
        ls = np.full((n, log_cap), -1, np.int32)
        lc = np.full((n, log_cap), -1, np.int32)
        lt = np.full((n, log_cap), -1, np.int32)
    lib().orc_mc(C.byref(P), n_all, n, _p(q), _p(ids), _p(nbr), _p(cnt), _p(dmax), _p(m_snap), _p(M), _p(x),
                 _p(y), _p(z),
                 float(dt_exe), C.c_uint64(seed), int(interval) & 0xFFFFFFFF, _p(m_out), _p(ev), _p(tie),
                 int(log_cap), _p(ls), _p(lc), _p(lt))
    return dict(m=m_out, events=ev, near_tie=tie.astype(bool), log_slot=ls, log_chan=lc, log_type=lt)


def audit(P: Problem, m_snap, m_new, M, group_of, gM, Cfac):
    m_snap, m_new, M, gM = (_c(v, np.float64) for v in (m_snap, m_new, M, gM))
    group_of = _c(group_of, np.int32)
    out = np.zeros(3)
    lib().orc_audit(C.byref(P), len(M), _p(m_snap), _p(m_new), _p(M), _p(group_of), _p(gM), Cfac, _p(out))
    return dict(C=out[0], worst=out[1], margin=out[2])


def push_local(z, vz, st_mid, M, dt):
    z = np.array(z, np.float64)
    vz = np.array(vz, np.float64)
    st_mid = _c(st_mid, np.float64)
    M = _c(M, np.float64)
    lib().orc_push_local(len(z), _p(z), _p(vz), _p(st_mid), _p(M), float(dt))
    return z, vz


def push_global(P: Problem, st: dict, dt: float) -> dict:
    """Advance a copy of the spherical state dict by dt (keys r, th, ph, vr, lth, lph, m, M, x, y, z)."""
    s = {k: np.array(st[k], np.float64) for k in ("r", "th", "ph", "vr", "lth", "lph", "m", "M", "x", "y", "z")}
    lib().orc_push_global(C.byref(P), len(s["r"]), _p(s["r"]), _p(s["th"]), _p(s["ph"]), _p(s["vr"]),
                          _p(s["lth"]), _p(s["lph"]), _p(s["m"]), _p(s["M"]), _p(s["x"]), _p(s["y"]),
                          _p(s["z"]), float(dt))
    return s


def pair_rate(P: Problem, xi, yi, zi, di, mi, mj, Mj):
    out = np.zeros(6)
    lib().orc_pair_rate(C.byref(P), xi, yi, zi, di, mi, mj, Mj, _p(out))
    return dict(lam_star=out[0], type=int(out[1]), rate0=out[2], rate1=out[3], Ng=out[4], V=out[5])


def gas_at(P: Problem, R, Z):
    out = np.zeros(9)
    lib().orc_gas_at(C.byref(P), R, Z, _p(out))
    keys = ("OmK", "hg", "Hg", "cs", "r", "rhog", "eta", "vgphi", "stfac")
    return dict(zip(keys, out))


def oc07(St1, St2, Vg2, tke):
    return lib().orc_oc07(St1, St2, Vg2, tke)


def reshuffle_index(N: int, seed: int, refresh: int, j: int) -> int:
    """pi(j) for the random bijection of [0, N) drawn for `refresh` (product-kernel test)."""
    return int(lib().orc_reshuffle_index(N, C.c_uint64(seed), refresh, j))


def reshuffle(nbr, cnt, N: int, seed: int, refresh: int):
    """Cached neighbour rows with every index but slot 0 relabelled by pi."""
    nb = _c(nbr, np.int32).copy()
    n, k = nb.shape
    lib().orc_reshuffle(n, k, _p(nb), _p(_c(cnt, np.int32)), N, C.c_uint64(seed), refresh)
    return nb


def diff_coeffs(P: Problem, R, Z, s):
    """Diffusion coefficients at cylindrical (R, Z) for grain diameter s:
    D_R, D_Z, D_phi, dD_R/dR, dD_Z/dZ, dln rho_g/dR, dln rho_g/dZ, ln rho_g."""
    out = np.zeros(8)
    lib().orc_diff_coeffs(C.byref(P), float(R), float(Z), float(s), _p(out))
    keys = ("D_R", "D_Z", "D_phi", "dDR_dR", "dDZ_dZ", "dlnrho_dR", "dlnrho_dZ", "lnrho")
    return dict(zip(keys, out))


def diff_normals(seed: int, pid: int, step: int):
    out = np.zeros(3)
    lib().orc_diff_normals(C.c_uint64(seed), pid, step, _p(out))
    return out


def diffuse(P: Problem, st: dict, dt: float, seed: int, step: int) -> dict:
    """One diffusion step (Sect. 2.4) on a copy of the spherical state dict
    (keys id, r, th, ph, vr, lth, lph, m, M, x, y, z)."""
    s = {k: np.array(st[k], np.float64) for k in ("r", "th", "ph", "vr", "lth", "lph", "m", "M", "x", "y", "z")}
    s["id"] = _c(st["id"], np.uint32)
    lib().orc_diffuse(C.byref(P), len(s["r"]), _p(s["id"]), _p(s["r"]), _p(s["th"]), _p(s["ph"]), _p(s["vr"]),
                      _p(s["lth"]), _p(s["lph"]), _p(s["m"]), _p(s["M"]), _p(s["x"]), _p(s["y"]), _p(s["z"]),
                      float(dt), C.c_uint64(seed), step)
    return s


PUSH_KINDS = {"none": 0, "local": 1, "global": 2}


def transport_dt(P: Problem, push: str, st: dict, d, dt_max: float, dt_out: float = math.inf,
                 c_orb: float = 0.05, c_adv: float = 0.5, c_diff: float = 0.5) -> float:
    """The shared transport step of Sect. 2.6 over the active particles of the
    state dict `st`, with d the neighbourhood radii (reading R36 in the C source)."""
    n = len(st["M"])
    zero = np.zeros(n)

    def arr(k):
        return _c(st[k], np.float64) if k in st and st[k] is not None else zero

    a = {k: arr(k) for k in ("x", "y", "r", "th", "vr", "lth", "lph", "vz", "m", "M")}
    dd = _c(d, np.float64)
    return float(lib().orc_transport_dt(C.byref(P), PUSH_KINDS[push], n, _p(a["x"]), _p(a["y"]), _p(a["r"]),
                                        _p(a["th"]), _p(a["vr"]), _p(a["lth"]), _p(a["lph"]), _p(a["vz"]),
                                        _p(a["m"]), _p(a["M"]), _p(dd), float(dt_max), float(dt_out),
                                        float(c_orb), float(c_adv), float(c_diff)))


def fsum(v):
    v = _c(v, np.float64)
    return lib().orc_fsum(len(v), _p(v))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def set_tie_margin(eps: float) -> None:
    """Relative margin below which mc() flags a decision as a near-tie (default 1e-12)."""
    lib().orc_set_tie_margin(C.c_double(eps))
