#!/usr/bin/env python3
"""Throughput of the collision hot path on one MI355X.

One step = one frozen-neighbour interval of the whole path on the 3D disk
annulus (1,048,576 particles, k = 32, full physics):

    gd_build_neighbors -> gd_collision_rates -> gd_sample_collisions -> gd_push

Inputs are resident in HBM before the timed region.  Prints one JSON line:
particle-intervals/s (the plain single-run form), per-interval p50/p99
latency, the dominant kernel against its roofline (timed live with HIP
events on the launch stream), and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VEC_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (FMA = 2 flops)

# Algorithmic (compulsory) HBM bytes per particle and launch, k = 32, FP64.
# The rows follow the fixed per-particle-interval accounting of the method's
# hot path (keys, sort, permute, cells, query, rates + sampling, push);
# neighbour gathers are cache hits under Morton order and are not counted.
# The sort is this build's: 30-bit keys in four 8-bit radix passes of
# (key, slot) pairs.  Intermediates that one kernel writes and the next reads
# back (the snapshot record, lambda*_i, a_i, b_i) are not compulsory and are
# not counted.
ALGO_BYTES = {
    "sort": 40 + 4 * 16 + 232,     # keys (read pos 24 + M 8, write key+slot 8); 4 radix passes; permute state
    "tree": 8,                     # cell (bucket) table
    "knn_query": 24 + 128 + 4 + 8,  # own position; write nbr row, cnt, d_i
    "rates": 128 + 4 + 8 + 40,     # nbr row, cnt, d_i; own position, M and m
    "mc": 16 + 8 + 4,              # own snapshot (m, id); write m', events
    "audit": 24,                   # m, m', M (the fixed accounting folds this into sampling)
    "push": 128,                   # spherical state and Cartesian cache, read and written
}
# The same accounting for the local column (x, y, z, v_z, St_mid, M, m state)
# and the constant-kernel box (static positions: no keys, sort, query or push
# per interval).
ALGO_BYTES_COLUMN = dict(ALGO_BYTES, sort=32 + 64 + 136, tree=4, push=40)
# Fixed bytes per particle-interval of the whole path, for the fraction of the
# HBM roofline the path reaches: ~930 B for the 3D disk, ~650 B for the
# column, and rates + sampling only (208 B) for the static box.
PATH_BYTES = {"disk3d": 930, "disk3d_warm": 930, "additive_col": 650, "const_box": 208}
PROF_KERNELS = ("sort", "tree", "knn_query", "rates", "mc", "audit", "push")
# source file of each profiled stage (the HBM counter summary is tied to it)
PROF_SOURCE = {"sort": ("gd_sort.hip",), "tree": ("gd_knn.hip",),
               "knn_query": ("gd_knn.hip", "gd_knn_tile.hip", "gd_knn_wave.hip", "gd_knn.hpp"),
               "rates": ("gd_rates.hip", "gd_physics.hpp"), "mc": ("gd_mc.hip", "gd_physics.hpp"),
               "audit": ("gd_mc.hip",), "push": ("gd_push.hip",), "diffuse": ("gd_diffuse.hip",)}
# the diffusion step on the ring: read id, the six spherical components and M
# (a constant Stokes number needs no m); write the six components and x, y, z
DIFFUSE_BYTES = 4 + 6 * 8 + 8 + 9 * 8
COPY_BYTES = 1 << 30  # the plain copy that calibrates the HBM byte counters


def source_digest(kernel):
    """Digest of the sources of a stage's kernels (a counter summary is valid
    only for the sources it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in PROF_SOURCE[kernel]:
        with open(os.path.join(ROOT, "paper_2609_35967_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the same counter's
    reading for a plain copy of known size); None if there is no summary or
    the kernel's source has changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                a, b = line.split("=", 1)
                kv[a.strip()] = b.strip()
    try:
        if kv.get("source_sha256_16") != source_digest(kernel):
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def measured_valu(kernel, launch_ms):
    """VALU issue utilisation of `kernel` from the committed counter summary:
    SQ_INSTS_VALU per dispatch x 4 cycles per wave64 instruction over the
    SIMD-cycles of a launch (1024 SIMDs at 2.4 GHz); None if there is no
    summary or the kernel's source has changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                a, b = line.split("=", 1)
                kv[a.strip()] = b.strip()
    try:
        if kv.get("source_sha256_16") != source_digest(kernel):
            return None
        insts = float(kv["valu_insts_per_dispatch"])
    except (KeyError, ValueError):
        return None
    lane_ops = insts * 64 / (launch_ms * 1e-3) / 1e12
    peak = 1024 * 16 * 2.4e9 / 1e12  # lane-operations per second, one per lane per cycle
    return dict(issue_util=round(insts * 4 / (1024 * 2.4e9 * launch_ms * 1e-3), 3),
                achieved_Tlane_ops=round(lane_ops, 2), peak_Tlane_ops=round(peak, 1))


def copy_calibration(reps):
    """A plain device copy of COPY_BYTES, `reps` times (run under rocprofv3 --pmc
    to read what FETCH_SIZE / WRITE_SIZE report for a known byte count)."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "reps": reps,
                      "GBps_read_plus_write": round(2 * COPY_BYTES / dt / 1e9, 1)}), flush=True)


class HipEvents:
    """Raw hipEvent_t handles (the library records them on its launch stream)."""

    def __init__(self):
        self.lib = C.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.lib.hipEventDestroy.argtypes = [C.c_void_p]

    def create(self):
        e = C.c_void_p()
        if self.lib.hipEventCreate(C.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def elapsed_ms(self, a, b) -> float:
        ms = C.c_float()
        rc = self.lib.hipEventElapsedTime(C.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def destroy(self, e):
        self.lib.hipEventDestroy(e)


def kernel_times(eng, hip, names, steps, step=None):
    """Run `steps` intervals with events around each named kernel; mean ms per launch."""
    import torch
    from paper_2609_35967_amd import binding
    pairs = {k: [(hip.create(), hip.create()) for _ in range(steps)] for k in names}
    for s in range(steps):
        for k in names:
            a, b = pairs[k][s]
            binding.check(eng.lib.gd_profile_events(binding.PROF[k], a, b))
        (step or eng.step)()
    torch.cuda.synchronize()
    for k in names:
        binding.check(eng.lib.gd_profile_events(binding.PROF[k], None, None))
    out = {}
    for k in names:
        t = [hip.elapsed_ms(a, b) for a, b in pairs[k]]
        out[k] = float(np.mean(t))
        for a, b in pairs[k]:
            hip.destroy(a)
            hip.destroy(b)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_interval(wl, params, seed, n, nq):
    """One interval of the oracle, as it stands, on a bounded sample: the Morton
    order of all particles, then its brute-force O(N^2) neighbour search, rates
    and sampling for `nq` sampled particles (all of them on the static box,
    whose neighbour lists are built once and not timed).  Returns (particles,
    seconds)."""
    import oracle
    params, st = workloads.by_name(wl, seed=seed, n=n if wl in ("disk3d", "disk3d_warm") else None)
    P = oracle.make_problem(params)
    if wl == "const_box":
        perm = oracle.sort_perm(oracle.morton_keys(st["x"], st["y"], st["z"], st["M"]))
        s = {k: v[perm] for k, v in st.items()}
        nbr, cnt, dmax = oracle.knn(P, s["x"], s["y"], s["z"], s["M"])
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 5.0:
            oracle.rates(P, nbr, cnt, dmax, s["m"], s["M"], s["x"], s["y"], s["z"])
            oracle.mc(P, s["id"], nbr, cnt, dmax, s["m"], s["M"], s["x"], s["y"], s["z"], params["dt_coll"], seed,
                      reps)
            reps += 1
        return n * reps, time.perf_counter() - t0
    t0 = time.perf_counter()
    perm = oracle.sort_perm(oracle.morton_keys(st["x"], st["y"], st["z"], st["M"]))
    s = {k: v[perm] for k, v in st.items()}
    q = np.sort(np.random.default_rng(seed).choice(n, min(nq, n), replace=False))
    nbr_q, cnt_q, dmax_q = oracle.knn(P, s["x"], s["y"], s["z"], s["M"], queries=q)
    nbr = np.full((n, P.k), -1, np.int32)
    cnt = np.zeros(n, np.int32)
    dmax = np.zeros(n)
    nbr[q], cnt[q], dmax[q] = nbr_q, cnt_q, dmax_q
    oracle.rates(P, nbr, cnt, dmax, s["m"], s["M"], s["x"], s["y"], s["z"], queries=q)
    oracle.mc(P, s["id"], nbr, cnt, dmax, s["m"], s["M"], s["x"], s["y"], s["z"], params["dt_coll"], seed, 0,
              queries=q)
    return len(q), time.perf_counter() - t0


def cpu_baseline(wl, params, seed, n, nq):
    """The FP64 oracle as it stands, on the host cores: one run on all of them
    (OpenMP over particles) and one on a single thread, each on a bounded
    sample of the same workload, scaled to particle-intervals/s."""
    import oracle
    cores = oracle.num_threads()
    np_all, t_all = _oracle_interval(wl, params, seed, n, nq)
    oracle.set_threads(1)
    try:
        np_one, t_one = _oracle_interval(wl, params, seed, n, max(256, nq // max(cores, 1)))
    finally:
        oracle.set_threads(cores)
    what = ("rates and sampling of every particle, neighbour lists built once" if wl == "const_box" else
            f"Morton order of all {n} particles, then brute-force O(N^2) kNN, rates and sampling of one interval "
            f"(dt = dt_coll) for the sampled particles")
    return dict(value=np_all / t_all, unit="particle-intervals/s", cores=cores, kind="oracle",
                sample=f"{what}: {np_all} particle-intervals in {t_all:.1f} s on {cores} threads, "
                       f"{np_one} in {t_one:.1f} s on 1 thread",
                value_1thread=np_one / t_one, cpu_model=_cpu_model(), host_threads=os.cpu_count())


def batch_bench(args):
    """Batched boxes: the plain per-box loop, the one-launch-per-stage form
    (launch shapes picked by the autotuner first) and the recorded graph of
    per-box launches, each over the same intervals from the same saved
    device state.  A round is one interval of every box."""
    import torch
    from paper_2609_35967_amd import load
    from paper_2609_35967_amd.batch import BoxBatch

    load()
    torch.cuda.set_device(0)
    boxes = workloads.box_batch(args.seed, nbox=args.batch)
    bb = BoxBatch(boxes, streams=args.streams)
    n = bb.n_particles
    rounds = max(2, min(args.steps, 20) // 2 * 2)

    def timed(fn, reps, per):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for r in range(reps):
            fn()
            ev[r + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]) / per
        return wall, lat

    print(f"[bench] {len(boxes)} boxes, {n} particles: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        bb.step_plain()
    rec = bb.tune()
    print(f"[bench] tuned {rec['choice']} ({len(rec['trials'])} trials, {rec['ms_per_interval']} ms)",
          file=sys.stderr, flush=True)
    saved = bb._save()
    wall_p, lat_p = timed(bb.step_plain, rounds, 1)
    print(f"[bench] plain {wall_p / rounds * 1e3:.2f} ms per round", file=sys.stderr, flush=True)
    bb._load(saved)
    bb.many(bb.tuned)
    wall_m, lat_m = timed(bb.step_many, rounds, 1)
    print(f"[bench] one launch per stage {wall_m / rounds * 1e3:.2f} ms per round", file=sys.stderr, flush=True)
    status = max(e.status() for e in bb.engines)
    ev_max = [int(e.events.max().item()) for e in bb.engines]
    heavy = int(np.argmax(ev_max))
    ev_total = sum(int(e.events.sum().item()) for e in bb.engines)
    bb._load(saved)
    bb.capture()
    wall_g, lat_g = timed(bb.replay, rounds // 2, 2)
    print(f"[bench] graph of per-box launches {wall_g / rounds * 1e3:.2f} ms per round", file=sys.stderr, flush=True)
    print(f"[bench] events of the last interval: most in one particle {ev_max[heavy]} (box {heavy}, "
          f"n={bb.engines[heavy].n}); total {ev_total}", file=sys.stderr, flush=True)
    value_m = n * rounds / wall_m
    value_p = n * rounds / wall_p
    value_g = n * rounds / wall_g

    def pct(lat, q):
        return round(float(np.percentile(lat, q)), 4)

    out = dict(
        metric="particle-intervals/s (kNN+rates+MC) at 1M; batched vs plain; p50/p99 latency",
        value=round(value_m, 1), unit="particle-intervals/s", n_gpus=1, steps=rounds, warmup=args.warmup,
        ms_per_step=round(wall_m / rounds * 1e3, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"box_batch: {len(boxes)} periodic local boxes of the annulus physics, "
                             f"{n} particles in all (N log-uniform 2^10..2^16), per-box alpha log-uniform "
                             "1e-4..1e-2 and v_frag uniform 1..10 m/s, k=32, no push",
                    n_particles=n, n_boxes=len(boxes), k=32,
                    form="one launch per stage over every box (gd_many_interval), launch shapes from the autotuner",
                    intervals=[args.warmup, args.warmup + rounds]),
        p50_ms=pct(lat_m, 50), p99_ms=pct(lat_m, 99),
        tuning=rec,
        plain=dict(value=round(value_p, 1), ms_per_step=round(wall_p / rounds * 1e3, 4), p50_ms=pct(lat_p, 50),
                   p99_ms=pct(lat_p, 99), form="plain per-box loop, eager launches on one stream"),
        graph=dict(value=round(value_g, 1), ms_per_step=round(wall_g / rounds * 1e3, 4), p50_ms=pct(lat_g, 50),
                   p99_ms=pct(lat_g, 99),
                   form=f"one HIP graph per two intervals of per-box launches, {args.streams} streams"),
        batched_over_plain=round(value_m / value_p, 3),
        events_max_per_particle=max(ev_max),
        status=status,
    )
    print(json.dumps(out), flush=True)


def _timed_loop(fn, steps):
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for s in range(steps):
        fn(s)
        ev[s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])


def diffusion_bench(args):
    """The diffusion operator on the dust-ring test of Sect. 3.2 at 2^20
    particles (concentration form, St = 1, dimensionless step 2e-4): one step
    is one gd_diffuse launch over every particle."""
    import torch
    from paper_2609_35967_amd import Engine, binding, load

    load()
    torch.cuda.set_device(0)
    n = args.n
    params = workloads.diffusion_ring_params("concentration", St=1.0, n=n, axisym=0)
    st = workloads.diffusion_ring(args.seed, n)
    eng = Engine(params, st, seed=args.seed)
    dt = 2e-4 / (1e-4 / 2.0)
    hip = HipEvents()
    for k in range(args.warmup):
        eng.diffuse(dt, k)
    pairs = [(hip.create(), hip.create()) for _ in range(args.steps)]

    def one(s):
        a, b = pairs[s]
        eng.lib.gd_profile_events(binding.PROF["diffuse"], a, b)
        eng.diffuse(dt, args.warmup + s)

    wall, lat = _timed_loop(one, args.steps)
    binding.check(eng.lib.gd_profile_events(binding.PROF["diffuse"], None, None))
    k_ms = float(np.mean([hip.elapsed_ms(a, b) for a, b in pairs]))
    value = n * args.steps / wall
    achieved = DIFFUSE_BYTES * n / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic("diffuse")
    out = dict(
        metric="particle-steps/s of the diffusion operator (Sect. 2.4)", value=round(value, 1),
        unit="particle-steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(wall / args.steps * 1e3, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"diffusion_ring: the dust-ring test of Sect. 3.2, {n} particles, ln(R/R0) ~ "
                             "N(0, 0.05^2), 1D radial disk h_g0=0.05, p=-1, q=0.5, alpha=0.04, St=1, Sc=1, "
                             "concentration form, azimuthal steps on, dimensionless step 2e-4",
                    n_particles=n),
        p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
        roofline=dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 5),
                      traffic=None if traffic is None else round(traffic / (k_ms * 1e-3) / 1e9, 2),
                      kernel="diffuse", algo_bytes_per_particle=DIFFUSE_BYTES, launch_ms=round(k_ms, 4),
                      traffic_bytes_per_launch=None if traffic is None else round(traffic)),
    )
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.make_problem(params)
        ref = {k: np.array(st[k], np.float64) for k in ("r", "th", "ph", "vr", "lth", "lph", "m", "M", "x", "y",
                                                         "z")}
        ref["id"] = st["id"]
        reps = 256
        t0 = time.perf_counter()
        for k in range(reps):
            ref = oracle.diffuse(P, ref, dt, args.seed, k)
            ref["id"] = st["id"]
        t = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=round(n * reps / t, 1), unit="particle-steps/s",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"{reps} diffusion steps of all {n} particles in {t:.1f} s")
    print(json.dumps(out), flush=True)


def strang_bench(args):
    """Transport steps in the paper's cadence C(dt/2) D(dt/2) T(dt) D(dt/2)
    C(dt/2) on the 1M disk with concentration diffusion; dt/2 = dt_coll."""
    import torch
    from paper_2609_35967_amd import Engine, load

    load()
    torch.cuda.set_device(0)
    params, st = workloads.by_name(args.workload, seed=args.seed, n=args.n)
    params = dict(params, diffusion="concentration", Sc=(1.0, 1.0, 1.0))
    eng = Engine(params, st, seed=args.seed)
    if args.groups:
        eng.set_groups(args.groups, concurrent=args.group_streams, device=args.group_device)
    n = eng.n
    for _ in range(args.warmup):
        eng.strang_step()
    counts = []
    wall, lat = _timed_loop(lambda s: counts.append(eng.strang_step()), args.steps)
    value = n * args.steps / wall
    out = dict(
        metric="particle-steps/s of the paper-cadence transport step (Sect. 2.6)", value=round(value, 1),
        unit="particle-steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(wall / args.steps * 1e3, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"{args.workload}: 3D disk annulus r in [10,100] au, {n} particles, k=32, "
                             "alpha=1e-3, v_frag=1 m/s, concentration diffusion Sc=1; one step is "
                             "C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2) with dt/2 = P(10 au)/50",
                    n_particles=n, k=32, groups=args.groups or 1),
        p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
        intervals_per_step=round(float(np.mean(counts)), 3),
        status=eng.status(),
    )
    print(json.dumps(out), flush=True)


def reshuffle_bench(args):
    """The product-kernel loop of Sect. 3.3 with static particles: before every
    neighbourhood refresh the cached neighbour indices are relabelled at
    random, then rates, plan and sampling run over the relabelled rows."""
    import torch
    from paper_2609_35967_amd import Engine, load

    load()
    torch.cuda.set_device(0)
    n = args.n
    params = dict(workloads.const_box_params(n), kernel="product")
    st = workloads.const_box(args.seed, n)
    eng = Engine(params, st, seed=args.seed)
    eng.build_neighbors()
    # the product kernel runs away (gelation at t = 1): past the first few
    # tens of intervals one particle's chain of events dominates, so the
    # default run stays in the early regime
    args.steps = min(args.steps, 20)
    args.warmup = min(args.warmup, 2)
    for s in range(args.warmup):
        eng.reshuffle_neighbors(s)
        eng.step(rebuild=False)
    print(f"[bench] reshuffling: {args.steps} timed intervals", file=sys.stderr, flush=True)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def one(s):
        a, b = pairs[s]
        a.record()
        eng.reshuffle_neighbors(args.warmup + s)
        b.record()
        eng.step(rebuild=False)

    wall, lat = _timed_loop(one, args.steps)
    r_ms = float(np.mean([a.elapsed_time(b) for a, b in pairs]))
    k = int(params["k"])
    bytes_pp = 2 * 4 * k + 4            # read and write the cached row, read cnt
    achieved = bytes_pp * n / (r_ms * 1e-3) / 1e9
    out = dict(
        metric="particle-intervals/s of the product-kernel loop with neighbour reshuffling (Sect. 3.3)",
        value=round(n * args.steps / wall, 1), unit="particle-intervals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(wall / args.steps * 1e3, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=f"const_box with the product kernel: {n} particles uniform in the periodic unit "
                             "cube, m = m0 = 1, k=32, neighbour lists built once, relabelled before every "
                             "interval", n_particles=n, k=k),
        p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
        roofline=dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 5), traffic=None, kernel="reshuffle",
                      algo_bytes_per_particle=bytes_pp, launch_ms=round(r_ms, 4), traffic_bytes_per_launch=None),
        status=eng.status(),
    )
    print(json.dumps(out), flush=True)


def groups_bench(args):
    """Collision steps C(dt_coll) without transport on the disk: the single-group
    operator against args.groups spatial groups with the ratio-16 rule, on the
    same particles (neighbour lists built once, as with static positions)."""
    import torch
    from paper_2609_35967_amd import Engine, load

    load()
    torch.cuda.set_device(0)
    params, st = workloads.by_name(args.workload, seed=args.seed, n=args.n)
    single = Engine(params, st, seed=args.seed)
    grouped = Engine(params, st, seed=args.seed)
    grouped.set_groups(args.groups, concurrent=args.group_streams, device=args.group_device)
    n = single.n
    for _ in range(max(1, args.warmup)):
        single.collide()
        grouped.collide_groups()
    counts = []
    wall_s, lat_s = _timed_loop(lambda s: counts.append(single.collide()), args.steps)
    gcounts = []
    wall_g, lat_g = _timed_loop(lambda s: gcounts.append(len(grouped.collide_groups())), args.steps)
    out = dict(
        metric="particle-collision-steps/s of the collision operator with spatial groups (Sect. 2.5.3)",
        value=round(n * args.steps / wall_g, 1), unit="particle-collision-steps/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(wall_g / args.steps * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=f"{args.workload}: 3D disk annulus r in [10,100] au, {n} particles, k=32, "
                             f"alpha=1e-3, v_frag=1 m/s; one collision step of dt_coll = P(10 au)/50 without "
                             f"transport, {args.groups} Morton-range groups", n_particles=n, groups=args.groups,
                    form=("the scheduler on the device, a workspace per group, one launch per stage over the "
                          "groups at each instant" if args.group_device else
                          "a workspace and stream per group" if args.group_streams else "one workspace and stream")),
        p50_ms=round(float(np.percentile(lat_g, 50)), 4), p99_ms=round(float(np.percentile(lat_g, 99)), 4),
        group_intervals_per_step=round(float(np.mean(gcounts)), 2),
        single=dict(value=round(n * args.steps / wall_s, 1), ms_per_step=round(wall_s / args.steps * 1e3, 4),
                    intervals_per_step=round(float(np.mean(counts)), 2)),
        status=grouped.status(),
    )
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Served stream: disk-annulus runs (N log-uniform 2^12..2^20, alpha and
    v_frag as the batched boxes, 50 intervals each) arrive as a Poisson
    process at 20 runs/s for args.serve seconds and are served under a 200 GB
    budget; then the same runs one after another in the plain single-run form."""
    import torch
    from paper_2609_35967_amd import Engine, load
    from paper_2609_35967_amd.serve import Run, Server, drive, gap_percentiles, latency_percentiles

    load()
    torch.cuda.set_device(0)
    rng = np.random.default_rng(args.seed)
    rate, intervals = 20.0, 50
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > args.serve:
            break
        arrivals.append(t)
    runs = []
    for r, ta in enumerate(arrivals):
        n = int(round(2.0 ** rng.uniform(12, 20)))
        p = workloads.disk3d_params(n, alpha=10.0 ** rng.uniform(-4, -2), v_frag=100.0 * rng.uniform(1, 10))
        runs.append(Run(rid=r, params=p, state=workloads.disk3d(args.seed * 1000 + r, n, params=p),
                        seed=args.seed * 1000 + r, intervals=intervals, arrival=ta))
    total = sum(len(r.state["x"]) for r in runs) * intervals
    print(f"[bench] {len(runs)} runs, {total} particle-intervals; serving", file=sys.stderr, flush=True)
    # warm the kernels outside the measurement
    from paper_2609_35967_amd.binding import ManyRuns
    w = Engine(runs[0].params, runs[0].state, seed=0, device_interval=True)
    w.step()
    m = ManyRuns([w])
    m.interval()
    torch.cuda.synchronize()
    m.close()
    del w, m
    def served(exclusive):
        for r in runs:
            r.done, r.finished, r.latencies_ms, r.ends_ms, r.engine = 0, 0, [], [], None
        torch.cuda.synchronize()
        srv = Server(budget_bytes=200e9, keep_results=False, exclusive=exclusive)
        t0 = time.perf_counter()
        drive(srv, [(r.arrival, r) for r in runs], lambda: time.perf_counter() - t0)
        wall = time.perf_counter() - t0
        srv.close()
        p50, p99 = latency_percentiles(srv.finished)
        g50, g99 = gap_percentiles(srv.finished)
        print(f"[bench] served ({'tiers in turn' if exclusive else 'tiers side by side'}) in {wall:.2f} s, "
              f"{srv.rounds} tier rounds, p50/p99 {p50:.3f}/{p99:.3f} ms, gap p50/p99 {g50:.3f}/{g99:.3f} ms",
              file=sys.stderr, flush=True)
        return dict(wall_s=round(wall, 3), tier_rounds=srv.rounds, p50_ms=round(p50, 3), p99_ms=round(p99, 3),
                    gap_p50_ms=round(g50, 3), gap_p99_ms=round(g99, 3))

    side = served(False)
    turn = served(True)
    wall_s = turn["wall_s"]
    # capacity: the same runs all submitted at once
    sat = Server(budget_bytes=200e9, keep_results=False)
    for r in runs:
        r.done, r.finished, r.latencies_ms, r.ends_ms, r.engine = 0, 0, [], [], None
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    drive(sat, [(0.0, r) for r in runs], lambda: 1.0)
    sat_s = time.perf_counter() - ts0
    srounds = sat.rounds
    sat.close()
    print(f"[bench] saturated {sat_s:.2f} s, {srounds} tier rounds; plain form", file=sys.stderr, flush=True)
    # the same runs in the plain single-run form, one after another
    plain_lat = []
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for r in runs:
        e = Engine(r.params, r.state, seed=r.seed)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(intervals + 1)]
        ev[0].record()
        for s_ in range(intervals):
            e.step()
            ev[s_ + 1].record()
        torch.cuda.synchronize()
        plain_lat += [ev[i].elapsed_time(ev[i + 1]) for i in range(intervals)]
        del e
    plain_s = time.perf_counter() - tp0
    out = dict(
        metric="particle-intervals/s (kNN+rates+MC) at 1M; batched vs plain; p50/p99 latency",
        value=round(total / wall_s, 1), unit="particle-intervals/s", n_gpus=1, steps=intervals, warmup=0,
        ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=f"served stream: {len(runs)} disk-annulus runs arriving at 20 runs/s over {args.serve} s "
                             "(Poisson), N log-uniform 2^12..2^20, alpha log-uniform 1e-4..1e-2, v_frag uniform "
                             f"1..10 m/s, {intervals} intervals each, 200 GB budget, k=32",
                    n_runs=len(runs), particle_intervals=total,
                    form="served: size tiers (N <= 2^14, <= 2^17, larger), not in lock-step, taking turns on one "
                         "stream (two rounds queued); a tier round is one launch per stage over a group of its runs "
                         "(at most 2^19 particles, gd_many_interval)"),
        wall_s=turn["wall_s"], tier_rounds=turn["tier_rounds"],
        p50_ms=turn["p50_ms"], p99_ms=turn["p99_ms"],
        latency="GPU time of the round that holds the interval",
        gap_p50_ms=turn["gap_p50_ms"], gap_p99_ms=turn["gap_p99_ms"],
        side_by_side=dict(side, value=round(total / side["wall_s"], 1),
                          form="the same tiers each on a stream of its own, running side by side"),
        plain=dict(value=round(total / plain_s, 1), wall_s=round(plain_s, 3),
                   p50_ms=round(float(np.percentile(plain_lat, 50)), 3),
                   p99_ms=round(float(np.percentile(plain_lat, 99)), 3),
                   form="the same runs one after another, plain single-run form"),
        saturated=dict(value=round(total / sat_s, 1), wall_s=round(sat_s, 3), tier_rounds=srounds,
                       form="the same runs all submitted at once, tiers side by side"),
        saturated_over_plain=round(plain_s / sat_s, 3),
    )
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="disk3d", choices=["disk3d", "disk3d_warm", "additive_col", "const_box"])
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=98304, help="particles in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rates-fp32", action="store_true",
                    help="the single-precision pair-rate form (FP64 positions, distances and push)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="REPS",
                    help="only run a plain 1 GiB device copy REPS times (HBM counter calibration)")
    ap.add_argument("--batch", type=int, default=0, metavar="NBOX",
                    help="the batched-boxes configuration instead: NBOX periodic local boxes "
                         "(N log-uniform 2^10..2^16), the plain per-box loop against the recorded graph")
    ap.add_argument("--streams", type=int, default=8, help="streams of the batched graph")
    ap.add_argument("--serve", type=float, default=0.0, metavar="SECONDS",
                    help="the served-stream configuration instead: Poisson arrivals (20 runs/s) of disk-annulus "
                         "runs for SECONDS, served under a 200 GB budget, against the same runs one after another")
    ap.add_argument("--diffusion", action="store_true",
                    help="the diffusion operator on the 2^20-particle dust-ring test instead")
    ap.add_argument("--strang", action="store_true",
                    help="paper-cadence transport steps C D T D C on the disk instead")
    ap.add_argument("--group-streams", action="store_true",
                    help="with --groups: a workspace and stream per group, so groups' sampling overlaps")
    ap.add_argument("--group-device", action="store_true",
                    help="with --groups: the group scheduler on the device (gd_group_sched_*)")
    ap.add_argument("--reshuffle", action="store_true",
                    help="the product-kernel loop with neighbour reshuffling instead")
    ap.add_argument("--groups", type=int, default=0, metavar="G",
                    help="collision steps with G spatial groups against the single group instead")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.diffusion or args.strang or args.groups or args.reshuffle:
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        if args.reshuffle:
            reshuffle_bench(args)
        elif args.diffusion:
            diffusion_bench(args)
        elif args.strang:  # with --groups G: grouped collision operators
            strang_bench(args)
        else:
            groups_bench(args)
        return
    if args.batch or args.serve:
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        if args.serve:
            serve_bench(args)
        else:
            batch_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs the single-GPU path only (asked for --gpus {args.gpus}); the multi-GPU "
              "split is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_35967_amd import Engine, load

    load()
    torch.cuda.set_device(0)
    wl = args.workload
    n_arg = args.n if wl in ("disk3d", "disk3d_warm") else None
    params, st = workloads.by_name(wl, seed=args.seed, n=n_arg)
    if args.rates_fp32:
        params["rates_fp32"] = 1
    eng = Engine(params, st, seed=args.seed)
    n = eng.n
    hip = HipEvents()
    static = wl == "const_box"  # positions never move: neighbour lists built once (App. A test)
    knn_once_ms = None
    if static:
        a, b = hip.create(), hip.create()
        from paper_2609_35967_amd import binding as _b
        torch.cuda.synchronize()
        _b.check(eng.lib.gd_profile_events(_b.PROF["knn_query"], a, b))
        eng.build_neighbors()
        torch.cuda.synchronize()
        _b.check(eng.lib.gd_profile_events(_b.PROF["knn_query"], None, None))
        knn_once_ms = hip.elapsed_ms(a, b)
    step = (lambda: eng.step(rebuild=False)) if static else eng.step
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel breakdown on a short pass (untimed for the headline)
    names = ("rates", "mc", "audit") if static else PROF_KERNELS
    brk = kernel_times(eng, hip, names, max(5, min(20, args.steps // 4)), step)
    dom = max(brk, key=brk.get)

    # timed region: the headline loop; events per interval and around the dominant kernel
    from paper_2609_35967_amd import binding
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    dpairs = [(hip.create(), hip.create()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for s_ in range(args.steps):
        a, b = dpairs[s_]
        eng.lib.gd_profile_events(binding.PROF[dom], a, b)
        step()
        ev[s_ + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    binding.check(eng.lib.gd_profile_events(binding.PROF[dom], None, None))
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    dom_ms = float(np.mean([hip.elapsed_ms(a, b) for a, b in dpairs]))
    ivs = eng.interval_state()
    status = eng.status()
    wall = t1 - t0
    value = n * args.steps / wall

    algo = ALGO_BYTES_COLUMN if wl in ("additive_col", "const_box") else ALGO_BYTES
    achieved = algo[dom] * n / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom) if wl == "disk3d" else None
    roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5),
                    traffic=None if traffic is None else round(traffic / (dom_ms * 1e-3) / 1e9, 2), kernel=dom,
                    algo_bytes_per_particle=algo[dom], launch_ms=round(dom_ms, 4),
                    traffic_bytes_per_launch=None if traffic is None else round(traffic))
    valu = measured_valu(dom, dom_ms) if wl == "disk3d" else None
    if valu is not None:
        roofline["valu"] = valu
    out = dict(
        metric="particle-intervals/s (kNN+rates+MC) at 1M; batched vs plain; p50/p99 latency",
        value=round(value, 1), unit="particle-intervals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(wall / args.steps * 1e3, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64+f32-rates" if args.rates_fp32 else "f64", data="synthetic",
        config=dict(workload=WORKLOAD_TEXT[wl].format(n=n), n_particles=n, k=int(params["k"]),
                    form="plain (single run)", rates="fp32 pairs, fp64 sums" if args.rates_fp32 else "fp64"),
        p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
        breakdown_ms={k: round(v, 4) for k, v in brk.items()},
        path_fraction_of_hbm=round(PATH_BYTES[wl] * value / (HBM_PEAK_GBS * 1e9), 5),
        path_bytes_per_particle_interval=PATH_BYTES[wl],
        roofline=roofline,
        interval=dict(dt_exe=ivs["dt_exe"], C=ivs["C"], n_events_last=ivs["n_events"],
                      n_intervals=ivs["n_intervals"], time=ivs["time"], status=status),
    )
    if knn_once_ms is not None:
        out["knn_once_ms"] = round(knn_once_ms, 4)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, params, args.seed, n, args.cpu_sample)
    print(json.dumps(out), flush=True)


WORKLOAD_TEXT = {
    "disk3d": ("disk3d: 3D disk annulus r in [10,100] au, {n} particles, k=32, alpha=1e-3, v_frag=1 m/s, "
               "Brownian+OC07, sticking/erosion/fragmentation, one push per interval"),
    "disk3d_warm": ("disk3d_warm: 3D disk annulus r in [10,100] au, {n} particles, grain radius log-uniform "
                    "1 um..1 mm, k=32, alpha=1e-3, v_frag=1 m/s, Brownian+OC07, sticking/erosion/fragmentation, "
                    "one push per interval"),
    "additive_col": ("additive_col: local column, {n} particles, additive kernel, k=32, z ~ N(0, H=1), "
                     "St log-uniform 1e-4..1e-1, one local settling push per interval"),
    "const_box": ("const_box: periodic unit cube, {n} particles, constant kernel, k=32, static positions "
                  "(neighbour lists built once, timed apart as knn_once_ms)"),
}


if __name__ == "__main__":
    main()
