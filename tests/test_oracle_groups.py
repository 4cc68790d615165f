"""Spatial groups on the oracle (Sect. 2.5.3): one group is the single-group
collision step; the executed intervals of every group tile the collision step
with aligned dyadic intervals; interacting groups keep interval ratios of at
most 16 while no group is forced below its limits; groups with no interaction
run exactly the intervals they request; a group of fast-evolving particles
waits to refine while what it asks for is below 1/16 of a slow neighbour's
scheduled interval."""
import math

import numpy as np
import pytest

import workloads
from oracle.pipeline import GroupedRun, OracleRun

T = 1 << 30


def two_speed_box(n=2048, seed=3):
    # constant kernel, lambda_ij ~ m0/m_j: grains of mass 1e-3 on the x >= 1/2
    # side see partners 1000 times lighter than the m = 1 side (faster rates)
    st = workloads.const_box(seed, n)
    st["m"] = np.where(st["x"] >= 0.5, 1e-3, 1.0)
    return st


def clusters(n_per, G, seed=4):
    # G compact clusters in distinct top-level Morton octants, far apart
    rng = np.random.default_rng(seed)
    corners = [(0.1, 0.1, 0.1), (0.9, 0.1, 0.1), (0.1, 0.9, 0.1), (0.9, 0.9, 0.1),
               (0.1, 0.1, 0.9), (0.9, 0.1, 0.9), (0.1, 0.9, 0.9), (0.9, 0.9, 0.9)][:G]
    xs = [np.asarray(c) + 0.02 * rng.standard_normal((n_per, 3)) for c in corners]
    p = np.concatenate(xs)
    n = len(p)
    m = np.concatenate([np.full(n_per, 10.0 ** (-g)) for g in range(G)])
    return dict(id=np.arange(n, dtype=np.uint32), x=p[:, 0], y=p[:, 1], z=p[:, 2], M=np.full(n, 1.0 / n), m=m)


def _tiles(done, G):
    for g in range(G):
        iv = sorted((s, z) for gg, s, z in done if gg == g)
        t = 0
        for s, z in iv:
            assert s == t and z >= 1 and (z & (z - 1)) == 0 and s % z == 0
            t = s + z
        assert t == T


def test_one_group_is_the_single_group_step():
    params = workloads.const_box_params(2048)
    st = two_speed_box()
    a = GroupedRun(params, st, seed=2, n_groups=1)
    b = OracleRun(params, st, seed=2)
    for _ in range(2):
        da = a.collide_groups()
        db = b.collide()
        assert len(da) == len(db)
    assert np.array_equal(a.st["m"], b.st["m"])
    assert a.gC[0] == b.C and a.interval == b.interval


def test_groups_tile_the_step_and_keep_the_ratio():
    params = workloads.const_box_params(2048)
    run = GroupedRun(params, two_speed_box(), seed=5, n_groups=8)
    for _ in range(2):
        done = run.collide_groups()
        _tiles(done, 8)
    # the fast side (high groups in Morton order of x) refines more than the slow side
    count = [sum(1 for g, _, _ in done if g == gg) for gg in range(8)]
    assert max(count) > 4 * min(count)
    # no group was forced below its limits, so every interval lies within 1/16..16
    # of each interacting group's interval at the time it was planned
    for e in run.log:
        assert e["lo"] <= e["hi"]
        assert e["lo"] <= e["ticks"] <= e["hi"]
    # and some fast group's refinement waited: it ran a longer interval than it
    # asked for because a slow neighbour's scheduled interval was 16 times longer
    assert any(e["ticks"] > e["requested"] for e in run.log)


def test_overlapping_intervals_of_interacting_groups_within_16():
    params = workloads.const_box_params(2048)
    run = GroupedRun(params, two_speed_box(), seed=6, n_groups=8)
    done = run.collide_groups()
    for g, s, z in done:
        for h, s2, z2 in done:
            if h in run.links[g] and s < s2 + z2 and s2 < s + z:
                assert max(z, z2) <= 16 * min(z, z2), (g, s, z, h, s2, z2)


def test_independent_groups_run_their_requests():
    params = dict(workloads.const_box_params(2048), periodic=(0, 0, 0))
    run = GroupedRun(params, clusters(256, 4), seed=7, n_groups=4)
    run.collide_groups()
    assert all(len(s) == 0 for s in run.links)
    assert all(e["ticks"] == e["requested"] for e in run.log)
    # clusters of lighter grains (faster rates) take more intervals
    n_int = [sum(1 for e in run.log if e["group"] == g) for g in range(4)]
    assert n_int == sorted(n_int) and n_int[-1] > n_int[0]


def test_grouped_strang_steps_regroup_after_motion():
    params = dict(workloads.diffusion_ring_params("density", n=1024), kernel="const", t0=1e3, m0=1.0, eps=0.08,
                  dt_fn_max=10.0)
    st = workloads.diffusion_ring(3, 1024)
    run = GroupedRun(params, st, seed=2, n_groups=4)
    out = run.strang_step()
    first = list(run.bounds)
    out += run.strang_step()
    assert len(out) == len(run.log) and run.diff_step == 4
    assert first == run.bounds == [0, 256, 512, 768, 1024]
    _tiles([(e["group"], e["start"], e["ticks"]) for e in run.log[-4:]], 4)
