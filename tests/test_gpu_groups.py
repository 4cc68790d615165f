"""GPU parity of collision steps with spatial groups (Sect. 2.5.3) against the
oracle's grouped run: the same schedule of group intervals (group, start,
ticks), the same masses bit for bit (dimensionless kernels) and the same
safety factor per group; one group equals the single-group step; the
interaction rows equal the oracle's."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle.pipeline import GroupedRun  # noqa: E402
from paper_2609_35967_amd import Engine, load  # noqa: E402


def _say(*a):
    print("[gpu]", *a, flush=True)


def two_speed_box(n, seed):
    st = workloads.const_box(seed, n)
    st["m"] = np.where(st["x"] >= 0.5, 1e-3, 1.0)
    return st


def _by_id(d):
    o = np.argsort(np.asarray(d["id"]).astype(np.int64))
    return {k: np.asarray(v)[o] for k, v in d.items()}


def _set(eng, G, mode):
    eng.set_groups(G, concurrent=mode == "streams", device=mode == "device")


@pytest.mark.parametrize("G,n,mode", [(8, 2048, "host"), (5, 4099, "host"), (64, 8192, "host"),
                                      (8, 2048, "streams"), (5, 4099, "streams"),
                                      (8, 2048, "device"), (5, 4099, "device"), (64, 8192, "device")])
def test_grouped_steps_match_oracle(G, n, mode):
    params = workloads.const_box_params(n)
    st = two_speed_box(n, 11)
    load()
    eng = Engine(params, st, seed=9)
    _set(eng, G, mode)
    run = GroupedRun(params, st, seed=9, n_groups=G)
    for step in range(2):
        d_gpu = eng.collide_groups()
        d_orc = run.collide_groups()
        _say("G", G, "step", step, "group intervals", len(d_gpu))
        assert not any(e["near_tie"] for e in run.log), "near tie: choose another seed"
        assert d_gpu == d_orc
        rows = [sorted(h for h in range(G) if (eng.group_rows[g] >> h) & 1) for g in range(G)]
        assert rows == [sorted(int(h) for h in s) for s in run.links]
        got = _by_id(eng.state_numpy())
        ref = _by_id(run.st)
        assert np.array_equal(got["m"], ref["m"])
        for g in range(G):
            assert eng.group_interval_state(g)["C"] == run.gC[g]
    assert eng.status() & ~0x4 == 0  # every group workspace included


def test_grouped_steps_with_inactive_particles():
    # inactive particles (M = 0) sort last and belong to no group
    n = 3000
    params = workloads.const_box_params(n)
    st = two_speed_box(n, 16)
    st["M"][::9] = 0.0
    load()
    eng = Engine(params, st, seed=8)
    eng.set_groups(6)
    run = GroupedRun(params, st, seed=8, n_groups=6)
    d_gpu = eng.collide_groups()
    d_orc = run.collide_groups()
    assert not any(e["near_tie"] for e in run.log), "near tie: choose another seed"
    assert d_gpu == d_orc
    assert eng.group_lo == run.bounds and run.bounds[-1] == n - len(range(0, n, 9))
    got, ref = _by_id(eng.state_numpy()), _by_id(run.st)
    assert np.array_equal(got["m"], ref["m"])
    assert np.array_equal(got["m"][::9], st["m"][::9])


@pytest.mark.parametrize("mode", ["host", "device"])
def test_one_group_equals_single_group_step(mode):
    n = 4096
    params = workloads.const_box_params(n)
    st = two_speed_box(n, 12)
    load()
    a = Engine(params, st, seed=3)
    _set(a, 1, mode)
    b = Engine(params, st, seed=3)
    for _ in range(2):
        da = a.collide_groups()
        nb = b.collide()
        assert len(da) == nb
    torch.cuda.synchronize()
    ga, gb = a.state_numpy(), b.state_numpy()
    assert np.array_equal(ga["m"], gb["m"])
    assert a.group_interval_state(0)["C"] == b.interval_state()["C"]


@pytest.mark.parametrize("mode", ["host", "streams", "device"])
def test_grouped_physical_disk(mode):
    n = 4096
    params = workloads.disk3d_params(n)
    st = workloads.disk3d(13, n, warm=True, params=params)
    load()
    eng = Engine(params, st, seed=4)
    _set(eng, 4, mode)
    run = GroupedRun(params, st, seed=4, n_groups=4)
    d_gpu = eng.collide_groups()
    d_orc = run.collide_groups()
    assert not any(e["near_tie"] for e in run.log), "near tie: choose another seed"
    assert d_gpu == d_orc
    got, ref = _by_id(eng.state_numpy()), _by_id(run.st)
    assert np.array_equal(got["m"], ref["m"])
    assert eng.status() & ~0x4 == 0  # every group workspace included


@pytest.mark.parametrize("mode", ["host", "streams", "device"])
def test_grouped_strang_steps_match_oracle(mode):
    """The paper's cadence with grouped collision operators on a warm disk with
    diffusion: groups are re-formed from the new Morton order after motion."""
    n = 4096
    params = dict(workloads.disk3d_params(n), diffusion="concentration", Sc=(1.0, 1.0, 1.0))
    st = workloads.disk3d(15, n, warm=True, params=params)
    load()
    eng = Engine(params, st, seed=6)
    _set(eng, 4, mode)
    run = GroupedRun(params, st, seed=6, n_groups=4)
    for step in range(2):
        n_gpu = eng.strang_step()
        res = run.strang_step()
        torch.cuda.synchronize()
        assert not any(r["mc"]["near_tie"].any() for r in res), f"near tie in step {step}: choose another seed"
        assert n_gpu == len(res)
        got, ref = _by_id(eng.state_numpy()), _by_id(run.st)
        assert np.array_equal(got["m"], ref["m"])
        np.testing.assert_allclose(got["r"], ref["r"], rtol=1e-10)
        np.testing.assert_allclose(got["ph"], ref["ph"], rtol=1e-10, atol=1e-10)
        for g in range(4):
            assert eng.group_interval_state(g)["C"] == run.gC[g]
        _say("grouped strang step", step, "group intervals", n_gpu)


@pytest.mark.parametrize("workload", ["disk3d", "disk3d_warm"])
def test_grouped_step_full_size_properties(workload):
    """The 1M disk with 8 groups, as bench.py --groups 8 runs it: every group's
    intervals tile the collision step with aligned dyadic intervals, overlapping
    intervals of interacting groups differ by at most 16 (no limit conflict
    arises on this disk), particle masses M are untouched and the status word
    is clean."""
    params, st = workloads.by_name(workload, seed=0, n=1 << 20)
    load()
    eng = Engine(params, st, seed=0)
    eng.set_groups(8)
    done = eng.collide_groups()
    _say(workload, "group intervals", len(done))
    T = 1 << 30
    for g in range(8):
        t = 0
        for s, z in sorted((s, z) for gg, s, z in done if gg == g):
            assert s == t and z >= 1 and (z & (z - 1)) == 0 and s % z == 0
            t = s + z
        assert t == T
    for g, s, z in done:
        for h, s2, z2 in done:
            if (eng.group_rows[g] >> h) & 1 and s < s2 + z2 and s2 < s + z:
                assert max(z, z2) <= 16 * min(z, z2)
    got = eng.state_numpy()
    assert np.array_equal(np.sort(got["M"]), np.sort(st["M"]))
    assert np.all(np.isfinite(got["m"])) and np.all(got["m"] > 0)
    assert eng.status() & ~0x4 == 0
