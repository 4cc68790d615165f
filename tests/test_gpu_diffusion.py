"""GPU parity of the diffusion operator (gd_diffuse, Sect. 2.4) against the CPU
oracle, element by element on the same seeded inputs, and the ring-spreading
test of Sect. 3.2 at its full size (2^20 particles) against its closed forms.

Bar: positions and velocities within 1e-12 relative (the two sides differ only
in the rounding of the transcendental functions and of the drift's algebra);
the activity flag M bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_35967_amd import Engine, load  # noqa: E402

KEYS = ("r", "th", "ph", "vr", "lth", "lph", "m", "M", "x", "y", "z")


def _say(*a):
    print("[gpu]", *a, flush=True)


def _compare(got, ref, rtol=1e-12):
    scale_r = np.abs(ref["r"]).max()
    for k in ("r", "th", "ph"):
        np.testing.assert_allclose(got[k], ref[k], rtol=rtol, atol=rtol * 1e-2 * (scale_r if k == "r" else 1.0),
                                   err_msg=k)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(got[k], ref[k], rtol=rtol, atol=rtol * 1e-1 * scale_r, err_msg=k)
    for k in ("vr", "lth", "lph"):
        scale = np.abs(ref[k]).max() + np.abs(ref["lph"]).max() / scale_r + 1e-300
        np.testing.assert_allclose(got[k], ref[k], rtol=rtol * 10, atol=rtol * scale, err_msg=k)
    assert np.array_equal(got["M"], ref["M"])


def _run_both(params, st, dts, seed=7):
    load()
    eng = Engine(params, st, seed=seed)
    P = oracle.make_problem(params)
    ref = {k: np.array(st[k], np.float64) for k in KEYS}
    ref["id"] = st["id"]
    for step, dt in enumerate(dts):
        eng.diffuse(dt, step)
        ref = oracle.diffuse(P, ref, dt, seed, step)
        ref["id"] = st["id"]
    torch.cuda.synchronize()
    return eng.state_numpy(), ref


@pytest.mark.parametrize("form", ["concentration", "density"])
def test_diffuse_disk3d_matches_oracle(form):
    n = 50000
    params = dict(workloads.disk3d_params(n), diffusion=form, Sc=(1.0, 2.0, 0.5))
    st = workloads.disk3d(9, n, warm=True, params=params)
    st["vr"] = np.random.default_rng(1).normal(0.0, 1e3, n)
    st["lth"] = np.random.default_rng(2).normal(0.0, 1e3, n) * st["r"]
    _say("disk3d", form, n)
    got, ref = _run_both(params, st, [params["dt_coll"] * 50, params["dt_coll"] * 3])
    assert not np.allclose(ref["r"], st["r"])
    _compare(got, ref)


@pytest.mark.parametrize("form,axisym,Sc", [("concentration", 1, (1.0, 1.0, 1.0)),
                                            ("density", 0, (2.0, 1.0, 0.5)),
                                            ("concentration", 0, (1.0, 1.0, 3.0))])
@pytest.mark.parametrize("St", [0.1, 10.0])
def test_diffuse_ring_matches_oracle(form, axisym, Sc, St):
    n = 5003
    params = workloads.diffusion_ring_params(form, St=St, n=n, Sc=Sc, axisym=axisym)
    st = workloads.diffusion_ring(3, n)
    D0 = 1e-4 / (1.0 + St * St)
    _say("ring", form, axisym, Sc, St)
    got, ref = _run_both(params, st, [1e-3 / D0] * 20)
    _compare(got, ref)


def test_diffuse_local_stokes_number_vint():
    # vertically integrated disk with the grain's own midplane Stokes number
    n = 4099
    params = dict(workloads.diffusion_ring_params("concentration", St=0.0, n=n, axisym=0), St0=0.5)
    st = workloads.diffusion_ring(4, n)
    st["m"] = np.random.default_rng(5).uniform(0.1, 5.0, n)
    got, ref = _run_both(params, st, [50.0] * 10)
    _compare(got, ref)


def test_diffuse_step_past_axis_and_inactive():
    n = 4096
    params = workloads.diffusion_ring_params("concentration", St=1.0, n=n, axisym=1, p=-3.0)
    st = workloads.diffusion_ring(8, n)
    st["r"] = np.full(n, 0.02)
    st["x"] = st["r"] * np.cos(st["ph"])
    st["y"] = st["r"] * np.sin(st["ph"])
    st["M"][::7] = 0.0                                 # inactive: left untouched
    got, ref = _run_both(params, st, [0.5 / 5e-5])
    crossed = (got["x"] * np.cos(st["ph"]) + got["y"] * np.sin(st["ph"])) < 0
    assert crossed.sum() > n // 20
    _compare(got, ref)
    for k in ("r", "th", "ph", "x", "y", "z"):
        assert np.array_equal(got[k][::7], st[k][::7]), k


def test_diffuse_none_and_zero_step():
    n = 1000
    st = workloads.diffusion_ring(9, n)
    params = workloads.diffusion_ring_params("none", n=n)
    load()
    eng = Engine(params, st, seed=1)
    eng.diffuse(1e6, 0)
    torch.cuda.synchronize()
    got = eng.state_numpy()
    for k in ("r", "th", "ph", "x", "y", "z"):
        assert np.array_equal(got[k], st[k]), k
    # dt = 0 moves nothing (up to the re-derived angles)
    got, ref = _run_both(workloads.diffusion_ring_params("density", n=n), st, [0.0])
    _compare(got, ref)
    np.testing.assert_allclose(got["r"], st["r"], rtol=1e-15)


def test_diffuse_single_particle():
    st = workloads.diffusion_ring(10, 1)
    got, ref = _run_both(workloads.diffusion_ring_params("density", n=1, axisym=0), st, [100.0, 200.0])
    _compare(got, ref)


@pytest.mark.parametrize("form,chi", [("concentration", 1.0), ("density", 0.0)])
def test_ring_full_size(form, chi):
    """2^20 particles to t~ = 0.1 in 500 steps: mean and variance of ln R against
    the closed forms, and 256 sampled particles against the oracle run alone
    (the step of a particle depends on nothing else)."""
    n, tt, dtt = 1 << 20, 0.1, 2e-4
    params = workloads.diffusion_ring_params(form, St=1.0, n=n)
    st = workloads.diffusion_ring(12, n)
    load()
    eng = Engine(params, st, seed=0x5EED)
    dt = dtt / (1e-4 / 2.0)
    steps = int(round(tt / dtt))
    for k in range(steps):
        eng.diffuse(dt, k)
    torch.cuda.synchronize()
    got = eng.state_numpy()
    _say("ring full size", form, "done")
    lnR = np.log(got["r"])
    mu_exact, var_exact = (2.0 + chi * -1.0) * tt, 0.05 ** 2 + 2.0 * tt
    assert abs(lnR.mean() - mu_exact) < 5.0 * math.sqrt(var_exact / n)
    assert abs(lnR.var() - var_exact) < 5.0 * var_exact * math.sqrt(2.0 / n)
    pick = np.random.default_rng(13).choice(n, 256, replace=False)
    P = oracle.make_problem(params)
    ref = {k: np.array(st[k][pick], np.float64) for k in KEYS}
    ref["id"] = st["id"][pick]
    for k in range(steps):
        ref = oracle.diffuse(P, ref, dt, 0x5EED, k)
        ref["id"] = st["id"][pick]
    sub = {k: got[k][pick] for k in KEYS}
    _compare(sub, ref, rtol=1e-11)


# ------------------------------------------------ the paper's step cadence ----
def _by_id(st):
    order = np.argsort(st["id"].astype(np.int64))
    return {k: np.asarray(v)[order] for k, v in st.items()}


def test_strang_steps_match_oracle():
    """C(dt/2) D(dt/2) T(dt) D(dt/2) C(dt/2) on a warm 3D disk, step by step
    against the oracle's composition of the same operators."""
    from oracle.pipeline import OracleRun
    n = 4096
    params = dict(workloads.disk3d_params(n), diffusion="concentration", Sc=(1.0, 1.0, 1.0))
    st = workloads.disk3d(14, n, warm=True, params=params)
    load()
    eng = Engine(params, st, seed=5)
    run = OracleRun(params, st, seed=5)
    for step in range(3):
        n_gpu = eng.strang_step()
        res = run.strang_step()
        torch.cuda.synchronize()
        assert not any(r["mc"]["near_tie"].any() for r in res), f"near tie in step {step}: choose another seed"
        assert n_gpu == len(res)
        ivs = eng.interval_state()
        assert ivs["ticks"] == 0 and ivs["C"] == run.C and ivs["n_intervals"] == run.interval
        got, ref = _by_id(eng.state_numpy()), _by_id(run.st)
        assert np.array_equal(got["m"], ref["m"])
        assert np.array_equal(got["M"], ref["M"])
        _compare(got, ref, rtol=1e-10)
        _say("strang step", step, "intervals", n_gpu, "events", ivs["n_events"])


# ------------------------------- the transport step from local constraints ----
LIMITS = dict(dt_max=1e30, c_orb=0.05, c_adv=0.5, c_diff=0.5)


@pytest.mark.parametrize("workload", ["disk3d", "additive_col"])
def test_transport_dt_matches_oracle(workload):
    """gd_transport_dt against the oracle's transport_dt, on the neighbourhood
    radii of a fresh search (a 64K warm disk with diffusion on, and the column)."""
    if workload == "disk3d":
        n = 65536
        params = dict(workloads.disk3d_params(n), diffusion="concentration", Sc=(1.0, 2.0, 0.7))
        st = workloads.disk3d(15, n, warm=True, params=params)
    else:
        n = 32768
        params = workloads.additive_col_params(n)
        st = workloads.additive_col(16, n)
    load()
    eng = Engine(params, st, seed=3)
    eng.build_neighbors()
    got = eng.transport_dt(LIMITS)
    s = eng.state_numpy()
    d = eng.dmax.cpu().numpy()
    P = oracle.make_problem(params)
    want = oracle.transport_dt(P, params.get("push", "none"), s, d, **LIMITS)
    assert math.isfinite(want) and want < 1e30
    assert got == pytest.approx(want, rel=1e-13)
    # with a cap below every particle's limit the cap is the step
    assert eng.transport_dt(dict(LIMITS, dt_max=0.5 * want)) == 0.5 * want
    assert eng.transport_dt(dict(LIMITS, dt_out=0.25 * want)) == 0.25 * want
    _say(workload, "transport dt", got)


def test_strang_steps_with_chosen_dt_match_oracle():
    """Three transport steps whose dt is chosen at the start of each step from
    the local constraints, against the oracle doing the same."""
    from oracle.pipeline import OracleRun
    n = 4096
    params = dict(workloads.disk3d_params(n), diffusion="concentration", Sc=(1.0, 1.0, 1.0))
    st = workloads.disk3d(14, n, warm=True, params=params)
    lim = dict(dt_max=2.0 * params["dt_coll"], c_orb=0.02, c_adv=0.5, c_diff=0.5)
    load()
    eng = Engine(params, st, seed=5)
    run = OracleRun(params, st, seed=5)
    dts = []
    for step in range(3):
        n_gpu = eng.strang_step(limits=lim)
        res = run.strang_step(limits=lim)
        torch.cuda.synchronize()
        assert not any(r["mc"]["near_tie"].any() for r in res), f"near tie in step {step}: choose another seed"
        assert eng.last_dt == pytest.approx(2.0 * run.dt_coll, rel=1e-13)
        dts.append(eng.last_dt)
        assert n_gpu == len(res)
        ivs = eng.interval_state()
        assert ivs["ticks"] == 0 and ivs["C"] == run.C and ivs["n_intervals"] == run.interval
        assert ivs["dt_coll"] == pytest.approx(run.dt_coll, rel=1e-13)
        got, ref = _by_id(eng.state_numpy()), _by_id(run.st)
        np.testing.assert_allclose(got["m"], ref["m"], rtol=1e-12, atol=0)
        assert np.array_equal(got["M"], ref["M"])
        _compare(got, ref, rtol=1e-10)
        _say("chosen-dt strang step", step, "dt", eng.last_dt, "intervals", n_gpu, "events", ivs["n_events"])
    assert min(dts) < lim["dt_max"]  # the local constraints chose the step, not the cap
