"""Serving (Server): runs that arrive at different rounds, admitted under an
HBM budget that makes some of them wait, each end in the state of the same
run stepped alone."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_35967_amd import Engine, load  # noqa: E402
from paper_2609_35967_amd.serve import Run, Server  # noqa: E402


def _say(*a):
    print("[gpu]", *a, flush=True)


def _runs():
    rng = np.random.default_rng(11)
    out = []
    for r, (n, arrive, iv) in enumerate([(6000, 0, 4), (3000, 0, 3), (9000, 1, 3), (4000, 2, 5), (5000, 2, 2)]):
        p = workloads.disk3d_params(n, alpha=10.0 ** rng.uniform(-4, -2), v_frag=100.0 * rng.uniform(1, 10))
        st = workloads.disk3d(100 + r, n, warm=True, params=p)
        out.append((Run(rid=r, params=p, state=st, seed=500 + r, intervals=iv), arrive))
    return out


def _state(e):
    st = e.state_numpy()
    st["iv"] = e.interval_state()
    st["nbr"] = e.nbr.cpu().numpy()
    return st


def test_served_runs_match_alone():
    load()
    runs = _runs()
    ref = {}
    for run, _ in runs:
        e = Engine(run.params, run.state, seed=run.seed)
        for _ in range(run.intervals):
            e.step()
        ref[run.rid] = _state(e)
    lib = load()
    sizes = sorted(Server.run_bytes(lib, r.params, len(r.state["x"])) for r, _ in runs)
    srv = Server(budget_bytes=sizes[-1] + sizes[-2] + 1, streams=3)
    rnd = 0
    waited = 0
    while True:
        for run, arrive in runs:
            if arrive == rnd:
                srv.submit(run)
        srv.admit()
        waited += len(srv.waiting)
        srv.round()
        rnd += 1
        if srv.idle() and rnd > max(a for _, a in runs):
            break
        assert rnd < 100
    _say("served", len(srv.finished), "runs in", rnd, "rounds; run-rounds spent waiting:", waited)
    assert waited > 0 and len(srv.finished) == len(runs)
    for run in srv.finished:
        got = _state(run.engine)
        want = ref[run.rid]
        for key in ("id", "x", "y", "z", "M", "m", "nbr"):
            assert np.array_equal(got[key], want[key]), f"run {run.rid}: {key} differs"
        for key in ("time", "ticks", "n_intervals", "n_events", "C"):
            assert got["iv"][key] == want["iv"][key], f"run {run.rid}: interval {key} differs"
        assert run.engine.status() == 0
