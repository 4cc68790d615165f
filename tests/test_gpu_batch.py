"""Batched boxes (BoxBatch): every box's state after the recorded graph's
replays, and after the plain per-box loop, equals the same box stepped alone.

The graph runs two intervals of every box per replay over three streams; the
replays are separated by eager work and synchronisations, and every replay is
checked."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_35967_amd import Engine, load  # noqa: E402
from paper_2609_35967_amd.batch import BoxBatch  # noqa: E402


def _say(*a):
    print("[gpu]", *a, flush=True)


def _boxes():
    # six local boxes of uneven size, per-box alpha and v_frag (each interval
    # has thousands of events at the workload's eps)
    return workloads.box_batch(5, nbox=6, lo=10.0, hi=12.5)


def _snap(e):
    st = e.state_numpy()
    return dict(st, nbr=e.nbr.cpu().numpy(), cnt=e.cnt.cpu().numpy(), dmax=e.dmax.cpu().numpy(),
                events=e.events.cpu().numpy(), iv=e.interval_state())


def _same(a, b, where):
    for key in ("id", "x", "y", "z", "M", "m", "nbr", "cnt", "dmax", "events"):
        assert np.array_equal(a[key], b[key]), f"{where}: {key} differs"
    for key in ("time", "ticks", "dt_exe", "n_intervals", "n_events", "C"):
        assert a["iv"][key] == b["iv"][key], f"{where}: interval {key} differs"


def _alone(boxes, rounds):
    ref = []
    for p, s, sd in boxes:
        e = Engine(p, s, seed=sd)
        snaps = []
        for _ in range(rounds):
            e.step()
            e.step()
            snaps.append(_snap(e))
        ref.append(snaps)
    return ref


def test_batch_graph_matches_alone():
    load()
    boxes = _boxes()
    _say("batch", len(boxes), "boxes", [len(s["x"]) for _, s, _ in boxes])
    ref = _alone(boxes, 3)
    assert all(r[-1]["iv"]["n_events"] > 0 for r in ref)
    _say("alone runs done")
    bb = BoxBatch(boxes, streams=3)
    bb.capture()
    _say("graph recorded")
    for r in range(3):
        bb.replay()
        torch.cuda.synchronize()
        assert float(torch.arange(1000, device="cuda", dtype=torch.float64).sum().item()) == 499500.0
        for b, e in enumerate(bb.engines):
            _same(_snap(e), ref[b][r], f"replay {r} box {b}")
            assert e.status() == 0
        _say("replay", r, "matches")


def test_batch_plain_matches_alone():
    load()
    boxes = _boxes()[:3]
    ref = _alone(boxes, 1)
    bb = BoxBatch(boxes)
    bb.step_plain()
    bb.step_plain()
    torch.cuda.synchronize()
    for b, e in enumerate(bb.engines):
        _same(_snap(e), ref[b][0], f"plain box {b}")


def test_table_sampling_matches_alone():
    # the three-call form (deferred pass per box, one table run, audits),
    # eager on one stream, equals gd_sample_collisions per box
    import ctypes as C
    from paper_2609_35967_amd.binding import check
    lib = load()
    boxes = _boxes()[:4]
    ref = _alone(boxes, 1)
    engines = [Engine(p, s, seed=sd, device_interval=True) for p, s, sd in boxes]
    sz = C.c_size_t()
    check(lib.gd_sample_table_size(len(engines), C.byref(sz)))
    table = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(2):
        for b, e in enumerate(engines):
            e.build_neighbors()
            e.collision_rates()
            e.sample_deferred(table.data_ptr(), sz.value, b)
        check(lib.gd_sample_table_run(C.c_void_p(table.data_ptr()), sz.value, len(engines), 32, 0, stream))
        for e in engines:
            e.sample_audit()
    torch.cuda.synchronize()
    for b, e in enumerate(engines):
        _same(_snap(e), ref[b][0], f"table box {b}")
        assert e.status() == 0


def test_batch_many_matches_alone():
    # one launch per stage over every box (gd_many_interval), default shapes:
    # every box equals the same box stepped alone, after every pair of intervals
    load()
    boxes = _boxes()
    ref = _alone(boxes, 3)
    bb = BoxBatch(boxes)
    for r in range(3):
        bb.step_many()
        bb.step_many()
        torch.cuda.synchronize()
        for b, e in enumerate(bb.engines):
            _same(_snap(e), ref[b][r], f"many round {r} box {b}")
            assert e.status() == 0
        _say("many round", r, "matches")


def _mixed():
    # runs of different kinds in one many-run form: dimensionless constant
    # kernel (periodic), additive column with the local push, a small disk
    # annulus with the global push (not periodic), and k = 48 and k = 96 boxes
    out = []
    p = workloads.const_box_params(3000)
    out.append((p, workloads.const_box(31, 3000), 31))
    p = workloads.additive_col_params(2500)
    out.append((p, workloads.additive_col(32, 2500), 32))
    p = workloads.disk3d_params(4000)
    out.append((p, workloads.disk3d(33, 4000, warm=True, params=p), 33))
    for k, sd in ((48, 34), (96, 35)):
        p = workloads.local_box_params(2000, alpha=3e-3, v_frag=300.0, k=k)
        out.append((p, workloads.local_box(sd, 2000, p), sd))
    return out


def test_many_mixed_runs_match_alone():
    load()
    runs = _mixed()
    ref = _alone(runs, 2)
    bb = BoxBatch(runs)
    for r in range(2):
        bb.step_many()
        bb.step_many()
        torch.cuda.synchronize()
        for b, e in enumerate(bb.engines):
            got = _snap(e)
            _same(got, ref[b][r], f"mixed round {r} run {b}")
            for key in ("r", "th", "ph", "vr", "lth", "lph", "vz"):
                if key in got:
                    assert np.array_equal(got[key], ref[b][r][key]), f"mixed round {r} run {b}: {key} differs"
            assert e.status() & ~0x4 == 0
        _say("mixed round", r, "matches")


def test_many_tuned_shapes_do_not_change_results():
    # the autotuner's trials run from a saved state; whatever it picks, the
    # next intervals equal those of the default shapes
    load()
    boxes = _boxes()[:4]
    ref = _alone(boxes, 2)
    bb = BoxBatch(boxes)
    bb.step_many()
    bb.step_many()
    torch.cuda.synchronize()
    rec = bb.tune(intervals=1, space=dict(knn_tile=(1, 0), heavy_blocks=(64, 768), event_div=(128, 4096),
                                          red_div=(256, 1 << 20)))
    assert len(rec["trials"]) >= 5 and set(rec["choice"]) >= {"knn_tile", "heavy_blocks"}
    for b, e in enumerate(bb.engines):  # tuning left the state where it was
        _same(_snap(e), ref[b][0], f"after tuning box {b}")
    bb.step_many()
    bb.step_many()
    torch.cuda.synchronize()
    for b, e in enumerate(bb.engines):
        _same(_snap(e), ref[b][1], f"tuned box {b}")
    _say("tuning", rec["choice"], rec["ms_per_interval"])


def test_many_in_stream_sets_matches_alone():
    # the boxes split into three sets, each stepped as one on its own stream
    load()
    boxes = _boxes()
    ref = _alone(boxes, 2)
    bb = BoxBatch(boxes)
    bb.many(dict(sets=3))
    for r in range(2):
        bb.step_many()
        bb.step_many()
        torch.cuda.synchronize()
        for b, e in enumerate(bb.engines):
            _same(_snap(e), ref[b][r], f"sets round {r} box {b}")
