"""The operator sequence of a transport step on the oracle (Sect. 2.6), host
logic only: with nothing moving the particles, C(dt/2) ... C(dt/2) is the
plain sequence of intervals over the same collision steps on one neighbour
list, and the lists are rebuilt only after positions changed."""
import numpy as np

import workloads
from oracle.pipeline import OracleRun


def test_static_strang_steps_equal_plain_intervals():
    params = workloads.const_box_params(2048)
    st = workloads.const_box(1, 2048)
    a = OracleRun(params, st, seed=4)
    b = OracleRun(params, st, seed=4)
    b.build_neighbors()
    n = 0
    for _ in range(2):
        n += len(a.strang_step())
    done = 0
    while done < 4:                      # four collision steps of dt_coll
        b.step(rebuild=False)
        if b.ticks == 0:
            done += 1
    assert a.interval == b.interval == n
    assert np.array_equal(a.st["m"], b.st["m"]) and a.C == b.C
    assert a.diff_step == 0 and not a.moved


def test_rebuild_only_after_motion():
    # slow constant kernel (t0 >> dt_coll): one interval per collision step
    params = dict(workloads.diffusion_ring_params("density", n=512), kernel="const", t0=1e6, m0=1.0, eps=0.08,
                  dt_fn_max=10.0)
    st = workloads.diffusion_ring(2, 512)
    run = OracleRun(params, st, seed=1)
    calls = []
    orig = run.build_neighbors

    def counting():
        calls.append(run.interval)
        return orig()

    run.build_neighbors = counting
    run.strang_step()
    run.strang_step()
    # one build for the first C, one after D T D, one more after the second D T D;
    # the first C of step 2 reuses the lists of the last C of step 1
    assert len(calls) == 3
    assert run.diff_step == 4
