"""Write the oracle's reference runs used by tests/test_gpu_configs.py.

  const_box_runs.json   the constant-kernel test of App. A on the 4096-particle
                        periodic box: 10 seeds, neighbour lists built once
                        (positions are static), 1000 collision steps of 0.01
                        to t = 10.  Per seed: intervals run, C, mean mass,
                        W1 against eq:sol_const at t = 10, near-tie count and a
                        digest of the final masses in id order.
  additive_col_run.json the additive-kernel column with local settling:
                        65,536 particles, seed 0, 100 intervals of the headline
                        loop.  Per interval: dt_exe, C, events; at the end a
                        digest of the masses, the mean mass, W1 against
                        eq:sol_linear at the reached time, and z, v_z of 64
                        sampled particles.

Calls only oracle/ and workloads/.  Run from the repository root:
    python tests/golden/make_run_goldens.py [const|additive]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import analytic  # noqa: E402
from oracle.pipeline import OracleRun  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def mass_digest(st):
    o = np.argsort(st["id"].astype(np.int64))
    return hashlib.sha256(np.ascontiguousarray(st["m"][o], np.float64).tobytes()).hexdigest()


def const_runs():
    out = []
    for seed in range(10):
        params, st = workloads.by_name("const_box", seed=seed)
        run = OracleRun(params, st, seed=seed)
        run.build_neighbors()
        steps = ties = 0
        t0 = time.time()
        while steps < 1000:
            r = run.step(rebuild=False, push=False)
            ties += int(r["mc"]["near_tie"].sum())
            if run.ticks == 0:
                steps += 1
        m, M = run.st["m"], run.st["M"]
        j, f = analytic.const_mass_fractions(10.0)
        w1 = analytic.w1_discrete(m, M, j, f)
        out.append(dict(seed=seed, n_intervals=run.interval, C=run.C, mean_m=float(np.mean(m)), w1=w1,
                        near_ties=ties, digest=mass_digest(run.st)))
        print(f"const seed {seed}: {run.interval} intervals, mean m {np.mean(m):.4f}, W1 {w1:.4f}, "
              f"ties {ties}, {time.time() - t0:.1f} s", flush=True)
    doc = dict(workload="const_box: 4096 particles, k = 32, t0 = m0 = 1, dt_coll = dt_fn_max = 0.01, eps = 0.08, "
                        "neighbour lists built once, run to t = 10 (1000 collision steps)",
               source="oracle.pipeline.OracleRun via tests/golden/make_run_goldens.py", runs=out)
    with open(os.path.join(HERE, "const_box_runs.json"), "w") as f:
        json.dump(doc, f, indent=1)


def additive_run():
    params, st = workloads.by_name("additive_col", seed=0)
    run = OracleRun(params, st, seed=0)
    per, ties = [], 0
    t0 = time.time()
    for it in range(100):
        r = run.step(push=True)
        ties += int(r["mc"]["near_tie"].sum())
        per.append(dict(dt_exe=r["plan"]["dt_exe"], C=run.C, events=int(r["mc"]["events"].sum())))
        if it % 10 == 9:
            print(f"additive interval {it + 1}: t = {run.time:.5f}, {time.time() - t0:.0f} s", flush=True)
    m, M = run.st["m"], run.st["M"]
    o = np.argsort(run.st["id"].astype(np.int64))
    ids = np.random.default_rng(0).choice(len(m), 64, replace=False)
    doc = dict(workload="additive_col: 65,536 particles, k = 32, seed 0, 100 intervals of kNN + rates + sampling "
                        "+ local settling push",
               source="oracle.pipeline.OracleRun via tests/golden/make_run_goldens.py",
               intervals=per, near_ties=ties, time=run.time, C=run.C, ticks=run.ticks, digest=mass_digest(run.st),
               mean_m=float(np.mean(m)), w1=analytic.w1_linear(m, M, run.time),
               sample_ids=[int(i) for i in ids],
               sample_z=[float(v) for v in run.st["z"][o][ids]], sample_vz=[float(v) for v in run.st["vz"][o][ids]])
    with open(os.path.join(HERE, "additive_col_run.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["const", "additive"]
    if "const" in which:
        const_runs()
    if "additive" in which:
        additive_run()
