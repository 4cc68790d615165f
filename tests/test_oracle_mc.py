"""Statistical pins of the oracle's Monte Carlo sampling (Sect. 2.5.3).

Laws checked: event counts are Poisson at a fixed rate; the partner of an
event is drawn with probability lambda*_ij/lambda*_i; fragment sizes follow
the CDF implied by eq:frag; the erosion debris share is psi lambda/lambda*_ij;
the constant kernel obeys E[m_i(t)] = m_i(0) + m0 t/t0 exactly; and the mass
distribution approaches the Smoluchowski solutions of App. A.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads
from oracle import analytic
from oracle.pipeline import OracleRun


def _box_neighbors(P, st):
    return oracle.knn(P, st["x"], st["y"], st["z"], st["M"])


def test_event_counts_are_poisson():
    # monodisperse constant kernel: lambda*_i = 1 and stays 1 after sticking
    # (the rate depends on the frozen partner masses only), so events in
    # [0, dt] are Poisson(dt).
    P = oracle.make_problem(workloads.const_box_params(4096))
    st = workloads.const_box(0, 4096)
    nbr, cnt, dmax = _box_neighbors(P, st)
    counts = []
    for iv in range(3):
        r = oracle.mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], 2.0, 7, iv)
        counts.append(r["events"])
        # every event is a sticking of an m0 grain
        assert np.array_equal(r["m"], 1.0 + r["events"])
    c = np.concatenate(counts)
    kmax = 7
    obs = np.array([np.sum(c == j) for j in range(kmax)] + [np.sum(c >= kmax)])
    p = np.array([stats.poisson.pmf(j, 2.0) for j in range(kmax)] + [stats.poisson.sf(kmax - 1, 2.0)])
    chi2 = stats.chisquare(obs, p * len(c))
    assert chi2.pvalue > 1e-4


def test_first_interval_constant_kernel():
    # m - 1 ~ Poisson(0.01) over the first interval of the constant-kernel test
    P = oracle.make_problem(workloads.const_box_params(4096))
    tot = 0
    n = 0
    for seed in range(6):
        st = workloads.const_box(seed, 4096)
        nbr, cnt, dmax = _box_neighbors(P, st)
        r = oracle.mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], 0.01, seed, 0)
        tot += int((r["m"] - 1).sum())
        n += 4096
    assert abs(tot - 0.01 * n) < 4 * math.sqrt(0.01 * n)


def test_partner_frequencies():
    # additive kernel, random masses: first-event partner ~ lambda*_ij / lambda*_i
    cfg = workloads.additive_col_params(512)
    P = oracle.make_problem(cfg)
    st = workloads.additive_col(3, 512)
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    lam, a, b, pairs = oracle.rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], True)
    obs = np.zeros_like(pairs)
    had = np.zeros(len(lam))
    reps = 60
    dt = 3.0 / lam.min()
    for iv in range(reps):
        r = oracle.mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"],
                      dt, 11, iv, log_cap=1)
        s = r["log_slot"][:, 0]
        ok = s >= 0
        had += ok
        np.add.at(obs, (np.nonzero(ok)[0], s[ok]), 1)
    # whether an event happens (U_w) is independent of its partner (U_p)
    expect = had[:, None] * pairs / lam[:, None]
    # pool cells into 32 slot columns (expected counts >= 5 each)
    o = obs.sum(0)
    e = expect.sum(0)
    assert stats.chisquare(o, e).pvalue > 1e-4
    # per-particle check pooled by expected-probability deciles
    q = np.quantile(expect.ravel(), np.linspace(0, 1, 11))
    idx = np.clip(np.searchsorted(q, expect.ravel(), side="right") - 1, 0, 9)
    o2 = np.bincount(idx, obs.ravel(), 10)
    e2 = np.bincount(idx, expect.ravel(), 10)
    assert stats.chisquare(o2, e2 * o2.sum() / e2.sum()).pvalue > 1e-4


def _disk_small(seed, n=1024, **over):
    # grain radii log-uniform over 10-100 um: rates within a few decades, so a
    # fixed interval gives every particle a handful of events
    cfg = workloads.disk3d_params(n)
    cfg.update(over)
    st = workloads.disk3d(seed, n, params=cfg)
    a = 10.0 ** np.random.default_rng(seed).uniform(-3.0, -2.0, n)
    st["m"] = math.pi * cfg["rho_s"] * (2 * a) ** 3 / 6.0
    P = oracle.make_problem(cfg)
    order = oracle.sort_perm(oracle.morton_keys(st["x"], st["y"], st["z"], st["M"]))
    st = {k: v[order] for k, v in st.items()}
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    return cfg, P, st, nbr, cnt, dmax


def test_fragment_size_distribution():
    # every collision fragments (v_frag tiny, no erosion); among particles with
    # exactly one event, s' obeys P(s' <= x) = (sqrt x - sqrt s_min)/(sqrt s_i - sqrt s_min)
    cfg, P, st, nbr, cnt, dmax = _disk_small(5, v_frag=1e-30, erosion=0)
    lam, _, _, _ = oracle.rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"])
    dt = 1.0 / np.median(lam)
    u = []
    for iv in range(8):
        r = oracle.mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], dt, 3, iv)
        one = r["events"] == 1
        s_i = (6 * st["m"][one] / (math.pi * cfg["rho_s"])) ** (1 / 3)
        s_new = (6 * r["m"][one] / (math.pi * cfg["rho_s"])) ** (1 / 3)
        a = math.sqrt(cfg["s_min"])
        u.append((np.sqrt(s_new) - a) / (np.sqrt(s_i) - a))
    u = np.concatenate(u)
    assert len(u) > 1500
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_erosion_debris_share():
    # fast collisions only; for first events on erosive pairs the debris channel
    # is taken with probability psi lambda / lambda*_ij (grouped remnant)
    cfg, P, st, nbr, cnt, dmax = _disk_small(6, v_frag=1e-30)
    lam, _, _, pairs = oracle.rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], True)
    dt = 3.0 / np.median(lam)
    hits, expect, var = 0, 0.0, 0.0
    for iv in range(100):
        r = oracle.mc(P, st["id"], nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], dt, 4, iv,
                      log_cap=1)
        sel = r["log_type"][:, 0] == 1
        i = np.nonzero(sel)[0]
        s = r["log_slot"][i, 0]
        psi = st["m"][nbr[i, s]] / st["m"][i]
        Ng = np.where(psi <= 1e-6, np.floor(1e-4 / psi), 1.0)
        p_deb = psi / ((1 - psi) / Ng + psi)
        hits += int((r["log_chan"][i, 0] == 1).sum())
        expect += p_deb.sum()
        var += (p_deb * (1 - p_deb)).sum()
    assert var > 5
    assert abs(hits - expect) < 4.5 * math.sqrt(var)


def test_constant_kernel_expectation_law_and_w1():
    # E[m_i(t)] = 1 + t exactly for the constant kernel (Sect. 3.3 normalisation);
    # the mass distribution approaches eq:sol_const.
    cfg = workloads.const_box_params(4096)
    means, w1s = [], []
    for seed in range(2):
        run = OracleRun(cfg, workloads.const_box(seed, 4096), seed=seed)
        while run.time < cfg["t_end"] - 1e-9:
            run.step(rebuild=False)
        m = run.st["m"]
        assert run.interval == 1000 and run.time == pytest.approx(10.0, abs=1e-12)
        means.append(m.mean())
        j, f = analytic.const_mass_fractions(run.time)
        w1s.append(analytic.w1_discrete(m, run.st["M"], j, f))
        se = m.std() / math.sqrt(len(m))
        assert abs(m.mean() - 11.0) < 5 * se
        # mass conservation: sum N_i m_i = sum M_i
        N = run.st["M"] / m
        assert abs((N * m).sum() - run.st["M"].sum()) < 1e-13
    assert max(w1s) < 0.03


def test_additive_kernel_mean_mass():
    # mass-weighted mean of the additive kernel grows as 2 exp(2 t); the frozen
    # neighbourhood lags it by O(eps) per unit of growth
    cfg = workloads.additive_col_params(4096)
    cfg["push"] = "none"
    run = OracleRun(cfg, workloads.additive_col(1, 4096), seed=1)
    while run.time < 0.5:
        run.step(rebuild=False)
    m = run.st["m"]
    want = analytic.linear_mass_weighted_mean(run.time)
    assert abs(m.mean() / want - 1) < 0.05
    assert analytic.w1_linear(m, run.st["M"], run.time) < 0.08
