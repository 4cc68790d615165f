"""Pins of the oracle's rates, outcome channels, moments and interval plan.

References: numerical quadrature (scipy) for the fragment moments; the
dimensionless kernels' closed sums; a Monte-Carlo volume estimate for the
boundary caps; hand-worked controller cases.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads


# ------------------------------------------------------- fragment moments ----
@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("x", [1.0 + 1e-6, 1.001, 1.05, 1.0999, 1.1001, 1.5, 3.0, 30.0, 1e4])
def test_fragment_moments_vs_quadrature(x):
    s_min = 2e-4
    s_i = s_min * x * x
    mJ, mJ2 = oracle.frag_moments(s_i, s_min)
    a, b = math.sqrt(s_min), math.sqrt(s_i)

    def J(U):
        w = a + U * (b - a)
        return abs(math.log(w * w / s_i))

    q1 = integrate.quad(J, 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
    q2 = integrate.quad(lambda U: J(U) ** 2, 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs(mJ - q1) <= 1e-11 * q1
    assert abs(mJ2 - q2) <= 1e-10 * q2


def test_fragment_moments_degenerate():
    assert oracle.frag_moments(2e-4, 2e-4) == (0.0, 0.0)
    d = 1e-7
    mJ, mJ2 = oracle.frag_moments(2e-4 * (1 + d) ** 2, 2e-4)
    assert abs(mJ - d) < 1e-13 and abs(mJ2 - 4 * d * d / 3) < 1e-20


# -------------------------------------------------- dimensionless kernels ----
def _mono_problem(kernel, k=32, **kw):
    return oracle.make_problem(dict(kernel=kernel, k=k, t0=1.0, m0=1.0, periodic=(1, 1, 1),
                                    L=(1.0, 1.0, 1.0), **kw))


def test_constant_kernel_monodisperse_rate_is_one():
    st = workloads.const_box(0, 1024)
    P = _mono_problem("const")
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    lam, a, b, pairs = oracle.rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], True)
    # lambda_i = k * (1/t0)(1/k)(m0/m0) = 1/t0 exactly (Sect. 3.3)
    assert (lam == 1.0).all()
    # every event doubles the grain: J = ln 2 / 3 for every pair
    np.testing.assert_allclose(a, math.log(2) / 3, rtol=1e-15)
    np.testing.assert_allclose(b, (math.log(2) / 3) ** 2, rtol=1e-15)


@pytest.mark.parametrize("kernel", ["additive", "product"])
def test_dimensionless_kernel_sums(kernel):
    st = workloads.additive_col(2, 2000)
    P = oracle.make_problem(dict(kernel=kernel, k=32, t0=2.0, m0=1.5, periodic=(1, 1, 0), L=(1, 1, 1)))
    nbr, cnt, dmax = oracle.knn(P, st["x"], st["y"], st["z"], st["M"])
    lam, a, b, pairs = oracle.rates(P, nbr, cnt, dmax, st["m"], st["M"], st["x"], st["y"], st["z"], True)
    m = st["m"]
    mi = m[:, None]
    mj = m[nbr]
    # lambda_ij = (1/t0)(1/N_K)(m0/m_j) K, K = (mi+mj)/m0 or mi mj/m0^2: sums in closed form
    if kernel == "additive":
        expect = (mi / mj + 1.0).sum(1) / (2.0 * 32)
    else:
        expect = mi[:, 0] * 32 / (1.5 * 2.0 * 32)
    np.testing.assert_allclose(lam, expect, rtol=1e-13)
    # moments: sticking only, J = ln(1 + psi)/3
    J = np.log1p(mj / mi) / 3.0
    np.testing.assert_allclose(a, (pairs * J).sum(1), rtol=1e-13)


def test_no_other_neighbour_means_no_rate():
    P = _mono_problem("const")
    nbr = np.full((2, 32), -1, np.int32)
    nbr[:, 0] = [0, 1]
    cnt = np.array([1, 1], np.int32)
    lam, a, b, _ = oracle.rates(P, nbr, cnt, np.zeros(2), np.ones(2), np.ones(2), np.zeros(2), np.zeros(2),
                                np.zeros(2))
    assert (lam == 0).all() and (a == 0).all() and (b == 0).all()


# -------------------------------------------------------------- channels ----
def _disk_problem(**over):
    p = workloads.disk3d_params(4096)
    p.update(over)
    return p, oracle.make_problem(p)


def test_grouping_factor_and_sticking_rate():
    # psi <= 1e-6 groups floor(1e-4/psi) sticking events into one (Sect. 2.5.2)
    p, P = _disk_problem(v_frag=1e30)
    R = 20 * workloads.AU
    base = oracle.pair_rate(P, R, 0.0, 0.0, 0.3 * workloads.AU, 1.0, 1.0, 1.0)
    for psi, Ng in [(1e-5, 1.0), (1e-6, 100.0), (3e-7, 333.0), (1e-9, 1e5)]:
        r = oracle.pair_rate(P, R, 0.0, 0.0, 0.3 * workloads.AU, 1.0, psi, 1.0)
        assert r["Ng"] == Ng and r["type"] == 0
        assert base["V"] == r["V"]


def test_erosion_and_fragmentation_channels():
    p, P = _disk_problem(v_frag=1e-30)  # every collision is fast
    R = 20 * workloads.AU
    di = 0.3 * workloads.AU
    mi = 1e-6
    for psi in (0.05, 0.1):
        r = oracle.pair_rate(P, R, 0.0, 0.0, di, mi, psi * mi, 1.0)
        assert r["type"] == 1
        lam = r["rate0"] + r["rate1"]
        # remnant (1-psi) lambda, debris psi lambda (Ng = 1): debris share is psi
        assert abs(r["rate1"] / lam - psi) < 1e-14
        assert r["lam_star"] == lam
    r = oracle.pair_rate(P, R, 0.0, 0.0, di, mi, 0.2 * mi, 1.0)
    assert r["type"] == 2 and r["rate1"] == 0.0
    p2, P2 = _disk_problem(v_frag=1e-30, erosion=0)
    r = oracle.pair_rate(P2, R, 0.0, 0.0, di, mi, 0.05 * mi, 1.0)
    assert r["type"] == 2


# --------------------------------------------------------- physical rate ----
def test_physical_rate_limits():
    p, P = _disk_problem()
    R = 30 * workloads.AU
    di = 0.5 * workloads.AU
    m = 1e-9
    # equal grains at the midplane: drift terms vanish; tight-coupling turbulence
    # vanishes for equal St; only Brownian motion is left
    g = oracle.gas_at(P, R, 0.0)
    r = oracle.pair_rate(P, R, 0.0, 0.0, di, m, m, 1.0)
    s = (6 * m / (math.pi * p["rho_s"])) ** (1 / 3)
    vB = math.sqrt(8 * p["mu_mH"] * g["cs"] ** 2 / math.pi * 2 / m)
    V = 4 * math.pi * di ** 3 / 3
    lam = (1.0 / m) * math.pi * (2 * s) ** 2 * vB / 4 / V
    assert abs(r["lam_star"] - lam) < 1e-12 * lam
    # Brownian speed is capped at the sound speed for tiny grains
    tiny = 1e-40
    r2 = oracle.pair_rate(P, R, 0.0, 0.0, di, tiny, tiny, 1.0)
    s2 = (6 * tiny / (math.pi * p["rho_s"])) ** (1 / 3)
    lam2 = (1.0 / tiny) * math.pi * (2 * s2) ** 2 * g["cs"] / 4 / V
    assert abs(r2["lam_star"] - lam2) < 1e-12 * lam2
    # the rate is symmetric in the roles of the two grains up to N_j (equal M here)
    a = oracle.pair_rate(P, R, 0.0, 0.0, di, 1e-9, 3e-7, 1.0)
    b = oracle.pair_rate(P, R, 0.0, 0.0, di, 3e-7, 1e-9, 1.0)
    # lambda_ij = N_j K/V: K symmetric, so lambda_ij m_j = lambda_ji m_i when types agree
    Ka = a["lam_star"] * 3e-7
    Kb = b["lam_star"] * 1e-9
    if a["type"] == b["type"] == 0:
        assert abs(Ka - Kb) < 1e-12 * Ka


@pytest.mark.parametrize("St_i,St_j", [(0.02, 0.005), (2.0, 0.3), (0.4, 0.9), (0.1, 0.1)])
def test_physical_rate_drift_terms(St_i, St_j):
    # Brownian and turbulent terms off: the collision speed is the three
    # prescribed relative motions of eq:dv (Sect. 2.5.2), written out here term
    # by term, and the rate is eq:rate with eq:kernel and an uncapped sphere
    p, P = _disk_problem(brownian=0, turbulence=0, v_frag=1e30)
    au = workloads.AU
    R, Z, di = 30 * au, 0.6 * au, 0.05 * au
    g = oracle.gas_at(P, R, Z)
    rho = p["rho_s"]
    s_i, s_j = St_i / g["stfac"], St_j / g["stfac"]
    m_i, m_j = math.pi * rho * s_i ** 3 / 6, math.pi * rho * s_j ** 3 / 6
    M_j = 7.0 * m_j
    r = oracle.pair_rate(P, R, 0.0, Z, di, m_i, m_j, M_j)
    # the grain sizes the oracle derives from the masses (Stokes numbers follow)
    s_i = (6 * m_i / (math.pi * rho)) ** (1 / 3)
    s_j = (6 * m_j / (math.pi * rho)) ** (1 / 3)
    St_i, St_j = g["stfac"] * s_i, g["stfac"] * s_j
    vK = R * g["OmK"]
    dvR = 2 * g["eta"] * vK * (St_i / (1 + St_i ** 2) - St_j / (1 + St_j ** 2))
    dvZ = Z * g["OmK"] * (min(St_i, 0.5) - min(St_j, 0.5))
    dvP = g["eta"] * vK * (1 / (1 + St_i ** 2) - 1 / (1 + St_j ** 2))
    dv = math.sqrt(dvR ** 2 + dvZ ** 2 + dvP ** 2)
    K = math.pi * (s_i + s_j) ** 2 * dv / 4
    lam = (M_j / m_j) * K / (4 * math.pi * di ** 3 / 3)
    assert r["type"] == 0 and r["Ng"] == 1.0
    assert abs(r["V"] - 4 * math.pi * di ** 3 / 3) <= 1e-14 * r["V"]
    if St_i == St_j:
        assert r["lam_star"] <= 1e-13 * (M_j / m_j) * math.pi * (2 * s_i) ** 2 * vK / r["V"]
    else:
        assert abs(r["lam_star"] - lam) <= 1e-11 * lam


def test_oc07_regimes():
    Vg2 = 2.0
    tke = 1e-3
    # identical grains: no turbulent relative speed in the tightly coupled regime
    assert oracle.oc07(1e-4, 1e-4, Vg2, tke) == 0.0
    # heavy regime: V_g^2 (1/(1+St1) + 1/(1+St2)) -> 0 for very heavy grains
    assert oracle.oc07(1e8, 1e8, Vg2, tke) < 1e-7
    # intermediate regime at eps = 1: 2 y_a - 2 + 2/2 (2/(1+y_a)) with y_a = 1.6
    br = 2 * 1.6 - 2 + (1 / 2.6 + 1 / 2.6)
    assert abs(oracle.oc07(0.1, 0.1, Vg2, tke) - Vg2 * br * 0.1) < 1e-15
    # monotone in the larger Stokes number inside the intermediate regime
    v = [oracle.oc07(s, 1e-5, Vg2, 1e-6) for s in np.geomspace(1e-5, 0.9, 40)]
    assert np.all(np.diff(v) > 0)


def test_boundary_caps_against_monte_carlo_volume():
    p, P = _disk_problem()
    rng = np.random.default_rng(3)
    au = workloads.AU
    for r_q, di in [(10.3 * au, 0.6 * au), (99.5 * au, 1.2 * au), (50 * au, 1.0 * au)]:
        r = oracle.pair_rate(P, r_q, 0.0, 0.0, di, 1e-9, 1e-9, 1.0)
        # volume of the ball that lies between the two boundary planes at r_in, r_out
        u = rng.uniform(-1, 1, (400000, 3)) * di
        inside = (u * u).sum(1) <= di * di
        xr = r_q + u[:, 0]
        ok = inside & (xr >= p["r_in"]) & (xr <= p["r_out"])
        est = ok.mean() * (2 * di) ** 3
        se = math.sqrt(ok.mean() * (1 - ok.mean()) / len(ok)) * (2 * di) ** 3
        assert abs(r["V"] - est) < 5 * se + 1e-12 * est


# ------------------------------------------------------------------ plan ----
def test_merge_rule_and_dyadic_plan():
    P = oracle.make_problem(dict(kernel="const", k=32, nbin_min=64, eps=0.08, dt_fn_max=1.0))
    counts = [10, 50, 5, 100, 3]
    m = np.concatenate([np.full(c, 2.0 ** b) for b, c in enumerate(counts)])
    M = np.ones_like(m)
    a = np.ones_like(m)
    b = np.zeros_like(m)
    pl = oracle.plan(P, m, M, a, b, 1.0, 0, 1.0)
    g = pl["group_of"]
    assert [g[oracle.bin_of(2.0 ** i)] for i in range(5)] == [0, 0, 0, 1, 1]
    # A = 1 in every group -> dt_req = eps C / A = 0.08 -> largest 2^-n <= 0.08 is 1/16
    assert pl["dt_req"] == 0.08
    assert pl["dt_exe"] == 0.0625 and pl["exe_ticks"] == 1 << 26
    # second moment binds when larger: B = 1 -> (eps C)^2 = 0.0064 -> 2^-8
    pl = oracle.plan(P, m, M, np.zeros_like(m), np.ones_like(m), 1.0, 0, 1.0)
    assert pl["dt_req"] == pytest.approx(0.0064, rel=1e-15) and pl["dt_exe"] == 2.0 ** -8
    # alignment: 3/16 of the step elapsed -> only sizes dividing 3 * 2^26 ticks
    pl = oracle.plan(P, m, M, np.zeros_like(m), np.zeros_like(m), 1.0, 3 << 26, 1.0)
    assert pl["dt_req"] == 13 / 16 and pl["dt_exe"] == 1 / 16
    # a smaller C shrinks the request in proportion
    pl = oracle.plan(P, m, M, a, b, 1.0, 0, 0.5)
    assert pl["dt_req"] == 0.04 and pl["dt_exe"] == 1 / 32


def test_plan_invariants_random():
    rng = np.random.default_rng(9)
    P = oracle.make_problem(dict(kernel="const", k=32, eps=0.08, dt_fn_max=0.3))
    for trial in range(50):
        n = 500
        m = 10 ** rng.uniform(-3, 3, n)
        a = 10 ** rng.uniform(-2, 2, n)
        b = 10 ** rng.uniform(-2, 2, n)
        ticks = int(rng.integers(0, 1 << 30)) & ~((1 << 20) - 1)
        pl = oracle.plan(P, m, np.ones(n), a, b, 1.0, ticks, rng.uniform(0.25, 1))
        assert pl["dt_exe"] <= pl["dt_req"] or pl["exe_ticks"] == 1
        assert ticks % pl["exe_ticks"] == 0
        assert pl["exe_ticks"] & (pl["exe_ticks"] - 1) == 0
        assert pl["dt_exe"] == pl["exe_ticks"] * 2.0 ** -30


def test_audit_rule():
    P = oracle.make_problem(dict(kernel="const", k=32, eps=0.08))
    m0 = np.ones(200)
    M = np.ones(200)
    g = np.zeros(128, np.int32) - 1
    g[oracle.bin_of(1.0)] = 0
    gM = np.zeros(128)
    gM[0] = 200.0
    # realised mean |ln(s'/s)| = ln(2)/3 * fraction doubled
    m1 = m0.copy()
    m1[:10] = 2.0
    au = oracle.audit(P, m0, m1, M, g, gM, 1.0)
    assert au["worst"] == pytest.approx(10 / 200 * math.log(2) / 3, rel=1e-14)
    assert au["C"] == 1.0  # 0.0116 < 2 eps C = 0.16: grows, capped at 1
    m1[:150] = 2.0
    au = oracle.audit(P, m0, m1, M, g, gM, 1.0)
    assert au["C"] == 0.5  # 0.173 > 0.16: halves
    au = oracle.audit(P, m0, m1, M, g, gM, 0.3)
    assert au["C"] == 0.25  # floor


def test_fsum_exact():
    rng = np.random.default_rng(4)
    import math as _m
    for _ in range(20):
        v = rng.standard_normal(1000) * 10.0 ** rng.integers(-30, 30, 1000)
        assert oracle.fsum(v) == _m.fsum(v)


@pytest.mark.parametrize("R_au,zr,ai,aj", [(17.43, 0.08536, 9.299e-05, 9.126e-05),
                                           (76.01, 0.04763, 6.768e-05, 6.548e-05),
                                           (26.99, 0.04518, 1.816e-04, 1.822e-04),
                                           (70.74, -0.03901, 6.12e-05, 6.527e-05)])
def test_dv_five_terms_compose_in_quadrature(R_au, zr, ai, aj):
    """eq:dv adds the Brownian, radial, vertical, azimuthal and turbulent speeds
    in quadrature, and the kernel (hence the pair rate with sticking only and no
    grouping) is linear in dv, so lambda^2 with every term equals lambda^2 with
    Brownian only plus lambda^2 with turbulence only minus lambda^2 with the
    drift terms alone -- at points where each part is 15% or more of the total."""
    import math

    base = dict(workloads.disk3d_params(1000), v_frag=math.inf, grouping=0, erosion=0)
    R = R_au * workloads.AU
    x, y, z = R * math.cos(0.3), R * math.sin(0.3), zr * R
    mi = math.pi * 1.6 * (2 * ai) ** 3 / 6
    mj = math.pi * 1.6 * (2 * aj) ** 3 / 6
    lam = {}
    for b in (0, 1):
        for t in (0, 1):
            P = oracle.make_problem(dict(base, brownian=b, turbulence=t))
            lam[(b, t)] = oracle.pair_rate(P, x, y, z, 1e-3 * R, mi, mj, 1e20)["lam_star"]
    d2 = lam[(0, 0)] ** 2
    B, T = lam[(1, 0)] ** 2 - d2, lam[(0, 1)] ** 2 - d2
    tot = d2 + B + T
    assert min(d2, B, T) > 0.15 * tot
    np.testing.assert_allclose(lam[(1, 1)] ** 2, tot, rtol=1e-12)
