"""The oracle's physical pair rate against an independent 50-digit evaluation.

The oracle evaluates eq:dv in rearranged forms that keep their accuracy for
nearly equal grains (St_i - St_j from the mass difference, the tightly coupled
Ormel & Cuzzi (2007) branch without its cancellation).  The evaluation below
takes none of them: it follows the printed passages term by term in mpmath at
50 digits, from the FP64 inputs taken exactly:

  gas disk at the query position        Sect. 2.2 (Sigma_g, h_g, H_g, c_s,
                                         Omega_K, rho_g, eta)
  Stokes number of each grain           Sect. 2.3.1 (analytic gas), computed
                                         for s_i and s_j separately
  relative speed                        eq:dv: Delta v_R, Delta v_Z, Delta v_phi
                                         as printed, Brownian capped at c_s,
                                         turbulence by the Ormel & Cuzzi closed
                                         forms (tightly coupled, intermediate
                                         with y_a = 1.6, heavy)
  kernel, rate                          eq:kernel, eq:rate, V_i = 4 pi d_i^3/3
                                         less the flat caps of nearby boundaries
  channels                              Sect. 2.5.2 (sticking with grouping,
                                         erosion remnant and debris,
                                         fragmentation)

Every pair below sits away from the branch thresholds, so the value is well
conditioned and the oracle must agree to 1e-13 relative.  Pairs are chosen
in each turbulence regime with distant, close and equal Stokes numbers, and
in the regime where St2 < Re^-1/2 <= St1.  Planted mistakes in each branch
and each term of the oracle must fail the comparison.
"""
from __future__ import annotations

import math

import mpmath as mp
import pytest

import oracle
import workloads

mp.mp.dps = 50
AU = workloads.AU
TOL = 1e-13


def _m(v):
    return mp.mpf(float(v))


def mp_gas(p, R, Z):
    """The analytic gas disk of Sect. 2.2 at cylindrical (R, Z)."""
    R, Z = _m(R), _m(Z)
    r = mp.sqrt(R * R + Z * Z)
    xr = R / _m(p["R0"])
    OmK = mp.sqrt(_m(p["GM"]) / R ** 3)
    hg = _m(p["h_g0"]) * xr ** ((_m(p["q"]) + 1) / 2)
    Hg = hg * R
    cs = Hg * OmK
    Sig = _m(p["Sigma_g0"]) * xr ** _m(p["p"])
    w = 1 - R / r
    rhog = Sig / (mp.sqrt(2 * mp.pi) * Hg) * mp.exp(-w / hg ** 2)
    eta = -(((_m(p["p"]) + _m(p["q"]) / 2 - mp.mpf(3) / 2) * hg ** 2 + _m(p["q"]) * w)) / 2
    return dict(R=R, Z=Z, r=r, xr=xr, OmK=OmK, hg=hg, Hg=Hg, cs=cs, rhog=rhog, eta=eta, w=w)


def mp_stokes(p, g, s):
    """St(R, Z, s) = St0 (s/s0) (R/R0)^-p exp((1 - R/r)/h_g^2)."""
    return _m(p["St0"]) * (s / _m(p["s0"])) * g["xr"] ** (-_m(p["p"])) * mp.exp(g["w"] / g["hg"] ** 2)


def mp_oc07(St1, St2, Vg2, t_eta):
    """Ormel & Cuzzi (2007) closed forms, St1 >= St2, as printed."""
    if St1 < t_eta:
        return Vg2 * (St1 - St2) / (St1 + St2) * (St1 ** 2 / (St1 + t_eta) - St2 ** 2 / (St2 + t_eta)), "tight"
    if St1 < 1:
        ya = mp.mpf("1.6")
        e = St2 / St1
        br = 2 * ya - (1 + e) + 2 / (1 + e) * (1 / (1 + ya) + e ** 3 / (ya + e))
        return Vg2 * br * St1, "intermediate"
    return Vg2 * (1 / (1 + St1) + 1 / (1 + St2)), "heavy"


def mp_pair(p, x, y, z, di, mi, mj, Mj):
    """Channel rates of one pair (eq:rate with eq:kernel and eq:dv)."""
    x, y, z, di, mi, mj, Mj = (_m(v) for v in (x, y, z, di, mi, mj, Mj))
    R = mp.sqrt(x * x + y * y)
    g = mp_gas(p, R, z)
    rho = _m(p["rho_s"])
    si = mp.cbrt(6 * mi / (mp.pi * rho))
    sj = mp.cbrt(6 * mj / (mp.pi * rho))
    Sti, Stj = mp_stokes(p, g, si), mp_stokes(p, g, sj)
    vK = R * g["OmK"]
    dvR = 2 * g["eta"] * vK * (Sti / (1 + Sti ** 2) - Stj / (1 + Stj ** 2))
    dvZ = z * g["OmK"] * (min(Sti, mp.mpf("0.5")) - min(Stj, mp.mpf("0.5")))
    dvP = g["eta"] * vK * (1 / (1 + Sti ** 2) - 1 / (1 + Stj ** 2))
    dv2 = dvR ** 2 + dvZ ** 2 + dvP ** 2
    kT = _m(p["mu_mH"]) * g["cs"] ** 2  # k_B T of the isothermal gas
    if p.get("brownian", 1):
        dvB = min(g["cs"], mp.sqrt(8 * kT / mp.pi * (1 / mi + 1 / mj)))
        dv2 += dvB ** 2
    regime = None
    St1, St2 = max(Sti, Stj), min(Sti, Stj)
    vth = mp.sqrt(8 / mp.pi) * g["cs"]
    lmfp = _m(p["mu_mH"]) / (g["rhog"] * _m(p["sigma_H2"]))
    nu_mol = vth * lmfp / 2
    Re = _m(p["alpha"]) * g["cs"] * g["Hg"] / nu_mol
    t_eta = 1 / mp.sqrt(Re)
    if p.get("turbulence", 1):
        dvt2, regime = mp_oc07(St1, St2, mp.mpf(3) / 2 * _m(p["alpha"]) * g["cs"] ** 2, t_eta)
        dv2 += dvt2
    dv = mp.sqrt(dv2)
    V = 4 * mp.pi * di ** 3 / 3
    if p.get("caps", 1):
        for delta in (g["r"] - _m(p["r_in"]), _m(p["r_out"]) - g["r"]):
            if delta < di:
                h = di - delta
                V -= mp.pi * h ** 2 * (3 * di - h) / 3
    K = mp.pi * (si + sj) ** 2 * dv / 4
    lam = (Mj / mj) * K / V
    psi = mj / mi
    Ng = mp.floor(mpf_1e4() / psi) if psi <= mp.mpf(1e-6) else mp.mpf(1)
    if dv < _m(p["v_frag"]):
        rates, kind = [lam / Ng], 0
    elif psi <= mp.mpf(0.1):
        rates, kind = [(1 - psi) * lam / Ng, psi * lam], 1
    else:
        rates, kind = [lam], 2
    return dict(rates=rates, type=kind, Ng=Ng, V=V, St1=St1, St2=St2, t_eta=t_eta, regime=regime, dv=dv)


def mpf_1e4():
    # 1e-4 as the FP64 constant the grouping rule compares against
    return mp.mpf(1e-4)


def _params(**kw):
    p = dict(workloads.disk3d_params(1000), **kw)
    return p, oracle.make_problem(p)


def _mass_for_stokes(p, R, Z, St):
    """FP64 grain mass whose Stokes number at (R, Z) is close to St."""
    g = mp_gas(p, R, Z)
    unit = mp_stokes(p, g, mp.mpf(1))  # St per unit diameter
    s = mp.mpf(St) / unit
    return float(mp.pi * _m(p["rho_s"]) * s ** 3 / 6), g


def _t_eta(p, R, Z):
    return float(mp_pair(p, R, 0.0, Z, 0.1 * AU, 1e-9, 1e-9, 1.0)["t_eta"])


def _compare(p, P, x, y, z, di, mi, mj, Mj, regime=None):
    ref = mp_pair(p, x, y, z, di, mi, mj, Mj)
    if regime is not None:
        assert ref["regime"] == regime
    # away from every threshold the value is well conditioned
    for thr in (ref["t_eta"], mp.mpf(1)):
        assert abs(ref["St1"] / thr - 1) > 1e-9
    assert abs(ref["dv"] / _m(p["v_frag"]) - 1) > 1e-9
    got = oracle.pair_rate(P, x, y, z, di, mi, mj, Mj)
    assert got["type"] == ref["type"]
    assert got["Ng"] == float(ref["Ng"])
    errs = [abs(_m(got["V"]) / ref["V"] - 1)]
    got_rates = [got["rate0"], got["rate1"]][:len(ref["rates"])]
    for g_, r_ in zip(got_rates, ref["rates"]):
        errs.append(abs(_m(g_) / r_ - 1) if r_ != 0 else abs(_m(g_)))
    return float(max(errs)), ref


# Query positions (R, Z in au; d_i in au): midplane-near, high, and within a
# neighbourhood radius of each boundary sphere (caps).
SITES = [(30.0, 0.6, 0.05), (55.0, 2.5, 0.3), (10.25, -0.08, 0.4), (99.6, 0.3, 0.7)]


def _pairs(p, R, Z):
    """(label, St1, St2) covering each turbulence regime with distant, close and
    equal Stokes numbers, and St2 < t_eta <= St1."""
    te = _t_eta(p, R, Z)
    return [
        ("tight, distant", 0.3 * te, 0.02 * te),
        ("tight, close", 0.3 * te, 0.3 * te * (1 - 1e-3)),
        ("tight, very close", 0.5 * te, 0.5 * te * (1 - 1e-7)),
        ("tight, equal", 0.4 * te, 0.4 * te),
        ("intermediate, St2 below t_eta", 30 * te, 0.5 * te),
        ("intermediate, just above t_eta", 1.5 * te, 0.3 * te),
        ("intermediate, near the heavy regime", 0.8, 0.1),
        ("intermediate, distant", 0.4, 1e-3),
        ("intermediate, close", 0.2, 0.2 * (1 - 1e-4)),
        ("intermediate, equal", 0.05, 0.05),
        ("heavy, distant", 3.0, 0.01),
        ("heavy, close", 2.0, 2.0 * (1 - 1e-5)),
        ("heavy, equal", 40.0, 40.0),
    ]


def _all_cases(p):
    cases = []
    for R_au, Z_au, d_au in SITES:
        R, Z, di = R_au * AU, Z_au * AU, d_au * AU
        x, y = R * math.cos(0.7), R * math.sin(0.7)
        for label, St1, St2 in _pairs(p, R, Z):
            mi, _ = _mass_for_stokes(p, R, Z, St1)
            mj, _ = _mass_for_stokes(p, R, Z, St2)
            regime = label.split(",")[0]
            # both roles: the query grain the larger and the smaller one
            cases.append((f"{label} @ {R_au} au", x, y, Z, di, mi, mj, 3.0e4 * mj, regime))
            cases.append((f"{label} (swapped) @ {R_au} au", x, y, Z, di, mj, mi, 7.0e2 * mi, regime))
    return cases


def test_pair_rate_matches_50_digit_evaluation_in_every_regime():
    p, P = _params(v_frag=math.inf)  # sticking only: lambda*_ij = lambda_ij (no grouping at these psi)
    worst = 0.0
    for label, x, y, z, di, mi, mj, Mj, regime in _all_cases(p):
        if mj / mi <= 1e-6:
            continue  # grouped pairs are checked below
        err, _ = _compare(p, P, x, y, z, di, mi, mj, Mj, regime)
        assert err <= TOL, (label, err)
        worst = max(worst, err)
    assert worst > 0.0  # the two evaluations are not the same arithmetic


def test_brownian_cap_and_channels_against_50_digit_evaluation():
    R, Z, di = 42.0 * AU, 0.9 * AU, 0.08 * AU
    x, y = R, 0.0
    # Brownian speed above the sound speed is capped at c_s (grains of a few
    # hydrogen masses), with and without turbulence
    for turb in (0, 1):
        p, P = _params(v_frag=math.inf, turbulence=turb)
        for mi, mj in ((1e-25, 3e-25), (2e-26, 2e-26)):
            err, ref = _compare(p, P, x, y, Z, di, mi, mj, 1e-12)
            assert err <= TOL, (turb, mi, mj, err)
    # channels: fragmentation (psi > 0.1), erosion remnant and debris
    # (psi <= 0.1), grouped sticking (psi <= 1e-6) and grouped erosion
    p, P = _params(v_frag=1.0)  # 1 cm/s: every pair below is fast
    mi, _ = _mass_for_stokes(p, R, Z, 0.3)
    for psi in (0.5, 0.1 * (1 - 1e-6), 3e-3, 1e-6 * (1 - 1e-3), 3.3e-9):
        mj = mi * psi
        err, ref = _compare(p, P, x, y, Z, di, mi, mj, 5e3 * mj)
        assert err <= TOL, (psi, err)
        assert ref["type"] == (2 if psi > 0.1 else 1)
    p, P = _params(v_frag=math.inf)
    for psi in (1e-6 * (1 - 1e-3), 2.7e-8):
        mj = mi * psi
        err, ref = _compare(p, P, x, y, Z, di, mi, mj, 5e3 * mj)
        assert err <= TOL and ref["Ng"] > 1, (psi, err)


# One planted mistake per branch and per term of the pair rate; each must be
# caught by the comparison above.
PLANTED = [
    ("tight numerator", "double num = St1 * St2 + tke * (St1 + St2);", "double num = St1 * St2 + tke * (St1 - St2);"),
    ("tight denominator", "(St1 + St2) * (St1 + tke) * (St2 + tke)", "(St1 + St2) * (St1 + tke) * (St1 + tke)"),
    ("tight threshold", "if (St1 < tke) {", "if (St1 < 2.0 * tke) {"),
    ("intermediate 1/(1+y_a)", "1.0 / (1.0 + ya)", "1.0 / (2.0 + ya)"),
    ("intermediate eps^3", "e * e * e / (ya + e)", "e * e / (ya + e)"),
    ("intermediate 2 y_a", "double br = 2.0 * ya - (1.0 + e)", "double br = 2.0 * ya - (1.0 - e)"),
    ("heavy St2 term", "Vg2 * (1.0 / (1.0 + St1) + 1.0 / (1.0 + St2))", "Vg2 * (1.0 / (1.0 + St1) + 1.0 / (1.0 + St1))"),
    ("heavy threshold", "if (St1 < 1.0) {", "if (St1 < 0.5) {"),
    ("V_g^2", "c->Vg2 = 1.5 * P->alpha", "c->Vg2 = 1.0 * P->alpha"),
    ("Reynolds number", "double numol = 0.5 * vth * lmfp;", "double numol = vth * lmfp;"),
    ("radial drift", "double da = dSt * (1.0 - Sti * Stj) / (qi * qj);", "double da = dSt * (1.0 + Sti * Stj) / (qi * qj);"),
    ("azimuthal drift", "double db = -dSt * (Sti + Stj) / (qi * qj);", "double db = -dSt * (Sti - Stj) / (qi * qj);"),
    ("settling cap", "double dz = (Sti < 0.5 && Stj < 0.5) ? dSt : zi - zj;", "double dz = (Sti < 0.5 && Stj < 0.5) ? dSt : zi + zj;"),
    ("Brownian cap", "if (dvB > c->g.cs) dvB = c->g.cs;", ""),
    ("boundary cap", "V = V - ORC_PI * h * h * (3.0 * di - h) / 3.0;", "V = V - ORC_PI * h * h * (3.0 * di + h) / 3.0;"),
    ("kernel", "double K = ORC_PI * ssum * ssum * dv / 4.0;", "double K = ORC_PI * ssum * ssum * dv / 2.0;"),
    ("erosion remnant", "o->rate[0] = (1.0 - psi) * lam / Ng;", "o->rate[0] = (1.0 - psi) * lam;"),
    ("stokes exponent", "g->stfac = P->St0 / P->s0 * pow(xr, -P->p)", "g->stfac = P->St0 / P->s0 * pow(xr, P->p)"),
]


@pytest.mark.parametrize("label,old,new", PLANTED, ids=[x[0] for x in PLANTED])
def test_planted_mistake_is_caught(label, old, new):
    def worst_error():
        worst = 0.0
        p, P = _params(v_frag=math.inf)
        for case in _all_cases(p):
            _, x, y, z, di, mi, mj, Mj, _ = case
            if mj / mi <= 1e-6:
                continue
            got = oracle.pair_rate(P, x, y, z, di, mi, mj, Mj)
            ref = mp_pair(p, x, y, z, di, mi, mj, Mj)
            worst = max(worst, float(abs(_m(got["lam_star"]) / ref["rates"][0] - 1)))
        R, Z, di = 42.0 * AU, 0.9 * AU, 0.08 * AU
        p, P = _params(v_frag=math.inf)
        got = oracle.pair_rate(P, R, 0.0, Z, di, 1e-25, 3e-25, 1e-12)
        ref = mp_pair(p, R, 0.0, Z, di, 1e-25, 3e-25, 1e-12)
        worst = max(worst, float(abs(_m(got["lam_star"]) / ref["rates"][0] - 1)))
        p, P = _params(v_frag=1.0)
        mi, _ = _mass_for_stokes(p, R, Z, 0.3)
        for psi in (3e-3, 3.3e-9):  # erosion, ungrouped and grouped
            mj = psi * mi
            got = oracle.pair_rate(P, R, 0.0, Z, di, mi, mj, 5e3 * mj)
            ref = mp_pair(p, R, 0.0, Z, di, mi, mj, 5e3 * mj)
            worst = max(worst, float(abs(_m(got["rate0"]) / ref["rates"][0] - 1)))
        return worst

    with oracle.planted((old, new)):
        assert worst_error() > 1e-9, label
