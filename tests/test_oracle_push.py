"""Pins of the oracle's semi-analytic push (Sect. 2.3.3).

References: exact damped-oscillator solution (local column, constant stopping
time), terminal settling, the eccentric-orbit test of Sect. 3.1 (values printed
in the paper, tests/golden/orbit_e05.txt) and the steady drift of a grain in a
sub-Keplerian disk (Nakagawa et al. 1986).
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import analytic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run_local(z0, v0, st, dt, nsteps):
    z = np.array([z0])
    v = np.array([v0])
    for _ in range(nsteps):
        z, v = oracle.push_local(z, v, np.array([st]), np.ones(1), dt)
    return z[0], v[0]


def test_local_push_second_order_against_damped_oscillator():
    # tiny amplitude: t_s = St exp(z^2/2) is constant to 1e-12, so z'' + z'/t_s + z = 0
    z0, v0, st, T = 1e-6, 0.0, 0.7, 6.0
    ze, ve = analytic.damped_oscillator(z0, v0, st, T)
    errs = []
    for n in (60, 120, 240, 480):
        z, v = _run_local(z0, v0, st, T / n, n)
        errs.append(abs(z - ze) / z0)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (orders > 1.8).all() and (orders < 2.3).all()
    assert errs[-1] < 1e-4


def test_local_push_drag_free_is_leapfrog():
    # St huge: DKD leapfrog on the harmonic oscillator, exact energy bounded
    z0, T = 0.5, 20.0
    for n in (200, 400):
        z, v = _run_local(z0, 0.0, 1e15, T / n, n)
        # leapfrog conserves a modified energy: error O(dt^2), bounded in time
        assert abs(0.5 * (z * z + v * v) - 0.5 * z0 * z0) < 0.5 * (T / n) ** 2 * z0 * z0


def test_local_push_stiff_terminal_settling():
    # St << dt << 1: each step gives the terminal velocity v = -z t_s, so
    # z(t) = z0 exp(-St t) (settling on the stopping time), any dt
    st, z0 = 1e-4, 1.0
    for dt in (0.05, 0.2):
        n = int(round(100.0 / dt))
        z, v = _run_local(z0, 0.0, st, dt, n)
        zt = z0 * math.exp(-st * n * dt)
        # z^2/2 variation of t_s is O(1): compare against the settling ODE dz/dt = -St e^{z^2/2} z
        from scipy.integrate import solve_ivp
        sol = solve_ivp(lambda t, y: [-st * math.exp(0.5 * y[0] ** 2) * y[0]], (0, n * dt), [z0],
                        rtol=1e-12, atol=1e-14)
        assert abs(z - sol.y[0, -1]) < 1e-3 * abs(sol.y[0, -1])
        assert abs(v + z * st * math.exp(0.5 * z * z)) < 1e-3 * abs(v)
        assert zt > 0


def _global_problem(**over):
    cfg = dict(kernel="physical", k=32, GM=1.0, R0=1.0, p=-1.0, q=-1.0, h_g0=0.05, Sigma_g0=1.0,
               rho_s=1.0, s0=1.0, s_min=1.0, St0=0.1, r_in=1e-3, r_out=1e3, drag=0)
    cfg.update(over)
    return oracle.make_problem(cfg)


def _orbit_state():
    # pericentre of an e = 0.5, a = 1 orbit: (R, phi, v_r, l_phi) = (1/2, 0, 0, sqrt(3)/2)
    r = np.array([0.5])
    th = np.array([math.pi / 2])
    return dict(r=r, th=th, ph=np.zeros(1), vr=np.zeros(1), lth=np.zeros(1),
                lph=np.array([math.sqrt(3) / 2]), m=np.ones(1), M=np.ones(1),
                x=r.copy(), y=np.zeros(1), z=np.zeros(1))


def _energy(s):
    r = s["r"][0]
    st = math.sin(s["th"][0])
    return 0.5 * (s["vr"][0] ** 2 + (s["lth"][0] / r) ** 2 + (s["lph"][0] / (r * st)) ** 2) - 1.0 / r


def test_eccentric_orbit_energy_error():
    gold = {}
    for line in open(os.path.join(GOLD, "orbit_e05.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            gold[k] = float(v)
    P = _global_problem()
    P0 = 2 * math.pi
    errs = []
    for div in (80, 160, 320, 640):
        s = _orbit_state()
        E0 = _energy(s)
        assert E0 == pytest.approx(gold["E_exact"], rel=1e-15)
        dt = P0 / div
        worst = 0.0
        for _ in range(int(gold["orbits"]) * div):
            s = oracle.push_global(P, s, dt)
            worst = max(worst, abs(_energy(s) - E0) / abs(E0))
        errs.append(worst)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # second-order energy error and the paper's bound at P0/640
    assert (orders > 1.7).all() and (orders < 2.3).all(), (errs, orders)
    assert errs[-1] < gold["max_rel_energy_error_at_P0_640"]


def test_eccentric_orbit_phase_converges():
    P = _global_problem()
    P0 = 2 * math.pi
    out = []
    for div in (160, 320):
        s = _orbit_state()
        n = 5 * div
        for _ in range(n):
            s = oracle.push_global(P, s, P0 / div)
        out.append(s["ph"][0] - 5 * 2 * math.pi)
    exact = analytic.kepler_true_anomaly(5 * P0, 0.5)[0]
    e1, e2 = abs(out[0] - exact), abs(out[1] - exact)
    assert e2 < e1 / 3.0


@pytest.mark.parametrize("St", [0.01, 0.1, 1.0, 10.0])
def test_global_push_terminal_drift(St):
    # a grain at the midplane of a p = q = -1 disk settles into the steady drift
    P = _global_problem(drag=1, St0=St)
    g = oracle.gas_at(P, 1.0, 0.0)
    s = dict(r=np.array([1.0]), th=np.array([math.pi / 2]), ph=np.zeros(1), vr=np.zeros(1),
             lth=np.zeros(1), lph=np.array([g["vgphi"]]), m=np.array([math.pi / 6]), M=np.ones(1),
             x=np.ones(1), y=np.zeros(1), z=np.zeros(1))
    ts = St  # Omega_K = 1 at R0
    dt = min(ts, 1.0) / 20.0
    n = int(math.ceil(max(15 * ts, 15.0) / dt))
    for _ in range(n):
        s = oracle.push_global(P, s, dt)
    R = s["r"][0]
    gR = oracle.gas_at(P, R, 0.0)
    St_R = gR["stfac"] * 1.0
    vK = math.sqrt(1.0 / R)
    vr_exp, dvphi_exp = analytic.terminal_drift(gR["eta"], vK, St_R)
    assert abs(s["vr"][0] - vr_exp) < 0.02 * abs(vr_exp)
    dvphi = s["lph"][0] / R - gR["vgphi"]
    vg_ref = -gR["eta"] * vK
    # azimuthal velocity relative to the gas, within a few per cent of eta v_K
    # (the global disk adds O(v_r/v_K) corrections to the local solution)
    assert abs(dvphi - dvphi_exp) < 0.05 * abs(vg_ref)
