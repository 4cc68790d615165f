"""The transport step of Sect. 2.6 on the oracle (reading R36): closed forms
for each constraint on its own, the caps, inactive particles, and the
minimum over many particles."""
import math

import numpy as np
import pytest

import oracle
import workloads


def _one(**kw):
    base = dict(x=1.0, y=0.0, z=0.0, r=1.0, th=0.5 * math.pi, vr=0.0, lth=0.0, lph=1.0, vz=0.0, m=1.0, M=1.0)
    base.update(kw)
    return {k: np.array([v], np.float64) for k, v in base.items()}


def _disk(**kw):
    p = dict(kernel="const", k=32, GM=1.0, R0=1.0, t0=1.0, m0=1.0, rho_s=1.0, s_min=1.0, s0=1.0, St0=1.0,
             h_g0=0.05, p=-1.0, q=0.5, alpha=0.04, Sigma_g0=1.0, r_in=1e-3, r_out=1e3)
    p.update(kw)
    return p


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def test_circular_orbit_has_only_the_orbital_constraint():
    P = oracle.make_problem(_disk())
    # at R = 1 (GM = 1) the circular speed is 1, so u = 0 whatever d is
    assert oracle.transport_dt(P, "global", _one(), [0.01], dt_max=10.0, c_orb=0.05) == 0.05
    # at R = 4: Omega = 1/8, l_phi = R v_K = 4 * 0.5
    st = _one(x=4.0, r=4.0, lph=2.0)
    assert oracle.transport_dt(P, "global", st, [0.01], dt_max=10.0, c_orb=0.05) == 0.4


def test_radial_and_azimuthal_drift():
    P = oracle.make_problem(_disk())
    # v_r = 0.25 on the circular orbit: u = 0.25, d = 0.5 -> c_adv d / u = 2 c_adv
    st = _one(vr=0.25)
    assert oracle.transport_dt(P, "global", st, [0.5], dt_max=10.0, c_orb=2.0, c_adv=0.5) == 1.0
    # v_phi = 2 against v_K = 1: u = 1
    st = _one(lph=2.0)
    assert oracle.transport_dt(P, "global", st, [0.3], dt_max=10.0, c_orb=2.0, c_adv=0.5) == pytest.approx(0.15, rel=1e-15)
    # v_theta = l_theta / r = 0.5 at r = 1 (u = 0.5), d = 0.1, c_adv = 0.5 -> 0.1
    st = _one(lth=0.5)
    assert oracle.transport_dt(P, "global", st, [0.1], dt_max=10.0, c_orb=2.0, c_adv=0.5) == pytest.approx(0.1, rel=1e-15)
    # no neighbourhood radius: the drift term is left out
    assert oracle.transport_dt(P, "global", _one(vr=0.25), [0.0], dt_max=10.0, c_orb=2.0) == 2.0


def test_local_column():
    P = oracle.make_problem(_disk())
    st = _one(vz=-2.0)
    # Omega = 1: the orbital limit is c_orb; drift |v_z| = 2 over d = 0.1
    assert oracle.transport_dt(P, "local", st, [0.1], dt_max=1.0, c_orb=0.05, c_adv=0.5) == 0.025
    assert oracle.transport_dt(P, "local", _one(), [0.1], dt_max=1.0, c_orb=0.05) == 0.05
    # without a push neither constraint applies
    assert oracle.transport_dt(P, "none", st, [0.1], dt_max=1.0, c_orb=0.05) == 1.0


def test_diffusive_constraint_on_the_ring_disk():
    # the ring disk of Sect. 3.2: nu = alpha h_g0^2 R^2 Omega_K = 1e-4 at R = 1,
    # D = nu / (Sc (1 + St^2)) = 5e-5 at St = 1; d = 0.01 -> c_diff d^2 / D = 2 c_diff
    P = oracle.make_problem(workloads.diffusion_ring_params(St=1.0, n=1))
    st = _one()
    got = oracle.transport_dt(P, "none", st, [0.01], dt_max=10.0, c_diff=0.5)
    assert got == pytest.approx(1.0, rel=4e-16)
    # St = 10: D is 101/2 times smaller
    P = oracle.make_problem(workloads.diffusion_ring_params(St=10.0, n=1))
    got = oracle.transport_dt(P, "none", st, [0.01], dt_max=1e9, c_diff=0.5)
    assert got == pytest.approx(50.5, rel=4e-16)
    # Sc_phi = 0.5 in a non-axisymmetric model: the azimuthal direction is the fastest
    cfg = dict(workloads.diffusion_ring_params(St=1.0, n=1), axisym=0, Sc=(1.0, 1.0, 0.5))
    got = oracle.transport_dt(oracle.make_problem(cfg), "none", st, [0.01], dt_max=10.0, c_diff=0.5)
    assert got == pytest.approx(0.5, rel=4e-16)


def test_caps_and_inactive_particles():
    P = oracle.make_problem(_disk())
    st = _one(vr=0.25)
    assert oracle.transport_dt(P, "global", st, [0.5], dt_max=0.3, c_orb=2.0) == 0.3
    assert oracle.transport_dt(P, "global", st, [0.5], dt_max=10.0, dt_out=0.2, c_orb=2.0) == 0.2
    st["M"][:] = 0.0
    assert oracle.transport_dt(P, "global", st, [0.5], dt_max=10.0, c_orb=0.01) == 10.0


def test_minimum_over_particles():
    g = np.random.default_rng(3)
    n = 200
    R = g.uniform(0.5, 3.0, n)
    ph = g.uniform(0, 2 * math.pi, n)
    st = dict(x=R * np.cos(ph), y=R * np.sin(ph), z=np.zeros(n), r=R, th=np.full(n, 0.5 * math.pi),
              vr=g.normal(0, 0.1, n), lth=g.normal(0, 0.05, n), lph=R / np.sqrt(R) + g.normal(0, 0.1, n),
              vz=np.zeros(n), m=np.ones(n), M=np.where(g.uniform(size=n) < 0.9, 1.0, 0.0))
    d = g.uniform(0.0, 0.2, n)
    P = oracle.make_problem(_disk(diffusion="concentration", St_diff=0.3))
    whole = oracle.transport_dt(P, "global", st, d, dt_max=10.0)
    each = [oracle.transport_dt(P, "global", {k: v[i:i + 1] for k, v in st.items()}, d[i:i + 1], dt_max=10.0)
            for i in range(n)]
    assert whole == min(each) and whole < 10.0
