"""Pins of the oracle's dust-diffusion step (Sect. 2.4) against what the paper
and the mathematics fix, independently of the oracle's own formulas:

  * the ring-spreading test of Sect. 3.2: ln(R/R0) of a ring under D = D0 (R/R0)^2
    keeps a normal distribution with mean (2 + chi p) D0 t / R0^2 and variance
    sigma0^2 + 2 D0 t / R0^2, for both the concentration (chi = 1) and the
    density (chi = 0) form; at equal dimensionless time and step the result does
    not depend on St (the coinciding panels of the test);
  * the azimuthal step has variance 2 D_phi dt / R^2, which for D ~ R^2 is the
    same for every particle;
  * the analytic gradients of D and ln rho_g equal central differences of the
    coefficients themselves (3D and vertically integrated disks, with a
    position-dependent Stokes number);
  * dust distributed like the gas is a stationary state of the concentration
    form (its flux vanishes when rho_d / rho_g is uniform) -- in 3D, where the
    vertical drift terms and the Stokes-number gradient matter;
  * the Cartesian velocity is unchanged by the step, and a radial step past
    the axis is the same Cartesian displacement.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def ring_params(chi_form="concentration", St=1.0, Sc=(1.0, 1.0, 1.0), axisym=1, p=-1.0):
    # 1D radial disk of the ring test: h_g0 = 0.05, p = -1, q = 0.5, alpha = 0.04,
    # code units GM = R0 = 1 (so nu = 1e-4 (R/R0)^2)
    return workloads.diffusion_ring_params(chi_form, St=St, Sc=Sc, axisym=axisym, p=p)


def ring_state(n, seed, sigma0=0.05):
    return workloads.diffusion_ring(seed, n, sigma0)


def run_ring(cfg, n, t_tilde, dtt, seed=11):
    P = oracle.make_problem(cfg)
    D0 = 1e-4 / (1.0 + cfg["St_diff"] ** 2)
    dt = dtt / D0                       # t~ = D0 t / R0^2
    st = ring_state(n, seed)
    ph0 = st["ph"].copy()
    for step in range(int(round(t_tilde / dtt))):
        st = oracle.diffuse(P, st, dt, 0x5EED, step)
    st["id"] = np.arange(n, dtype=np.uint32)
    return st, ph0


@pytest.mark.parametrize("form,chi", [("concentration", 1.0), ("density", 0.0)])
def test_ring_mean_and_variance(form, chi):
    n, tt = 1 << 16, 0.1
    st, _ = run_ring(ring_params(form), n, tt, 2e-4)
    lnR = np.log(st["r"])
    mu, var = lnR.mean(), lnR.var()
    p = -1.0
    mu_exact = (2.0 + chi * p) * tt
    var_exact = 0.05 ** 2 + 2.0 * tt
    assert abs(var_exact - 0.2025) < 1e-15
    # sampling errors: sd(mu) = sigma/sqrt(n), sd(var) = var sqrt(2/n)
    assert abs(mu - mu_exact) < 5.0 * math.sqrt(var_exact / n), (mu, mu_exact)
    assert abs(var - var_exact) < 5.0 * var_exact * math.sqrt(2.0 / n), (var, var_exact)
    # the distribution stays normal in ln R: skewness and excess kurtosis near 0
    zs = (lnR - mu) / math.sqrt(var)
    assert abs((zs ** 3).mean()) < 5.0 * math.sqrt(6.0 / n)
    assert abs((zs ** 4).mean() - 3.0) < 5.0 * math.sqrt(24.0 / n)


def test_ring_schmidt_number_rescales_time():
    # Sc_R = 2 halves D_R: the ring at t~ = 0.1 looks like Sc = 1 at t~ = 0.05
    n, tt = 1 << 15, 0.1
    st, _ = run_ring(ring_params("concentration", Sc=(2.0, 1.0, 1.0)), n, tt, 4e-4)
    lnR = np.log(st["r"])
    mu_exact = (2.0 - 1.0) * tt / 2.0
    var_exact = 0.05 ** 2 + 2.0 * tt / 2.0
    assert abs(lnR.mean() - mu_exact) < 5.0 * math.sqrt(var_exact / n)
    assert abs(lnR.var() - var_exact) < 5.0 * var_exact * math.sqrt(2.0 / n)


def test_ring_independent_of_stokes_number_at_equal_dimensionless_time():
    a, _ = run_ring(ring_params("density", St=0.1), 4096, 0.01, 1e-3)
    b, _ = run_ring(ring_params("density", St=10.0), 4096, 0.01, 1e-3)
    np.testing.assert_allclose(a["r"], b["r"], rtol=1e-12, atol=0)


def test_azimuthal_step_variance():
    # D_phi = D0 R^2 / Sc_phi: every step has variance 2 D0 dt / Sc_phi whatever R
    n, tt = 1 << 15, 0.1
    st, ph0 = run_ring(ring_params("concentration", Sc=(1.0, 1.0, 2.0), axisym=0), n, tt, 4e-4)
    dphi = st["ph"] - ph0
    var_exact = 2.0 * tt / 2.0
    assert abs(dphi.mean()) < 5.0 * math.sqrt(var_exact / n)
    assert abs(dphi.var() - var_exact) < 5.0 * var_exact * math.sqrt(2.0 / n)
    # the radial distribution is that of the axisymmetric run (same normals)
    ax, _ = run_ring(ring_params("concentration", Sc=(1.0, 1.0, 2.0), axisym=1), n, tt, 4e-4)
    np.testing.assert_allclose(st["r"], ax["r"], rtol=1e-13, atol=0)


def disk3d_params(form="concentration", St_diff=0.0, vint=0):
    return dict(kernel="physical", k=32, GM=1.0, R0=1.0, p=-1.5, q=-0.5, h_g0=0.05, alpha=0.02, Sigma_g0=1.0,
                St0=1.0, s0=1.0, rho_s=1.0, r_in=0.1, r_out=10.0, diffusion=form, vint=vint, axisym=0,
                Sc=(1.0, 1.5, 0.7), St_diff=St_diff)


@pytest.mark.parametrize("vint,St_diff", [(0, 0.0), (0, 0.3), (1, 0.0)])
def test_gradients_match_central_differences(vint, St_diff):
    P = oracle.make_problem(disk3d_params(St_diff=St_diff, vint=vint))
    rng = np.random.default_rng(3)
    for _ in range(40):
        R = rng.uniform(0.4, 2.5)
        H = 0.05 * R ** 0.25 * R
        Z = 0.0 if vint else rng.uniform(-3.0, 3.0) * H
        s = rng.uniform(0.05, 3.0)
        c = oracle.diff_coeffs(P, R, Z, s)
        h = 1e-5 * R
        cp, cm = oracle.diff_coeffs(P, R + h, Z, s), oracle.diff_coeffs(P, R - h, Z, s)
        np.testing.assert_allclose(c["dDR_dR"], (cp["D_R"] - cm["D_R"]) / (2 * h), rtol=1e-6,
                                   atol=1e-9 * c["D_R"] / R)
        np.testing.assert_allclose(c["dlnrho_dR"], (cp["lnrho"] - cm["lnrho"]) / (2 * h), rtol=1e-6, atol=1e-8 / R)
        if not vint:
            hz = 1e-5 * H
            zp, zm = oracle.diff_coeffs(P, R, Z + hz, s), oracle.diff_coeffs(P, R, Z - hz, s)
            np.testing.assert_allclose(c["dDZ_dZ"], (zp["D_Z"] - zm["D_Z"]) / (2 * hz), rtol=1e-6,
                                       atol=1e-9 * c["D_Z"] / H)
            np.testing.assert_allclose(c["dlnrho_dZ"], (zp["lnrho"] - zm["lnrho"]) / (2 * hz), rtol=1e-6,
                                       atol=1e-8 / H)
        # D itself: nu = alpha c_s H_g with c_s = h_g v_K, H_g = h_g R, h_g = h_g0 (R/R0)^((q+1)/2)
        hg = 0.05 * R ** 0.25
        nu = 0.02 * hg * hg * R * R * math.sqrt(1.0 / R ** 3)
        if St_diff > 0:
            St = St_diff
        else:
            Zg = 0.0 if vint else Z
            w = 1.0 - R / math.hypot(R, Zg)
            St = 1.0 * s * R ** 1.5 * math.exp(w / hg ** 2)
        for a, Sc in enumerate((1.0, 1.5, 0.7)):
            key = ("D_R", "D_Z", "D_phi")[a]
            np.testing.assert_allclose(c[key], nu / (Sc * (1.0 + St * St)), rtol=1e-11)


def _rho_gas(R, Z, p=-1.5, q=-0.5, h0=0.05):
    # Sect. 2.2: rho_g = Sigma_g/(sqrt(2 pi) H_g) exp(-(1 - R/r)/h_g^2), Sigma_g ~ R^p, h_g ~ R^((q+1)/2)
    hg = h0 * R ** ((q + 1.0) / 2.0)
    r = np.hypot(R, Z)
    return R ** p / (math.sqrt(2 * math.pi) * hg * R) * np.exp(-(1.0 - R / r) / hg ** 2)


def _gas_like_sample(n, seed):
    # cylindrical number density R rho_g(R, Z) on 0.4 < R < 1.6 by rejection
    rng = np.random.default_rng(seed)
    Rg = np.linspace(0.4, 1.6, 400)
    fmax = 1.05 * float((Rg * _rho_gas(Rg, 0.0)).max())
    R = np.empty(0)
    Z = np.empty(0)
    while len(R) < n:
        r_ = rng.uniform(0.4, 1.6, 4 * n)
        z_ = rng.uniform(-0.5, 0.5, 4 * n)
        keep = rng.uniform(0.0, fmax, 4 * n) < r_ * _rho_gas(r_, z_)
        R = np.concatenate([R, r_[keep]])
        Z = np.concatenate([Z, z_[keep]])
    R, Z = R[:n], Z[:n]
    ph = rng.uniform(0.0, 2 * math.pi, n)
    s = rng.uniform(0.3, 1.0, n)                    # St = 0.3 .. 1 at R0, larger off the midplane
    r = np.hypot(R, Z)
    z0 = np.zeros(n)
    return dict(id=np.arange(n, dtype=np.uint32), r=r, th=np.arctan2(R, Z), ph=ph, vr=z0.copy(), lth=z0.copy(),
                lph=z0.copy(), m=math.pi / 6.0 * s ** 3, M=np.ones(n), x=R * np.cos(ph), y=R * np.sin(ph), z=Z)


def _band_stats(st):
    R = st["r"] * np.sin(st["th"])
    Z = st["r"] * np.cos(st["th"])
    band = (R > 0.85) & (R < 1.15) & (st["M"] > 0)
    H = 0.05 * R[band] ** 0.25 * R[band]
    return band.mean(), (Z[band] / H) ** 2, Z[band] / H, int(band.sum())


def test_gas_like_dust_is_stationary_under_concentration_diffusion():
    n = 1 << 17
    P = oracle.make_problem(disk3d_params("concentration"))
    st = _gas_like_sample(n, 21)
    for step in range(400):                         # t = 200 ~ 2-4 vertical mixing times H^2/D
        st = oracle.diffuse(P, st, 0.5, 0xD1FF, step)
        st["id"] = np.arange(n, dtype=np.uint32)
    ref = _gas_like_sample(n, 22)                   # an independent sample of the initial state
    fa, z2a, za, na = _band_stats(st)
    fb, z2b, zb, nb = _band_stats(ref)
    sd = math.sqrt(2.0 * fb * (1.0 - fb) / n)
    assert abs(fa - fb) < 5.0 * sd, (fa, fb)
    sd2 = math.sqrt(z2a.var() / na + z2b.var() / nb)
    assert abs(z2a.mean() - z2b.mean()) < 5.0 * sd2, (z2a.mean(), z2b.mean())
    assert abs(za.mean()) < 5.0 * math.sqrt(za.var() / na)


def test_density_form_spreads_gas_like_dust():
    # the density form has no term holding dust to the gas: the same state
    # thickens vertically (control for the stationarity test above)
    n = 1 << 14
    P = oracle.make_problem(disk3d_params("density"))
    st = _gas_like_sample(n, 21)
    for step in range(200):
        st = oracle.diffuse(P, st, 0.5, 0xD1FF, step)
        st["id"] = np.arange(n, dtype=np.uint32)
    _, z2a, _, _ = _band_stats(st)
    _, z2b, _, _ = _band_stats(_gas_like_sample(n, 22))
    assert z2a.mean() > 1.25 * z2b.mean()


def _cart_velocity(st):
    r, th, ph = st["r"], st["th"], st["ph"]
    R = r * np.sin(th)
    vr, vt, vp = st["vr"], st["lth"] / r, st["lph"] / R
    e_r = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    e_t = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    e_p = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)])
    return vr * e_r + vt * e_t + vp * e_p


def test_cartesian_velocity_and_position_consistency():
    n = 2000
    st = _gas_like_sample(n, 5)
    rng = np.random.default_rng(6)
    st["vr"] = rng.normal(0, 0.05, n)
    st["lth"] = rng.normal(0, 0.05, n) * st["r"]
    st["lph"] = (1.0 + rng.normal(0, 0.05, n)) * np.sqrt(st["r"] * np.sin(st["th"]))
    P = oracle.make_problem(disk3d_params("concentration"))
    v0 = _cart_velocity(st)
    out = oracle.diffuse(P, st, 50.0, 7, 0)
    np.testing.assert_allclose(_cart_velocity(out), v0, rtol=1e-12, atol=1e-14)
    r, th, ph = out["r"], out["th"], out["ph"]
    np.testing.assert_allclose(out["x"], r * np.sin(th) * np.cos(ph), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["y"], r * np.sin(th) * np.sin(ph), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["z"], r * np.cos(th), rtol=1e-13, atol=1e-15)
    assert not np.allclose(out["r"], st["r"])


def test_step_past_the_axis_is_a_cartesian_displacement():
    # without azimuthal and vertical steps the displacement lies along e_R(phi0):
    # (x', y') . e_R(phi0) = R + dR, also when R + dR < 0.  With chi = 1 and
    # p = -3 the drift D/R + dD/dR + D dln Sigma_g/dR of D = D0 R^2 vanishes,
    # so dR is normal with mean 0 and variance 2 D dt = (0.02)^2 for D0 dt = 1/2.
    P = oracle.make_problem(ring_params("concentration", St=1.0, axisym=1, p=-3.0))
    n = 4096
    st = ring_state(n, 8)
    st["r"] = np.full(n, 0.02)
    st["x"] = st["r"] * np.cos(st["ph"])
    st["y"] = st["r"] * np.sin(st["ph"])
    D0 = 1e-4 / 2.0
    out = oracle.diffuse(P, st, 0.5 / D0, 9, 0)
    proj = out["x"] * np.cos(st["ph"]) + out["y"] * np.sin(st["ph"])
    perp = -out["x"] * np.sin(st["ph"]) + out["y"] * np.cos(st["ph"])
    crossed = proj < 0
    assert crossed.sum() > n // 20 and (~crossed).any()
    np.testing.assert_allclose(np.abs(proj), out["r"], rtol=1e-12)
    np.testing.assert_allclose(perp, 0.0, atol=1e-13)
    dR = proj - 0.02
    var = 0.02 ** 2
    assert abs(dR.mean()) < 5.0 * math.sqrt(var / n)
    assert abs(dR.var() - var) < 5.0 * var * math.sqrt(2.0 / n)


def test_normals_are_standard():
    z = np.array([oracle.diff_normals(42, i, 3) for i in range(20000)])
    assert np.all(np.abs(z.mean(axis=0)) < 5.0 / math.sqrt(20000))
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 5.0 * math.sqrt(2.0 / 20000))
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5.0 / math.sqrt(20000)
    # two steps draw different numbers
    assert not np.allclose(oracle.diff_normals(42, 1, 3), oracle.diff_normals(42, 1, 4))
