"""Seeded synthetic workloads shared by the tests, the oracle and the benchmark.

This module only draws inputs and states problem parameters.  It contains none
of the method's steps: no neighbour search, rate, outcome, controller or push
arithmetic.  Random numbers are numpy PCG64 streams keyed by the seed.

Workloads (stand-ins for the paper's coagulation tests and disk benchmark,
whose own setups and data are not available):

  const_box      4096 particles, uniform in a periodic unit cube, m = m0 = 1,
                 equal particle masses, constant kernel, k = 32 (App. A test).
  additive_col   65,536 particles, x, y uniform in a periodic unit square,
                 z ~ N(0, 1), St_mid log-uniform 1e-4..1e-1, m ~ Gamma(2, 1),
                 equal particle masses, additive kernel, k = 32, local settling.
  disk3d         1,048,576 particles in a 3D annulus r in [10, 100] au with
                 dN/dr constant (Sigma_g ~ r^-1), z/r ~ N(0, h_g = 0.05),
                 uniform azimuth, grain diameter 2 um (radius 1 um), density
                 1.6 g/cm^3, dust-to-gas 0.01, alpha = 1e-3, v_frag = 1 m/s,
                 k = 32, Keplerian initial velocities.  cgs units.
  disk3d_warm    as disk3d but grain radius log-uniform 1 um .. 1 mm (a builder
                 addition that exercises fragmentation, erosion and grouping).
  local_box      a periodic cube of side 0.005 R at the midplane of the annulus
                 at radius R: the annulus physics (gas model, Brownian + OC07,
                 sticking / erosion / fragmentation), no push, grain radius
                 log-uniform 1 um .. 1 mm, dust-to-gas 0.01 of the midplane
                 gas density, per-box alpha and v_frag.
  box_batch      256 such boxes: N log-uniform 2^10..2^16, R uniform in
                 [10, 100] au, alpha log-uniform 1e-4..1e-2, v_frag uniform
                 1..10 m/s (the batched-boxes configuration).
  diffusion_ring the dust-ring test of Sect. 3.2: 2^20 particles with
                 ln(R/R0) ~ N(0, 0.05^2) at zero velocity in a 1D radial disk
                 (h_g0 = 0.05, p = -1, q = 0.5, alpha = 0.04, GM = R0 = 1),
                 Sc = 1, one spatially constant St in {0.1, 1, 10},
                 concentration or density form; uniform azimuth.
"""
from __future__ import annotations

import math

import numpy as np

# cgs constants
G_CGS = 6.67430e-8
MSUN = 1.98847e33
AU = 1.495978707e13
YR = 3.15576e7
M_H = 1.6735575e-24

PHYS_KEYS = ("r", "th", "ph", "vr", "lth", "lph")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------- #
def const_box_params(n: int = 4096, k: int = 32) -> dict:
    return dict(name="const_box", kernel="const", k=k, n=n, t0=1.0, m0=1.0, eps=0.08,
                dt_fn_max=0.01, dt_coll=0.01, t_end=10.0, periodic=(1, 1, 1), L=(1.0, 1.0, 1.0),
                erosion=0, grouping=1, push="none")


def const_box(seed: int, n: int = 4096) -> dict:
    g = _rng(seed)
    pos = g.random((3, n))
    return dict(id=np.arange(n, dtype=np.uint32), x=pos[0], y=pos[1], z=pos[2],
                M=np.full(n, 1.0 / n), m=np.ones(n))


def additive_col_params(n: int = 65536, k: int = 32) -> dict:
    return dict(name="additive_col", kernel="additive", k=k, n=n, t0=1.0, m0=1.0, eps=0.08,
                dt_fn_max=0.2, dt_coll=0.2, n_intervals=100, periodic=(1, 1, 0), L=(1.0, 1.0, 1.0),
                erosion=0, grouping=1, push="local")


def additive_col(seed: int, n: int = 65536) -> dict:
    g = _rng(seed)
    x = g.random(n)
    y = g.random(n)
    z = g.standard_normal(n)
    st = 10.0 ** g.uniform(-4.0, -1.0, n)
    m = g.gamma(2.0, 1.0, n)
    return dict(id=np.arange(n, dtype=np.uint32), x=x, y=y, z=z, vz=np.zeros(n), st_mid=st,
                M=np.full(n, 1.0 / n), m=m)


def disk3d_params(n: int = 1 << 20, k: int = 32, alpha: float = 1e-3, v_frag: float = 100.0) -> dict:
    GM = G_CGS * MSUN
    R0 = 10.0 * AU
    r_in, r_out = 10.0 * AU, 100.0 * AU
    m_gas = 0.01 * MSUN
    # Sigma_g = Sigma_g0 (R/R0)^-1 holding m_gas between r_in and r_out
    sigma_g0 = m_gas / (2.0 * math.pi * R0 * (r_out - r_in))
    rho_s = 1.6
    s0 = 2.0e-4  # reference (= minimum) grain diameter: radius 1 um
    # Epstein midplane Stokes number of the reference grain at R0
    st0 = math.pi * rho_s * s0 / (4.0 * sigma_g0)
    period10 = 2.0 * math.pi / math.sqrt(GM / R0 ** 3)
    return dict(name="disk3d", kernel="physical", k=k, n=n, eps=0.08,
                dt_fn_max=period10 / 50.0, dt_coll=period10 / 50.0,
                periodic=(0, 0, 0), L=(1.0, 1.0, 1.0), erosion=1, grouping=1, push="global",
                rho_s=rho_s, s_min=s0, s0=s0, St0=st0, v_frag=v_frag, GM=GM, Sigma_g0=sigma_g0,
                R0=R0, p=-1.0, q=-1.0, h_g0=0.05, alpha=alpha, mu_mH=2.34 * M_H, sigma_H2=2.0e-15,
                r_in=r_in, r_out=r_out, drag=1, brownian=1, turbulence=1, caps=1,
                dust_to_gas=0.01, m_gas=m_gas)


def disk3d(seed: int, n: int = 1 << 20, warm: bool = False, params: dict | None = None) -> dict:
    P = params or disk3d_params(n)
    g = _rng(seed)
    r = g.uniform(P["r_in"], P["r_out"], n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    zeta = np.clip(g.normal(0.0, P["h_g0"], n), -0.9, 0.9)  # cos(theta) = z/r
    th = np.arccos(zeta)
    st = np.sin(th)
    x = r * st * np.cos(ph)
    y = r * st * np.sin(ph)
    z = r * np.cos(th)
    if warm:
        a = 10.0 ** g.uniform(-4.0, -1.0, n)  # grain radius 1 um .. 1 mm
        s = 2.0 * a
    else:
        s = np.full(n, P["s0"])
    m = math.pi * P["rho_s"] * s ** 3 / 6.0  # grain mass of a sphere of diameter s
    Md = P["dust_to_gas"] * P["m_gas"]
    R = r * st
    lph = np.sqrt(P["GM"] * R)  # Keplerian specific angular momentum
    return dict(id=np.arange(n, dtype=np.uint32), x=x, y=y, z=z, r=r, th=th, ph=ph,
                vr=np.zeros(n), lth=np.zeros(n), lph=lph, M=np.full(n, Md / n), m=m)


def local_box_params(n: int, R_au: float = 30.0, alpha: float = 1e-3, v_frag: float = 100.0, k: int = 32) -> dict:
    """A periodic cube of side 0.005 R at the midplane of the annulus at R."""
    P = disk3d_params(n, k=k, alpha=alpha, v_frag=v_frag)
    R = R_au * AU
    side = 0.005 * R
    period = 2.0 * math.pi / math.sqrt(P["GM"] / R ** 3)
    P.update(name="local_box", periodic=(1, 1, 1), L=(side, side, side), push="none",
             dt_fn_max=period / 50.0, dt_coll=period / 50.0, R_box=R)
    return P


def local_box(seed: int, n: int, params: dict) -> dict:
    g = _rng(seed)
    R, side = params["R_box"], params["L"][0]
    x = R + side * g.random(n)
    y = side * (g.random(n) - 0.5)
    z = side * (g.random(n) - 0.5)
    a = 10.0 ** g.uniform(-4.0, -1.0, n)  # grain radius 1 um .. 1 mm
    m = math.pi * params["rho_s"] * (2.0 * a) ** 3 / 6.0
    # dust-to-gas 0.01 of the midplane gas density Sigma_g / (sqrt(2 pi) H), H = h_g0 R
    sigma = params["Sigma_g0"] * (R / params["R0"]) ** params["p"]
    rho_g = sigma / (math.sqrt(2.0 * math.pi) * params["h_g0"] * R)
    Md = params["dust_to_gas"] * rho_g * side ** 3
    return dict(id=np.arange(n, dtype=np.uint32), x=x, y=y, z=z, M=np.full(n, Md / n), m=m)


def box_batch(seed: int, nbox: int = 256, lo: int = 10, hi: int = 16):
    """[(params, state, seed)] of nbox independent local boxes."""
    g = _rng(seed)
    out = []
    for b in range(nbox):
        n = int(round(2.0 ** g.uniform(lo, hi)))
        R_au = g.uniform(10.0, 100.0)
        alpha = 10.0 ** g.uniform(-4.0, -2.0)
        v_frag = 100.0 * g.uniform(1.0, 10.0)  # cm/s
        P = local_box_params(n, R_au=R_au, alpha=alpha, v_frag=v_frag)
        out.append((P, local_box(seed * 1000 + b, n, P), seed * 1000 + b))
    return out


def diffusion_ring_params(form: str = "concentration", St: float = 1.0, n: int = 1 << 20,
                          Sc=(1.0, 1.0, 1.0), axisym: int = 1, p: float = -1.0) -> dict:
    """The 1D radial disk of the ring-spreading test (code units GM = R0 = 1)."""
    return dict(name="diffusion_ring", kernel="physical", k=32, n=n, GM=1.0, R0=1.0, p=p, q=0.5, h_g0=0.05,
                alpha=0.04, Sigma_g0=1.0, St0=1.0, s0=1.0, rho_s=1.0, s_min=1.0, r_in=1e-3, r_out=1e3,
                push="none", diffusion=form, vint=1, axisym=axisym, Sc=tuple(Sc), St_diff=St, dt_coll=1.0,
                t0=1.0, m0=1.0)


def diffusion_ring(seed: int, n: int = 1 << 20, sigma0: float = 0.05) -> dict:
    g = _rng(seed)
    R = np.exp(g.normal(0.0, sigma0, n))
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    th = np.full(n, 0.5 * math.pi)
    zero = np.zeros(n)
    return dict(id=np.arange(n, dtype=np.uint32), r=R, th=th, ph=ph, vr=zero.copy(), lth=zero.copy(),
                lph=zero.copy(), m=np.ones(n), M=np.full(n, 1.0 / n), x=R * np.cos(ph), y=R * np.sin(ph),
                z=zero.copy())


def lattice_box(nside: int, jitter: float = 0.0, seed: int = 0) -> dict:
    """Particles on a cubic lattice in the periodic unit cube (exact distance ties)."""
    g = _rng(seed)
    c = (np.arange(nside) + 0.5) / nside
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    if jitter:
        x = x + jitter * g.standard_normal(x.size)
        y = y + jitter * g.standard_normal(x.size)
        z = z + jitter * g.standard_normal(x.size)
    n = x.size
    return dict(id=np.arange(n, dtype=np.uint32), x=x, y=y, z=z, M=np.full(n, 1.0 / n), m=np.ones(n))


def by_name(name: str, seed: int, n: int | None = None):
    """(params, state) of a named workload."""
    if name == "const_box":
        P = const_box_params(n or 4096)
        return P, const_box(seed, P["n"])
    if name == "additive_col":
        P = additive_col_params(n or 65536)
        return P, additive_col(seed, P["n"])
    if name in ("disk3d", "disk3d_warm"):
        P = disk3d_params(n or (1 << 20))
        if name == "disk3d_warm":
            P["name"] = "disk3d_warm"
        return P, disk3d(seed, P["n"], warm=(name == "disk3d_warm"), params=P)
    raise KeyError(name)
