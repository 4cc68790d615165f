"""Closed-form references used to pin the oracle (test infrastructure only).

* Smoluchowski solutions of App. A: constant kernel (eq:sol_const), linear
  kernel (eq:sol_linear in its overflow-safe I_1e form) and product kernel.
* The dimensionless Wasserstein distance W1 of App. B between mass-weighted
  cumulative distributions in log10 of the grain mass.
* Kepler's equation for the eccentric-orbit test of Sect. 3.1.
* Terminal radial/azimuthal drift of a grain in a sub-Keplerian disk
  (Nakagawa, Sekiya & Hayashi 1986), the limit the drift terms of eq:dv are
  built from.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize, special, stats


# ---- constant kernel, App. A -------------------------------------------------
def const_mass_fractions(t: float, jmax: int | None = None):
    """Mass fraction in j-mers, f_j = j x^(j-1)/(1+x)^(j+1), x = t/2.

    Follows from eq:sol_const: m n(m) is proportional to m~ (t/2)^(m~-1)/(1+t/2)^(m~+1).
    """
    x = 0.5 * t
    if jmax is None:
        jmax = int(max(64, 60 * (1 + x)))
    j = np.arange(1, jmax + 1, dtype=np.float64)
    logf = np.log(j) + (j - 1) * np.log(x if x > 0 else 1e-300) - (j + 1) * np.log1p(x)
    if x == 0:
        f = np.zeros_like(j)
        f[0] = 1.0
    else:
        f = np.exp(logf)
    return j, f


def const_mpeak(t: float) -> float:
    """eq:m_peak: peak of m^2 n(m) for the constant kernel."""
    return -2.0 / np.log(t / (2.0 + t))


# ---- linear kernel, App. A ---------------------------------------------------
def linear_mass_density(mt, t: float):
    """Mass per unit dimensionless mass, m n(m) m0 / M_d, eq:sol_linear (I_1e form)."""
    mt = np.asarray(mt, dtype=np.float64)
    g = np.exp(-t)
    if t == 0:
        return mt * np.exp(-mt)
    sq = np.sqrt(1.0 - g)
    return g / sq * np.exp(-mt * (g / (1.0 + sq)) ** 2) * special.i1e(2.0 * mt * sq)


def linear_mass_weighted_mean(t: float) -> float:
    """Ratio of the second to the first mass moment: 2 exp(2t) for n(m,0) = e^-m."""
    return 2.0 * np.exp(2.0 * t)


# ---- product kernel, App. A --------------------------------------------------
def product_mass_fractions(t: float, jmax: int = 4000):
    """Mass fraction in j-mers, f_j = (j t)^(j-1) e^(-j t)/j! (product-kernel solution)."""
    j = np.arange(1, jmax + 1, dtype=np.float64)
    if t == 0:
        f = np.zeros_like(j)
        f[0] = 1.0
        return j, f
    logf = (j - 1) * np.log(j * t) - special.gammaln(j + 1) - j * t
    return j, np.exp(logf)


# ---- W1, App. B --------------------------------------------------------------
def w1_discrete(m_sim, M_sim, values, weights) -> float:
    """W1 in log10(m) between a weighted sample and a discrete reference."""
    return float(stats.wasserstein_distance(np.log10(m_sim), np.log10(values),
                                            u_weights=M_sim, v_weights=weights))


def w1_linear(m_sim, M_sim, t: float, npts: int = 4000) -> float:
    """W1 against the linear-kernel solution, reference discretised on a log grid."""
    lo = max(1e-6, np.min(m_sim) * 0.5)
    hi = max(np.max(m_sim) * 2.0, 50.0 * linear_mass_weighted_mean(t))
    edges = np.geomspace(lo, hi, npts + 1)
    mid = np.sqrt(edges[1:] * edges[:-1])
    w = linear_mass_density(mid, t) * np.diff(edges)
    return float(stats.wasserstein_distance(np.log10(m_sim), np.log10(mid), u_weights=M_sim, v_weights=w))


# ---- Kepler orbit, Sect. 3.1 -------------------------------------------------
def kepler_true_anomaly(t, e: float):
    """True anomaly at time t for a = GM = 1, pericentre at t = 0."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.empty_like(t)
    for i, ti in enumerate(t):
        M = ti
        u = optimize.brentq(lambda u: u - e * np.sin(u) - M, M - 1.5, M + 1.5, xtol=1e-15)
        out[i] = 2.0 * np.arctan(np.sqrt((1 + e) / (1 - e)) * np.tan(u / 2.0))
    return out


# ---- Nakagawa et al. 1986 drift ---------------------------------------------
def terminal_drift(eta: float, vK: float, St: float):
    """(v_r, v_phi - v_gas,phi) of a single grain in steady drift, dust-to-gas -> 0.

    Dust: v_r = -2 eta v_K St/(1+St^2), v_phi - v_K = -eta v_K/(1+St^2); gas:
    v_phi - v_K = -eta v_K.  The grain therefore leads the gas by eta v_K St^2/(1+St^2).
    """
    return -2.0 * eta * vK * St / (1.0 + St * St), eta * vK * St * St / (1.0 + St * St)


def damped_oscillator(z0: float, v0: float, ts: float, t):
    """Exact solution of z'' + z'/ts + z = 0 (local column, constant stopping time)."""
    t = np.asarray(t, dtype=np.float64)
    g = 0.5 / ts
    w2 = 1.0 - g * g
    if w2 > 0:
        w = np.sqrt(w2)
        A = z0
        B = (v0 + g * z0) / w
        z = np.exp(-g * t) * (A * np.cos(w * t) + B * np.sin(w * t))
        v = np.exp(-g * t) * ((-g * A + w * B) * np.cos(w * t) + (-g * B - w * A) * np.sin(w * t))
    else:
        k = np.sqrt(-w2)
        r1, r2 = -g + k, -g - k
        c1 = (v0 - r2 * z0) / (r1 - r2)
        c2 = z0 - c1
        z = c1 * np.exp(r1 * t) + c2 * np.exp(r2 * t)
        v = c1 * r1 * np.exp(r1 * t) + c2 * r2 * np.exp(r2 * t)
    return z, v
