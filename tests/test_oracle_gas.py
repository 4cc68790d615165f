"""Pins of the oracle's gas disk (Sect. 2.2) and Stokes number (Sect. 2.3.1)
against physics they must satisfy, independently of how the oracle writes
them:

  * the vertical integral of rho_g is Sigma_g up to O(h_g^2) (slightly above:
    the density profile exp(-(1 - R/r)/h^2) has heavier tails than a Gaussian);
  * the gas is in hydrostatic balance with P = rho_g c_s^2: vertically,
    (1/rho) dP/dZ = -GM Z/r^3, and radially the azimuthal speed carries the
    rest, v_phi^2/R = GM R/r^3 + (1/rho) dP/dR (derivatives by central
    differences of the oracle's own rho_g and c_s), for several density and
    temperature slopes;
  * the Stokes number follows the Epstein scaling St ~ Omega_K s/(rho_g c_s).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
import workloads

AU = workloads.AU


def _problem(p, q):
    return oracle.make_problem(dict(workloads.disk3d_params(1000), p=p, q=q))


@pytest.mark.parametrize("p,q", [(-1.0, -1.0), (-1.5, -0.5), (-0.5, 0.0)])
def test_vertical_integral_is_the_surface_density(p, q):
    P = _problem(p, q)
    for R_au in (12.0, 45.0, 90.0):
        R = R_au * AU
        g = oracle.gas_at(P, R, 0.0)
        Sig = P.Sigma_g0 * (R / P.R0) ** p
        H = g["Hg"]
        col = quad(lambda z: oracle.gas_at(P, R, z)["rhog"], -15 * H, 15 * H, limit=200)[0]
        h2 = g["hg"] ** 2
        assert 1.0 < col / Sig < 1.0 + 3.0 * h2, (R_au, col / Sig)


@pytest.mark.parametrize("p,q", [(-1.0, -1.0), (-1.5, -0.5), (-0.5, 0.0), (-2.0, 0.5)])
def test_hydrostatic_balance(p, q):
    P = _problem(p, q)

    def pressure(R, Z):
        g = oracle.gas_at(P, R, Z)
        return g["rhog"] * g["cs"] ** 2

    for R_au in (15.0, 40.0, 85.0):
        R = R_au * AU
        H = oracle.gas_at(P, R, 0.0)["Hg"]
        for zf in (0.0, 0.7, 2.0):
            Z = zf * H
            g = oracle.gas_at(P, R, Z)
            r = math.hypot(R, Z)
            dR = 1e-5 * R
            dPdR = (pressure(R + dR, Z) - pressure(R - dR, Z)) / (2 * dR)
            np.testing.assert_allclose(g["vgphi"] ** 2 / R, P.GM * R / r ** 3 + dPdR / g["rhog"], rtol=1e-8)
            if zf > 0:
                dZ = 1e-5 * H
                dPdZ = (pressure(R, Z + dZ) - pressure(R, Z - dZ)) / (2 * dZ)
                np.testing.assert_allclose(dPdZ / g["rhog"], -P.GM * Z / r ** 3, rtol=1e-7)


def test_epstein_scaling_of_the_stokes_number():
    # St = t_s Omega_K with t_s ~ rho_s s/(rho_g c_s): St rho_g c_s/Omega_K is the
    # same for every position
    P = _problem(-1.0, -1.0)
    vals = []
    for R_au in (11.0, 30.0, 95.0):
        R = R_au * AU
        for zf in (0.0, 1.0, 2.5):
            g = oracle.gas_at(P, R, zf * oracle.gas_at(P, R, 0.0)["Hg"])
            vals.append(g["stfac"] * g["rhog"] * g["cs"] / g["OmK"])
    np.testing.assert_allclose(vals, vals[0], rtol=1e-10)
