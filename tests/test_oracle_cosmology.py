"""Pins of the oracle's background cosmology (Sec. 3.5, Sec. 5.1, App. E).

Each check compares the oracle with something other than itself: a special
case with a textbook solution, an independent quadrature or hypergeometric
closed form, or a value the paper prints (tests/golden/paper_values.json).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle as orc

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
ARCSEC = math.pi / 180 / 3600


def _c(p):
    return orc.cosmo(*p)


def test_scale_factor_is_one_today():
    """eq. scalefac2 with the square-root reading of eq. lookbacksingularity gives a(0) = 1."""
    for p in [(0.3, 0.7, 0.7), (0.27, 0.73, 0.71), (0.05, 0.95, 0.6)]:
        a, adot = orc.scale_factor(_c(p), 0.0)
        assert abs(a - 1.0) < 1e-13
        # Friedmann today: da/dt(lookback) = -H0
        assert abs(adot / orc.H0(_c(p)) + 1.0) < 1e-12


def test_literal_t0_fails_the_normalisation():
    """The literal eq. lookbacksingularity (no square root) does not give a(0) = 1:
    documents why the oracle reads it with the square root."""
    c = (0.3, 0.7, 0.7)
    H0 = orc.H0(_c(c))
    t0_lit = 2 / (3 * H0 * math.sqrt(0.7)) * math.asinh(0.7 / 0.3)
    a_lit = (0.3 / 0.7 * math.sinh(1.5 * math.sqrt(0.7) * H0 * t0_lit) ** 2) ** (1 / 3)
    assert abs(a_lit - 1.0) > 0.1


def test_scale_factor_matches_independent_lookback_integral():
    """a(t(z)) = 1/(1+z), with t(z) = int_0^z dz' / ((1+z') H(z')) by scipy quad."""
    for p in [(0.3, 0.7, 0.7), (0.27, 0.73, 0.71)]:
        c = _c(p)
        H0 = orc.H0(c)
        for z in [0.05, 0.25, 0.5, 1.0, 3.0]:
            t, _ = integrate.quad(lambda x: 1.0 / ((1 + x) * math.sqrt(p[0] * (1 + x) ** 3 + p[1])), 0, z,
                                  epsabs=0, epsrel=1e-13, limit=200)
            a, adot = orc.scale_factor(c, t / H0)
            assert abs(a * (1 + z) - 1.0) < 1e-11
            # and adot / a = -H(z)
            Hz = H0 * math.sqrt(p[0] * (1 + z) ** 3 + p[1])
            assert abs(adot / a / Hz + 1.0) < 1e-10


def test_scale_factor_einstein_de_sitter_limit():
    """For Omega_Lambda -> 0 eq. scalefac2 tends to the matter-only a = (1 - 3 H0 t / 2)^(2/3)."""
    c = _c((1.0 - 1e-9, 1e-9, 0.7))
    H0 = orc.H0(c)
    for t in [0.0, 0.1 / H0, 0.4 / H0]:
        a, _ = orc.scale_factor(c, t)
        assert abs(a / (1 - 1.5 * H0 * t) ** (2 / 3) - 1) < 1e-7


def _chi_hyp(p, z):
    """Closed form of int_0^z dz / sqrt(Om (1+z)^3 + OL) through 2F1(1/3, 1/2; 4/3; -x)."""
    om, ol, h = p
    def F(zz):
        u = (1 + zz)
        return u * special.hyp2f1(1 / 3, 1 / 2, 4 / 3, -om * u ** 3 / ol) / math.sqrt(ol)
    return (F(z) - F(0.0)) * 2997.92458 / h


def test_comoving_distance_hypergeometric():
    """eq. raytracedistance against its hypergeometric closed form."""
    for p in [(0.3, 0.7, 0.7), (0.27, 0.73, 0.71)]:
        for z in [0.1, 0.25, 0.5, 0.8, 2.0]:
            assert abs(orc.comoving_distance(_c(p), z) / _chi_hyp(p, z) - 1) < 1e-12


def test_hubble_parameter_and_critical_density():
    """H0 = 100 h km/s/Mpc and rho_c0 = 2.775e11 h^2 Msun/Mpc^3 (textbook value)."""
    c = _c((0.3, 0.7, 0.7))
    assert abs(orc.H0(c) * 299792.458 / 70.0 - 1) < 1e-15
    assert abs(orc.rho_crit0(c) / (0.49 * 2.7754e11) - 1) < 2e-4
    # G M_sun / c^2 = 1476.625 m
    assert abs(orc.G_over_c2() * 3.0856775814913673e22 / 1476.6250 - 1) < 1e-6


def test_empty_beam_distance_exceeds_full_beam():
    """App. E: D_eb > D_fb for z > 0, both -> z/H0 as z -> 0."""
    c = _c((0.3, 0.7, 0.7))
    for z in [0.1, 0.5, 1.0]:
        assert orc.empty_beam_distance(c, z) > orc.comoving_distance(c, z) / (1 + z)
    z = 1e-4
    assert abs(orc.empty_beam_distance(c, z) * orc.H0(c) / z - 1) < 1e-3
    # independent quadrature of eq. DRempty
    v, _ = integrate.quad(lambda x: 1 / ((1 + x) ** 2 * orc.E(c, x)), 0, 0.5, epsabs=0, epsrel=1e-13)
    assert abs(orc.empty_beam_distance(c, 0.5) * orc.H0(c) / v - 1) < 1e-12


def test_printed_minimum_magnification():
    g = GOLDEN["mu_fb_min_z05"]
    c = _c(g["cosmology"])
    z = g["z"]
    d_fb = orc.comoving_distance(c, z) / (1 + z)
    d_eb = orc.empty_beam_distance(c, z)
    assert abs((d_fb / d_eb) ** 2 / g["value"] - 1) < g["rel_tol"]


def test_printed_distances_and_patch():
    c = _c(GOLDEN["angular_diameter_distance_z05_mpc_h"]["cosmology"])
    h = c.h
    d_a = orc.comoving_distance(c, 0.5) / 1.5
    g = GOLDEN["angular_diameter_distance_z05_mpc_h"]
    assert abs(d_a * h / g["value"] - 1) < g["rel_tol"]
    g = GOLDEN["sampled_patch_deg"]
    ang = g["width_mpc_h"] / h / d_a * 180 / math.pi
    assert abs(ang / g["value"] - 1) < g["rel_tol"]
    g = GOLDEN["boxes_to_z05"]
    n = orc.comoving_distance(c, 0.5) * h / g["box_mpc_h"]
    assert abs(n - g["value"]) <= g["abs_tol"]


def test_printed_einstein_angle():
    """App. C eq. Eangle with the oracle's distances vs the printed 65.6 arcsec."""
    g = GOLDEN["einstein_angle_arcsec"]
    c = _c(g["cosmology"])
    cl, cs = orc.comoving_distance(c, g["z_l"]), orc.comoving_distance(c, g["z_s"])
    dd, ds, dds = cl / (1 + g["z_l"]), cs / (1 + g["z_s"]), (cs - cl) / (1 + g["z_s"])
    th = math.sqrt(4 * orc.G_over_c2() * g["mass_msun"] * dds / (dd * ds)) / ARCSEC
    assert abs(th / g["value"] - 1) < g["rel_tol"]


def test_printed_nfw_angular_extent():
    """Sec. 4.2: twice the virial radius (Delta = 200 rho_c(z)) of the 1e14 Msun halo is 343 arcsec."""
    g = GOLDEN["nfw_two_rvir_arcsec"]
    c = _c(g["cosmology"])
    rho = orc.rho_crit0(c) * orc.E(c, g["z_l"]) ** 2
    r200 = (3 * g["m_vir"] / (4 * math.pi * g["delta_c"] * rho)) ** (1 / 3)
    dd = orc.comoving_distance(c, g["z_l"]) / (1 + g["z_l"])
    assert abs(2 * r200 / dd / ARCSEC / g["value"] - 1) < g["rel_tol"]
