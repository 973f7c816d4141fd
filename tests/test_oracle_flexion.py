"""Pins of the oracle's bundle flexion (Sec. 6: flexion, the gradient of the shear,
through ray bundles): exact maps of known derivatives, the thin-lens point mass in
closed form, and a traced point mass against it."""
import math

import numpy as np
import pytest

from oracle import flexion as ofx
from tests.oracle_run import oracle_run
from tests.test_oracle_geodesic import _point_mass_workload

RING = np.array([[math.cos(2 * math.pi * k / 8), math.sin(2 * math.pi * k / 8)] for k in range(8)])


def _rays_of_map(beta, centres, radius, chi_s):
    """Source-plane rays [8, 9 B] of the angular map beta at bundles centred on centres [B, 2]."""
    rays = np.zeros((8, 9 * len(centres)))
    for b, tc in enumerate(centres):
        for j, t in enumerate([tc] + [tc + radius * e for e in RING]):
            rays[1:3, 9 * b + j] = chi_s * beta(t)
    return rays


def test_fit_recovers_a_quadratic_map_and_ignores_cubic_terms():
    rng = np.random.default_rng(11)
    chi_s, r = 1500.0, 1e-5
    for trial in range(5):
        A = np.eye(2) + 0.1 * rng.normal(size=(2, 2))
        D = rng.normal(size=(2, 2, 2)) * 30.0
        D = 0.5 * (D + D.transpose(0, 2, 1))                     # symmetric in the last two indices
        C = rng.normal(size=(2, 2, 2, 2)) * 3e3 * (trial > 0)
        C = (C + C.transpose(0, 2, 3, 1) + C.transpose(0, 3, 1, 2)) / 3.0   # symmetric enough: only C(d,d,d) enters
        tc = rng.normal(size=2) * 1e-3

        def beta(t, A=A, D=D, C=C, tc=tc):
            d = t - tc
            return (A @ d + 0.5 * np.einsum("ijl,j,l->i", D, d, d) + np.einsum("ijlm,j,l,m->i", C, d, d, d) / 6.0)

        F, G, Dm, Af = ofx.bundle_flexion(chi_s, _rays_of_map(beta, [tc], r, chi_s), r)
        want = [D[0, 0, 0], D[0, 0, 1], D[0, 1, 1], D[1, 0, 0], D[1, 0, 1], D[1, 1, 1]]
        assert np.allclose(Dm[:, 0], want, rtol=0, atol=1e-6 * np.abs(D).max()), trial
        if trial == 0:
            assert np.allclose(Af[:, 0], A.ravel(), rtol=0, atol=1e-10)


def test_flexion_of_a_cubic_lens_potential():
    """beta = theta - grad psi with psi a cubic polynomial: Dm_ijl = -psi_ijl everywhere, and
    F = (psi_111 + psi_122, psi_112 + psi_222) / 2, G = (psi_111 - 3 psi_122, 3 psi_112 - psi_222) / 2."""
    p111, p112, p122, p222 = 40.0, -25.0, 10.0, 70.0
    p11, p12, p22 = 0.1, -0.05, 0.2

    def grad_psi(t):
        x, y = t
        # psi = p111 x^3/6 + p112 x^2 y/2 + p122 x y^2/2 + p222 y^3/6 + p11 x^2/2 + p12 x y + p22 y^2/2
        return np.array([p111 * x * x / 2 + p112 * x * y + p122 * y * y / 2 + p11 * x + p12 * y,
                         p112 * x * x / 2 + p122 * x * y + p222 * y * y / 2 + p12 * x + p22 * y])

    centres = np.array([[1e-3, -2e-3], [-4e-4, 5e-4]])
    F, G, Dm, A = ofx.bundle_flexion(900.0, _rays_of_map(lambda t: t - grad_psi(t), centres, 2e-6, 900.0), 2e-6)
    for b in range(2):
        assert np.allclose(F[:, b], [0.5 * (p111 + p122), 0.5 * (p112 + p222)], rtol=1e-7)
        assert np.allclose(G[:, b], [0.5 * (p111 - 3 * p122), 0.5 * (3 * p112 - p222)], rtol=1e-7)
        assert np.allclose(Dm[:, b], [-p111, -p112, -p122, -p112, -p122, -p222], rtol=1e-7)


@pytest.mark.parametrize("x", [1.2, 2.0, 5.0])
def test_thin_lens_point_mass(x):
    """psi = theta_E^2 ln|theta|: kappa = 0 off the lens, so F = 0, and gamma = -theta_E^2 / conj(theta)^2
    gives G = d gamma = 2 d/d conj(theta) gamma = 4 theta_E^2 / conj(theta)^3 (spin 3)."""
    th_e = 1.3e-5
    phis = np.array([0.0, 0.4, 2.0, -2.7])
    centres = x * th_e * np.stack([np.cos(phis), np.sin(phis)], axis=1)
    beta = lambda t: t - th_e ** 2 * t / (t @ t)
    F, G, Dm, A = ofx.bundle_flexion(2000.0, _rays_of_map(beta, centres, 1e-3 * th_e, 2000.0), 1e-3 * th_e)
    want = 4 / (x ** 3 * th_e) * np.stack([np.cos(3 * phis), np.sin(3 * phis)])
    assert np.max(np.abs(G - want)) < 1e-6 * np.abs(want).max()
    assert np.max(np.abs(F)) < 1e-6 * np.abs(want).max()


def test_traced_point_mass_flexion_is_the_thin_lens_value():
    """The oracle's own z-form trace through a point mass (Sec. 4.1 Schwarzschild lens), bundles of
    radius 0.01 theta_E: G within 1e-4 of 4 theta_E^2 / conj(theta)^3 and |F| below 1e-4 |G|,
    the thin-lens agreement level of the traced magnification."""
    xs = [1.2, 1.5, 2.0, 3.0, 5.0]
    w = _point_mass_workload([1.5])
    th_e = w.fields[0].meta["theta_E"]
    w = _point_mass_workload(xs, radius_arcsec=0.01 * th_e * 180 / math.pi * 3600)
    r = oracle_run(w)
    F, G, Dm, A = ofx.bundle_flexion(r["chi_s"], r["rays"], w.bundle_radius)
    th = r["theta"]
    tn, ph = np.linalg.norm(th, axis=0), np.arctan2(th[1], th[0])
    want = 4 * th_e ** 2 / tn ** 3 * np.stack([np.cos(3 * ph), np.sin(3 * ph)])
    err = np.hypot(*(G - want)) / np.hypot(*want)
    assert np.all(err < 1e-4), err
    assert np.all(np.hypot(*F) < 1e-4 * np.hypot(*want))


def test_rotating_map_flexion_is_the_gradient_of_kappa_and_gamma():
    """A map that is no gradient (Dm_ijl not symmetric in i, j): F and G are the derivatives of the
    kappa and gamma that the bundle magnification reads from A (kappa = 1 - tr A / 2,
    gamma1 = (A22 - A11) / 2, gamma2 = -(A12 + A21) / 2), taken here by central differences of the
    exact A(theta) = A0 + Dm (theta - theta_c)."""
    rng = np.random.default_rng(5)
    A0 = np.eye(2) + 0.05 * rng.normal(size=(2, 2))
    D = rng.normal(size=(2, 2, 2)) * 40.0
    D = 0.5 * (D + D.transpose(0, 2, 1))
    tc = np.array([3e-4, -1e-4])
    beta = lambda t: A0 @ (t - tc) + 0.5 * np.einsum("ijl,j,l->i", D, t - tc, t - tc)
    F, G, Dm, A = ofx.bundle_flexion(1000.0, _rays_of_map(beta, [tc], 1e-6, 1000.0), 1e-6)

    def kg(t):
        At = A0 + np.einsum("ijl,l->ij", D, t - tc)
        return np.array([1 - 0.5 * (At[0, 0] + At[1, 1]), 0.5 * (At[1, 1] - At[0, 0]), -0.5 * (At[0, 1] + At[1, 0])])

    h = 1e-7
    d1 = (kg(tc + [h, 0]) - kg(tc - [h, 0])) / (2 * h)
    d2 = (kg(tc + [0, h]) - kg(tc - [0, h])) / (2 * h)
    assert np.allclose(F[:, 0], [d1[0], d2[0]], rtol=1e-6, atol=1e-6)
    assert np.allclose(G[:, 0], [d1[1] - d2[2], d2[1] + d1[2]], rtol=1e-6, atol=1e-6)
