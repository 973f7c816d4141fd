"""Pins of the oracle's field of softened point masses and of the uniform-cuboid
background (Sec. 3.3, eq. psi, derivs, perturbation, meanmatterdens)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as orc

C0 = orc.cosmo(0.3, 0.7, 0.7)
G = orc.G_over_c2()


def _set(xyz, m, eps=0.0, bg=False, lo=(0, 0, 0), hi=(0, 0, 0)):
    return orc.ParticleSet(xyz=np.asarray(xyz, float), m=np.asarray(m, float), softening=eps, background=bg,
                           lo=lo, hi=hi)


def test_field_brute_force_extended_precision():
    """Direct sum against 40-digit mpmath on small random sets (with and without softening)."""
    rng = np.random.default_rng(7)
    mp.mp.dps = 40
    for n, eps in [(1, 0.0), (5, 0.01), (37, 0.003), (64, 0.0)]:
        xyz = rng.normal(size=(n, 3))
        m = rng.uniform(1e9, 1e12, n)
        p = rng.normal(size=3) * 0.5
        phi, g = orc.field_at(C0, _set(xyz, m, eps), p)
        sp = mp.mpf(0)
        sg = [mp.mpf(0)] * 3
        for j in range(n):
            d = [mp.mpf(p[i]) - mp.mpf(xyz[j, i]) for i in range(3)]
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mp.mpf(eps) ** 2
            sp += mp.mpf(m[j]) / mp.sqrt(r2)
            for i in range(3):
                sg[i] += mp.mpf(m[j]) * d[i] / r2 ** mp.mpf(1.5)
        ref_phi = -mp.mpf(G) * sp
        assert abs(phi - float(ref_phi)) <= 1e-14 * abs(float(ref_phi))
        gn = max(abs(float(v)) for v in sg) * G
        for i in range(3):
            assert abs(g[i] - float(mp.mpf(G) * sg[i])) <= 1e-14 * gn


def test_single_mass_closed_form_and_direction():
    """One mass: phi = -G m / sqrt(r^2 + eps^2), gradient points away from the mass."""
    m, eps = 3e12, 0.02
    x0 = np.array([0.1, -0.2, 5.0])
    p = np.array([0.4, 0.3, 5.5])
    phi, g = orc.field_at(C0, _set([x0], [m], eps), p)
    d = p - x0
    r2 = d @ d + eps * eps
    assert abs(phi / (-G * m / math.sqrt(r2)) - 1) < 1e-15
    assert np.allclose(g, G * m * d / r2 ** 1.5, rtol=1e-15, atol=0)
    assert g @ d > 0      # potential rises away from the mass


def test_superposition_and_gradient_consistency():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(20, 3)); b = rng.normal(size=(13, 3))
    ma = rng.uniform(1, 2, 20) * 1e11; mb = rng.uniform(1, 2, 13) * 1e11
    p = np.array([0.3, 0.1, -0.2])
    pa, ga = orc.field_at(C0, _set(a, ma, 0.05), p)
    pb, gb = orc.field_at(C0, _set(b, mb, 0.05), p)
    pab, gab = orc.field_at(C0, _set(np.vstack([a, b]), np.concatenate([ma, mb]), 0.05), p)
    assert abs(pab - (pa + pb)) < 1e-14 * abs(pab)
    assert np.allclose(gab, ga + gb, rtol=1e-13, atol=1e-14 * np.abs(gab).max())
    # gradient = derivative of the potential (central differences)
    h = 1e-5
    for i in range(3):
        e = np.zeros(3); e[i] = h
        fd = (orc.field_at(C0, _set(a, ma, 0.05), p + e)[0] - orc.field_at(C0, _set(a, ma, 0.05), p - e)[0]) / (2 * h)
        assert abs(fd - ga[i]) < 1e-7 * np.abs(ga).max()


def _cubature(lo, hi, p, n=48):
    """Gauss-Legendre product rule for U and grad U of a uniform cuboid (p outside it)."""
    x, w = np.polynomial.legendre.leggauss(n)
    pts = [0.5 * (hi[i] - lo[i]) * x + 0.5 * (hi[i] + lo[i]) for i in range(3)]
    wts = [0.5 * (hi[i] - lo[i]) * w for i in range(3)]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    W = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
    dx, dy, dz = p[0] - X, p[1] - Y, p[2] - Z
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    U = np.sum(W / r)
    g = np.array([-np.sum(W * d / r ** 3) for d in (dx, dy, dz)])
    return U, g


@pytest.mark.parametrize("p", [(3.0, 0.5, 0.2), (-1.7, 2.2, 0.9), (0.5, 0.5, 4.0), (2.5, -2.5, -1.5)])
def test_prism_against_cubature(p):
    lo, hi = (-1.0, -0.5, 0.0), (1.0, 0.5, 2.0)
    U, g = orc.prism(lo, hi, p)
    Uc, gc = _cubature(lo, hi, np.array(p))
    assert abs(U / Uc - 1) < 1e-10
    assert np.allclose(g, gc, rtol=1e-8, atol=1e-10 * np.abs(gc).max())


def test_prism_far_field_and_symmetry():
    lo, hi = (-1.0, -2.0, -0.5), (1.0, 2.0, 0.5)
    V = 2 * 4 * 1
    p = np.array([0.0, 0.0, 300.0])
    U, g = orc.prism(lo, hi, p)
    assert abs(U / (V / 300.0) - 1) < 1e-4
    assert abs(g[2] / (-V / 300.0 ** 2) - 1) < 1e-4
    # on the axis through the centre the transverse gradient vanishes by symmetry
    U, g = orc.prism(lo, hi, [0.0, 0.0, 0.2])
    assert abs(g[0]) < 1e-12 and abs(g[1]) < 1e-12


def test_prism_poisson_equation():
    """Laplacian of U is -4 pi inside the cuboid and 0 outside (central differences)."""
    lo, hi = (-1.0, -1.0, 0.0), (1.0, 1.0, 3.0)
    h = 1e-3
    for p, want in [((0.2, -0.3, 1.1), -4 * math.pi), ((2.0, 0.5, 1.0), 0.0), ((0.1, 0.1, -0.7), 0.0)]:
        p = np.array(p)
        lap = 0.0
        for i in range(3):
            e = np.zeros(3); e[i] = h
            lap += (orc.prism(lo, hi, p + e)[1][i] - orc.prism(lo, hi, p - e)[1][i]) / (2 * h)
        assert abs(lap - want) < 1e-5


def test_prism_on_face_is_continuous():
    """The observer sits on a face of the first box replica: U and grad U are finite
    and continuous there."""
    lo, hi = (-5.0, -5.0, 0.0), (5.0, 5.0, 10.0)
    U0, g0 = orc.prism(lo, hi, [0.0, 0.0, 0.0])
    U1, g1 = orc.prism(lo, hi, [0.0, 0.0, 1e-9])
    assert np.isfinite(U0) and np.all(np.isfinite(g0))
    assert abs(U0 - U1) < 1e-6 * U0 and np.allclose(g0, g1, rtol=1e-6, atol=1e-6)
    # corner and edge points
    for p in ([-5.0, -5.0, 0.0], [5.0, 0.0, 10.0], [-5.0, 2.0, 0.0]):
        U, g = orc.prism(lo, hi, p)
        assert np.isfinite(U) and np.all(np.isfinite(g))


def test_mean_density_subtraction_cancels_a_uniform_lattice():
    """A lattice of particles at the mean density minus the uniform cuboid leaves a
    field far smaller than either part (sign and normalisation of the background)."""
    n, L = 12, 10.0
    cell = L / n
    q = (np.arange(n) + 0.5) * cell - 0.5 * L
    X, Y, Z = np.meshgrid(q, q, q + 0.5 * L, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    rho = C0.omega_m * orc.rho_crit0(C0)
    m = np.full(len(xyz), rho * L ** 3 / n ** 3)
    eps = 0.3 * cell
    # a lattice vertex off the centre (between eight particles)
    p = np.array([3 * cell, -2 * cell, 0.5 * L + 2 * cell])
    phi_p, g_p = orc.field_at(C0, _set(xyz, m, eps), p)
    phi_t, g_t = orc.field_at(C0, _set(xyz, m, eps, True, (-L / 2, -L / 2, 0), (L / 2, L / 2, L)), p)
    assert np.linalg.norm(g_t) < 0.02 * np.linalg.norm(g_p)
    assert abs(phi_t) < 0.02 * abs(phi_p)
    # with the background added instead of subtracted the field would double
    U, gU = orc.prism((-L / 2, -L / 2, 0), (L / 2, L / 2, L), p)
    assert np.linalg.norm(g_p - G * rho * gU) > 1.5 * np.linalg.norm(g_p)
