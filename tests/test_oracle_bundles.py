"""Pins of the oracle's bundle construction, magnification, Jacobian, source-
weighted PDF (Sec. 3.1, 5.3, eq. lensmap, magnification, weighthisto) and of
its step schedule."""
import math

import numpy as np
import pytest

import oracle as orc
from tests.oracle_run import oracle_fields
from paper_1110_4894_amd import workloads as wl

C0 = orc.cosmo(0.3, 0.7, 0.7)


def test_bundle_geometry_and_null_initial_wavevector():
    w = wl.empty(n_bundles=5)
    c, chi_s, fields, theta = oracle_fields(w)
    # put a mass near the observer so that phi_obs != 0
    fields[0].sets = [orc.ParticleSet(xyz=np.array([[0.01, 0.0, 0.02]]), m=np.array([1e15]), softening=0.001)]
    fields[0].step_set[:] = 0
    rb = 1e-3 * wl.ARCSEC
    rays = orc.build_bundles(c, fields, theta, rb)
    phi0, _ = orc.field_at(c, fields[0].sets[0], [0, 0, 0])
    assert abs(phi0) > 1e-9
    E0, F0 = 1 + 2 * phi0, 1 - 2 * phi0
    kt, kx, ky, kz = rays[4:8]
    assert np.all(rays[:4] == 0) and np.all(kt == 1)
    assert np.max(np.abs(-E0 * kt ** 2 + F0 * (kx ** 2 + ky ** 2 + kz ** 2))) < 1e-15
    # gnomonic directions: k_perp / kz = theta of each ray
    tx, ty = kx / kz, ky / kz
    for b in range(5):
        assert abs(tx[9 * b] - theta[0, b]) < 1e-18 and abs(ty[9 * b] - theta[1, b]) < 1e-18
        d = np.stack([tx[9 * b + 1: 9 * b + 9] - theta[0, b], ty[9 * b + 1: 9 * b + 9] - theta[1, b]])
        assert np.allclose(np.hypot(*d), rb, rtol=1e-9)
        ang = np.unwrap(np.arctan2(d[1], d[0]))
        assert np.allclose(np.diff(ang), math.pi / 4, atol=1e-6)     # counter-clockwise, regular
        assert abs(ang[0]) < 1e-6                                      # first ring ray along +x


def _rays_from_linear_map(A, theta, rb, chi_s, shift=(0.3, -0.2)):
    """Exit positions of an exactly linear lens map x = chi_s A theta + shift."""
    nb = theta.shape[1]
    rays = np.zeros((8, 9 * nb))
    ang = np.arange(8) * math.pi / 4
    for b in range(nb):
        pts = [theta[:, b]] + [theta[:, b] + rb * np.array([math.cos(a), math.sin(a)]) for a in ang]
        for k, p in enumerate(pts):
            x = chi_s * A @ p + np.asarray(shift)
            rays[1, 9 * b + k], rays[2, 9 * b + k] = x
            rays[3, 9 * b + k] = chi_s
    return rays


def test_magnification_and_jacobian_of_a_linear_map():
    """For an affine map both the polygon area and the least-squares Jacobian are exact:
    mu = 1 / det A and (kappa, gamma, omega) are recovered (eq. lensmap, magnification)."""
    rng = np.random.default_rng(5)
    chi_s, rb = 1888.6, 5e-9
    for _ in range(10):
        kap, g1, g2, om = rng.uniform(-0.3, 0.3, 4)
        A = np.array([[1 - kap - g1, -g2 - om], [-g2 + om, 1 - kap + g1]])
        theta = rng.uniform(-1e-3, 1e-3, (2, 3))
        rays = _rays_from_linear_map(A, theta, rb, chi_s)
        mu, jac = orc.magnification(chi_s, rays, rb)
        assert np.allclose(mu, 1 / np.linalg.det(A), rtol=1e-6)
        assert np.allclose(jac[:, 0], [kap, g1, g2, om], atol=1e-6)
    # parity flip gives negative mu
    A = np.diag([1.2, -0.5])
    rays = _rays_from_linear_map(A, np.zeros((2, 1)), rb, chi_s)
    mu, _ = orc.magnification(chi_s, rays, rb)
    assert mu[0] < 0 and abs(mu[0] * 1.2 * -0.5 - 1) < 1e-6


def test_magnification_is_source_area_ratio_brute_force():
    """mu equals the homogeneous-octagon area over the shoelace area of the traced octagon,
    computed here from the vertices with an independent polygon routine."""
    rng = np.random.default_rng(9)
    chi_s, rb = 1000.0, 1e-8
    rays = np.zeros((8, 9))
    ang = np.arange(8) * math.pi / 4
    rays[1, 0], rays[2, 0] = 0.1, 0.2
    pts = np.stack([np.cos(ang), np.sin(ang)], 1) * rb * chi_s * (1 + 0.2 * rng.random((8, 1)))
    rays[1, 1:] = 0.1 + pts[:, 0]
    rays[2, 1:] = 0.2 + pts[:, 1]
    mu, _ = orc.magnification(chi_s, rays, rb)
    area = 0.5 * abs(np.dot(pts[:, 0], np.roll(pts[:, 1], -1)) - np.dot(pts[:, 1], np.roll(pts[:, 0], -1)))
    hom = 8 * 0.5 * (rb * chi_s) ** 2 * math.sin(math.pi / 4)
    assert abs(mu[0] / (hom / area) - 1) < 1e-12


def test_mu_histogram_weights_and_moments():
    """eq. weighthisto: bundles weighted by 1/mu; weighted mean = N / sum(1/mu); a PDF over
    bins of width d mu whose integral is the in-range weight fraction."""
    rng = np.random.default_rng(1)
    mu = np.concatenate([np.exp(rng.normal(0.0, 0.05, 5000)), [-2.0, 0.0, 0.5, 5.0]])
    pdf, mom = orc.mu_histogram(mu, 200, -0.1, 0.3)
    pos = mu[mu > 0]
    assert mom[0] == pytest.approx(np.sum(1 / pos), rel=1e-12)
    assert mom[1] == pytest.approx(len(pos) / np.sum(1 / pos), rel=1e-12)
    w = 1 / pos
    var = np.sum(w * (pos - mom[1]) ** 2) / np.sum(w)
    assert mom[2] == pytest.approx(math.sqrt(var), rel=1e-10)
    assert mom[3] == 2 and mom[4] == np.sum(np.log10(pos) < -0.1) and mom[5] == np.sum(np.log10(pos) >= 0.3)
    edges = 10 ** np.linspace(-0.1, 0.3, 201)
    inrange = (np.log10(pos) >= -0.1) & (np.log10(pos) < 0.3)
    assert np.sum(pdf * np.diff(edges)) == pytest.approx(np.sum(w[inrange]) / np.sum(w), rel=1e-12)
    # a single magnification lands in the bin that contains it
    pdf1, _ = orc.mu_histogram(np.array([1.0]), 200, -0.1, 0.3)
    assert np.argmax(pdf1) == 50 and np.count_nonzero(pdf1) == 1


def test_schedule_structure():
    chi_s = 1888.6
    nodes = orc.make_schedule(chi_s, 1007.14, 1009.14, 1000, 1.1)
    assert nodes[0] == 0.0 and nodes[-1] == chi_s
    h = np.diff(nodes)
    assert np.all(h > 0)
    i0 = int(np.searchsorted(nodes, 1007.14))
    assert nodes[i0] == 1007.14 and nodes[i0 + 1000] == 1009.14
    assert np.allclose(h[i0:i0 + 1000], 0.002, rtol=1e-9)
    # outer steps grow by q away from the fine interval (except the merged end steps)
    up = h[i0 + 1000: -1]
    assert np.allclose(up[1:] / up[:-1], 1.1, rtol=1e-9)
    lo = h[1:i0][::-1]
    assert np.allclose(lo[1:] / lo[:-1], 1.1, rtol=1e-9)
    # the merged final steps lie between half and one and a half nominal steps
    assert 0.5 * 1.1 * up[-1] <= h[-1] <= 1.6 * 1.1 * up[-1]
    # uniform schedule
    u = orc.make_schedule(chi_s, 0.0, chi_s, 2000, 1.0)
    assert len(u) == 2001 and np.allclose(np.diff(u), chi_s / 2000, rtol=1e-10)


def test_replica_selection_by_midpoint():
    nodes = np.array([0.0, 4.0, 10.0, 10.5, 19.0, 20.0, 31.0])
    ss = orc.replica_step_sets(nodes, 10.0, 3)
    # midpoints 2, 7, 10.25, 14.75, 19.5, 25.5 -> replicas 0, 0, 1, 1, 1, 2
    assert list(ss) == [0, 0, 1, 1, 1, 2]
    # an exact tie (midpoint on a boundary) goes to the farther replica
    assert list(orc.replica_step_sets(np.array([0.0, 20.0]), 10.0, 3)) == [1]


def test_shear_histogram_against_numpy():
    """Source-weighted |gamma| histogram equals numpy's weighted histogram of hypot(g1, g2)."""
    rng = np.random.default_rng(12)
    n = 4000
    mu = np.exp(rng.normal(0, 0.05, n))
    mu[:3] = [-1.0, 0.0, 2.0]
    jac = rng.normal(0, 0.02, (4, n))
    pdf, mom = orc.shear_histogram(mu, jac, 50, 0.0, 0.08)
    ok = mu > 0
    g = np.hypot(jac[1], jac[2])[ok]
    w = 1 / mu[ok]
    h, edges = np.histogram(g, bins=50, range=(0.0, 0.08), weights=w)
    assert np.allclose(pdf, h / (w.sum() * np.diff(edges)), rtol=1e-12, atol=0)
    assert mom[0] == pytest.approx(w.sum(), rel=1e-13)
    assert mom[1] == pytest.approx(np.sum(w * g) / w.sum(), rel=1e-12)
    assert mom[2] == pytest.approx(math.sqrt(np.sum(w * (g - mom[1]) ** 2) / w.sum()), rel=1e-10)
    assert mom[3] == 2 and mom[5] == np.sum(g >= 0.08)
