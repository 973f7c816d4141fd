"""Pins of the oracle's particle-mesh field (Sec. 3.3) and App. B interpolation."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle as orc
from oracle import pm


def test_cic_conserves_mass_and_centre_of_mass():
    """Linear CIC weights put a particle's mass on 8 nodes with its exact centre of mass."""
    rng = np.random.default_rng(3)
    n, h, origin = 12, 0.25, np.array([-1.0, 2.0, 10.0])
    xyz = origin + rng.uniform(0.5, n - 1.5, (200, 3)) * h
    m = rng.uniform(1.0, 5.0, 200)
    g = pm.cic_deposit(xyz, m, origin, h, n)
    assert g.sum() == pytest.approx(m.sum(), rel=1e-14)
    idx = np.indices((n, n, n)).reshape(3, -1).T * h + origin
    com = (g.reshape(-1)[:, None] * idx).sum(0) / g.sum()
    assert np.allclose(com, (m[:, None] * xyz).sum(0) / m.sum(), rtol=0, atol=1e-12)
    # a particle on a node deposits there only; one outside loses its mass
    g1 = pm.cic_deposit(np.array([origin + h * np.array([3, 4, 5])]), np.array([2.0]), origin, h, n)
    assert g1[3, 4, 5] == 2.0 and np.count_nonzero(g1) == 1
    g2 = pm.cic_deposit(np.array([origin - 5 * h]), np.array([2.0]), origin, h, n)
    assert g2.sum() == 0.0


@pytest.mark.parametrize("eps", [0.0, 0.07])
def test_isolated_field_is_the_direct_sum_over_node_masses(eps):
    """The zero-padded FFT convolution equals the brute-force Plummer sum over nodes."""
    rng = np.random.default_rng(1)
    n, h = 5, 0.3
    mass = rng.uniform(0.0, 1e12, (n, n, n)) * (rng.random((n, n, n)) < 0.4)
    f = pm.isolated_field(mass, h, eps)
    G = orc.G_over_c2()
    nodes = np.indices((n, n, n)).reshape(3, -1).T * h
    M = mass.reshape(-1)
    for t in rng.choice(n ** 3, 12, replace=False):
        d = nodes[t] - nodes
        r2 = (d * d).sum(1) + eps * eps
        keep = r2 > 0
        phi = -G * np.sum(M[keep] / np.sqrt(r2[keep]))
        grad = G * np.sum((M[keep] * r2[keep] ** -1.5)[:, None] * d[keep], axis=0)
        i, j, k = np.unravel_index(t, (n, n, n))
        scale = G * M.sum() / h
        assert abs(f[0, i, j, k] - phi) < 1e-12 * scale
        assert np.allclose(f[1:, i, j, k], grad, rtol=0, atol=1e-12 * scale / h)


def test_spline_second_derivatives_are_the_natural_spline():
    rng = np.random.default_rng(4)
    y = rng.normal(size=(3, 17))
    h = 0.4
    y2 = pm.spline_y2_line(y, h)
    x = np.arange(17) * h
    for r in range(3):
        assert np.allclose(y2[r], CubicSpline(x, y[r], bc_type="natural")(x, 2), rtol=0, atol=1e-10)


def _grid_of(fn, n, h, origin):
    i = np.arange(n) * h
    X, Y, Z = np.meshgrid(origin[0] + i, origin[1] + i, origin[2] + i, indexing="ij")
    return fn(X, Y, Z)


@pytest.mark.parametrize("n_int", [1, 2, 3])
def test_appb_exact_on_nodes_and_for_linear_fields(n_int):
    n, h, origin = 10, 0.5, np.array([1.0, -2.0, 3.0])
    lin = lambda X, Y, Z: 0.3 + 1.5 * X - 0.7 * Y + 2.0 * Z
    F = np.stack([_grid_of(lin, n, h, origin)] * 4)
    F2 = pm.z_second_derivatives(F, h)
    rng = np.random.default_rng(n_int)
    for _ in range(20):
        p = origin + rng.uniform(0, n - 1, 3) * h
        assert np.allclose(pm.appb_eval(F, F2, origin, h, n_int, p), lin(*p), rtol=0, atol=1e-12)
    G = np.stack([np.random.default_rng(9).normal(size=(n, n, n))] * 4)
    G2 = pm.z_second_derivatives(G, h)
    for ijk in [(0, 0, 0), (3, 4, 5), (9, 9, 9), (9, 0, 4)]:
        p = origin + h * np.array(ijk)
        assert np.allclose(pm.appb_eval(G, G2, origin, h, n_int, p), G[0][ijk], rtol=0, atol=1e-12)
    # outside the nodes the field is zero
    assert np.all(pm.appb_eval(G, G2, origin, h, n_int, origin - 0.1 * h) == 0)


def test_appb_reduces_to_one_dimensional_natural_splines():
    """A field varying along x^1 only is the local natural spline through the window's
    2 n_int nodes; one varying along x^3 only is the natural spline through the whole line."""
    n, h, origin = 12, 0.2, np.zeros(3)
    rng = np.random.default_rng(7)
    fx = rng.normal(size=n)
    fz = rng.normal(size=n)
    Fx = np.broadcast_to(fx[:, None, None], (n, n, n)).copy()
    Fz = np.broadcast_to(fz[None, None, :], (n, n, n)).copy()
    for n_int in (2, 3):
        for u in [0.3, 2.5, 5.7, 10.9]:
            p = np.array([u, 4.2, 6.6]) * h
            got = pm.appb_eval(np.stack([Fx] * 4), pm.z_second_derivatives(np.stack([Fx] * 4), h), origin, h,
                               n_int, p)[0]
            k = min(int(u), n - 2)
            start = min(max(k - n_int + 1, 0), n - 2 * n_int)
            nodes = np.arange(start, start + 2 * n_int)
            want = CubicSpline(nodes * h, fx[nodes], bc_type="natural")(u * h)
            assert got == pytest.approx(float(want), abs=1e-12)
            p = np.array([4.2, 6.6, u]) * h
            got = pm.appb_eval(np.stack([Fz] * 4), pm.z_second_derivatives(np.stack([Fz] * 4), h), origin, h,
                               n_int, p)[0]
            want = CubicSpline(np.arange(n) * h, fz, bc_type="natural")(u * h)
            assert got == pytest.approx(float(want), abs=1e-12)


def test_appb_converges_and_improves_with_n_int():
    """The local natural splines of App. B carry the O(h^2) end error of a natural spline
    into the window's centre, damped by about 0.27 per node: halving the spacing divides
    the error by ~4 (asymptotically), and every extra node per side lowers it."""
    fn = lambda X, Y, Z: np.sin(1.3 * X) * np.cos(0.9 * Y) * np.sin(0.7 * Z + 0.2)
    rng = np.random.default_rng(11)
    pts = rng.uniform(2.0, 3.0, (30, 3))
    errs = {}
    for n, h in [(51, 0.1), (101, 0.05)]:
        F = np.stack([_grid_of(fn, n, h, np.zeros(3))] * 4)
        F2 = pm.z_second_derivatives(F, h)
        for n_int in (1, 2, 3):
            errs[h, n_int] = max(abs(pm.appb_eval(F, F2, np.zeros(3), h, n_int, p)[0] - fn(*p)) for p in pts)
    for n_int in (1, 2, 3):
        assert 3.2 < errs[0.1, n_int] / errs[0.05, n_int] < 5.0
    assert errs[0.1, 1] > 3 * errs[0.1, 2] > 9 * errs[0.1, 3]


def test_pm_field_of_a_compact_cloud_far_away_is_the_direct_sum():
    """Outside a compact cloud the CIC smoothing is a small near-field effect: the PM field a
    few cells away agrees with the direct Plummer sum over the particles."""
    rng = np.random.default_rng(5)
    n, h = 32, 0.05
    origin = np.array([-0.8, -0.8, 99.2])
    xyz = np.array([0.0, 0.0, 100.0]) + rng.normal(size=(300, 3)) * 0.05
    m = np.full(300, 1e10)
    eps = 0.01
    pts = np.array([[0.45, 0.1, 100.2], [-0.5, -0.4, 99.7], [0.1, 0.52, 100.5]]).T
    phi, grad = pm.pm_field(xyz, m, eps, origin, h, n, 2, pts)
    s = orc.ParticleSet(xyz=xyz, m=m, softening=eps)
    c = orc.cosmo()
    for i in range(pts.shape[1]):
        p0, g0 = orc.field_at(c, s, pts[:, i])
        assert abs(phi[i] / p0 - 1) < 2e-3
        assert np.linalg.norm(grad[:, i] - g0) < 1e-2 * np.linalg.norm(g0)


def _empty_field_rays(c, theta, radius, nodes):
    f = orc.Field([], nodes, np.full(len(nodes) - 1, -1, np.int32), 0, theta.shape[1])
    return orc.build_bundles(c, [f], theta, radius)


def test_lambda_integrator_straight_rays_without_mass():
    """Sec. 3.4 integrator with no field: x/z stays constant along every ray, so the
    overshooting step's linear interpolation lands exactly on theta chi_s and mu = 1."""
    c = orc.cosmo()
    chi_s = orc.comoving_distance(c, 0.02)
    theta = np.array([[1e-3, -2e-3], [4e-4, 7e-4]])
    radius = 1e-3 * math.pi / 180 / 3600
    rays = _empty_field_rays(c, theta, radius, np.array([0.0, chi_s]))
    n, h = 8, 0.5
    F = np.zeros((4, n, n, n))
    out, flags, steps = pm.trace_pm_lambda(c, chi_s, rays.copy(), F, F, np.array([-2.0, -2.0, 10.0]), h, 2, 1.0,
                                           10 ** 6)
    assert not flags.any()
    assert np.all(np.abs(out[3] / chi_s - 1) < 1e-13)
    th = np.repeat(theta, 9, axis=1)
    ang = np.tile(np.concatenate([[0.0], np.arange(8) * math.pi / 4]), 2)
    ring = np.tile(np.concatenate([[0.0], np.ones(8)]), 2) * radius
    tx, ty = th[0] + ring * np.cos(ang), th[1] + ring * np.sin(ang)
    assert np.allclose(out[1], tx * chi_s, rtol=1e-11, atol=0)
    assert np.allclose(out[2], ty * chi_s, rtol=1e-11, atol=0)
    mu, _ = orc.magnification(chi_s, out, radius)
    assert np.all(np.abs(mu - 1) < 1e-6)
    # dz/dlambda grows towards the source (k scales with 1 + z), so a little fewer than
    # chi_s / (f_RK h) steps
    assert np.all((steps > chi_s / 0.5 / (1 + 0.03)) & (steps <= chi_s / 0.5 + 1))
    # null invariant E kt^2 - F |k|^2 with phi = 0 (E = 1, F = a^2)
    a = np.array([orc.scale_factor(c, t)[0] for t in out[0]])
    # (RK4 truncation of 0.5 Mpc steps and the interpolated last step: ~1e-8)
    assert np.max(np.abs(out[4] ** 2 - a * a * (out[5] ** 2 + out[6] ** 2 + out[7] ** 2)) / out[4] ** 2) < 5e-8


def test_lambda_integrator_converges_to_the_z_integrator():
    """Through the same particle-mesh field, the lambda-stepping integrator approaches the
    z-stepping one as f_RK shrinks.  The field stops at the grid's faces, and a fixed step
    straddles a face wherever it falls, so the convergence is first order with a constant that
    depends on that phase: only the overall decrease is pinned (Sec. 4.1 finds f_RK = 0.5
    sufficient)."""
    c = orc.cosmo()
    z_s = 0.02
    chi_s = orc.comoving_distance(c, z_s)
    chi_l = 0.5 * chi_s
    rng = np.random.default_rng(2)
    xyz = np.array([0.0, 0.0, chi_l]) + rng.normal(size=(200, 3)) * 0.02
    m = np.full(200, 5e11)
    n, h = 16, 0.02
    origin = np.array([-0.15, -0.15, chi_l - 0.15])
    F = pm.isolated_field(pm.cic_deposit(xyz, m, origin, h, n), h, 0.005)
    F2 = pm.z_second_derivatives(F, h)
    theta = np.array([[0.06 / chi_l], [0.02 / chi_l]])
    radius = 0.05 * math.pi / 180 / 3600
    nodes = orc.make_schedule(chi_s, origin[2], origin[2] + (n - 1) * h, 300, 1.02)
    ref, fl = pm.trace_pm(c, nodes, _empty_field_rays(c, theta, radius, nodes), F, F2, origin, h, 2)
    assert not fl.any()
    mu_ref, _ = orc.magnification(chi_s, ref, radius)
    defl = np.hypot(ref[1] - theta[0] * chi_s, ref[2] - theta[1] * chi_s)
    assert defl.min() > 1e-5                          # the rays are deflected
    errs = []
    for f_rk in (8.0, 0.5):
        out, flags, _ = pm.trace_pm_lambda(c, chi_s, _empty_field_rays(c, theta, radius, nodes), F, F2, origin, h,
                                           2, f_rk, 10 ** 6)
        assert not flags.any()
        mu, _ = orc.magnification(chi_s, out, radius)
        errs.append(max(np.max(np.hypot(out[1] - ref[1], out[2] - ref[2]) / defl), abs(mu[0] / mu_ref[0] - 1)))
    assert errs[1] < 1e-3
    assert errs[0] > 20 * errs[1]


def test_slab_lookup_takes_the_grid_of_the_slab_holding_the_point():
    """Sec. 5.2 stack of cubes along the line of sight: grid k holds the constant field k + 1
    (App. B reproduces constants exactly), so the looked-up value names the grid used."""
    n, h = 4, 1.0
    grids = []
    for k in range(3):
        F = np.full((4, n, n, n), k + 1.0)
        grids.append((F, np.zeros_like(F), np.array([-2.0, -2.0, 4.0 * k]), h, True))
    bounds = np.array([0.0, 4.0, 8.0, 12.0, 16.0])
    slab_grid = np.array([0, 2, -1, 1])
    want = {-1e-12: 0.0, 0.0: 1.0, 3.999: 1.0, 4.0: 3.0, 7.5: 3.0, 8.0: 0.0, 11.9: 0.0, 12.0: 2.0, 15.999: 2.0,
            16.0: 0.0, 1e3: 0.0}
    for z, v in want.items():
        got = pm.slab_field(grids, bounds, slab_grid, 2, np.array([0.3, -0.7, z]))
        assert np.all(got == v), (z, got)


def _smooth_periodic_grid(n, h, z0, amp, x0, y0):
    """A periodic grid holding phi = amp sin^2(pi (z - z0) / L) cos(k (x - x0)) cos(k (y - y0))
    (L = n h, k = 2 pi / L) and its gradient: zero with zero slope on the faces z = z0 + j L."""
    L = n * h
    origin = np.array([-0.5 * L, -0.5 * L, z0])
    u = np.arange(n) * h
    X, Y, Z = np.meshgrid(origin[0] + u, origin[1] + u, origin[2] + u, indexing="ij")
    k = 2 * np.pi / L
    sz, cx, cy = np.sin(np.pi * (Z - z0) / L) ** 2, np.cos(k * (X - x0)), np.cos(k * (Y - y0))
    F = np.array([amp * sz * cx * cy, -amp * k * sz * np.sin(k * (X - x0)) * cy,
                  -amp * k * sz * cx * np.sin(k * (Y - y0)),
                  amp * np.pi / L * np.sin(2 * np.pi * (Z - z0) / L) * cx * cy])
    return (F, pm.spline_y2_periodic(F, h), origin, h, True)


def test_lambda_integrator_through_a_stack_of_slabs_converges_to_the_z_integrator():
    """Two adjacent periodic cubes of different fields, each looked up only inside its own
    slab (Sec. 5.2), traced by the lambda-stepping RK4 (Sec. 3.4, eq. RKstepsize) and by the
    z-stepping RK4 with nodes on the slab faces (where its step-midpoint choice of grid is the
    per-point choice exactly).  The fields vanish with zero slope on the faces, so the lambda
    steps that straddle a face cost little and the two converge as f_RK shrinks; a lookup that
    misplaced the faces by half a grid spacing, or took the wrong grid, would miss by 1e-3
    and 1e-1 of the deflection."""
    c = orc.cosmo()
    chi_s = orc.comoving_distance(c, 0.02)
    n, h = 8, 0.5
    grids = [_smooth_periodic_grid(n, h, 20.0, 3e-6, 0.3, -0.2), _smooth_periodic_grid(n, h, 24.0, -2e-6, -0.5, 0.9)]
    bounds = np.array([20.0, 24.0, 28.0])
    theta = np.array([[0.02], [0.015]])
    radius = 0.05 * math.pi / 180 / 3600
    nodes = np.concatenate([np.linspace(0, 20, 21)[:-1], np.linspace(20, 28, 161)[:-1], np.linspace(28, chi_s, 41)])
    mid = 0.5 * (nodes[1:] + nodes[:-1])
    step_grid = np.where((mid >= 20) & (mid < 24), 0, np.where((mid >= 24) & (mid < 28), 1, -1))
    ref, fl = pm.trace_pm_steps(c, nodes, _empty_field_rays(c, theta, radius, nodes), grids, step_grid, 2)
    assert not fl.any()
    mu_ref, _ = orc.magnification(chi_s, ref, radius)
    defl = np.hypot(ref[1] - np.repeat(theta[0], 9) * chi_s, ref[2] - np.repeat(theta[1], 9) * chi_s)
    assert defl.min() > 5e-4                           # the rays are deflected
    errs = []
    for f_rk in (2.0, 0.25):
        out, flags, steps = pm.trace_pm_lambda_slabs(c, chi_s, _empty_field_rays(c, theta, radius, nodes), grids,
                                                     bounds, np.array([0, 1]), h, 2, f_rk, 10 ** 6)
        assert not flags.any()
        assert np.all(np.abs(out[3] / chi_s - 1) < 1e-13)
        mu, _ = orc.magnification(chi_s, out, radius)
        errs.append(max(np.max(np.hypot(out[1] - ref[1], out[2] - ref[2]) / defl), abs(mu[0] / mu_ref[0] - 1)))
    assert errs[1] < 2e-5
    assert errs[0] > 10 * errs[1]


def test_periodic_deposit_wraps_and_conserves_mass():
    n, h, origin = 8, 0.5, np.zeros(3)
    rng = np.random.default_rng(8)
    xyz = rng.uniform(-2.0, 6.0, (300, 3))                 # also outside the first period
    m = rng.uniform(1, 2, 300)
    g = pm.cic_deposit_periodic(xyz, m, origin, h, n)
    assert g.sum() == pytest.approx(m.sum(), rel=1e-14)
    # a particle half a cell below the upper face shares its mass with node 0 (wrap)
    g1 = pm.cic_deposit_periodic(np.array([[3.75, 0.0, 0.0]]), np.array([2.0]), origin, h, n)
    assert g1[7, 0, 0] == 1.0 and g1[0, 0, 0] == 1.0
    # shifting every particle by one period changes nothing
    g2 = pm.cic_deposit_periodic(xyz + np.array([4.0, -4.0, 8.0]), m, origin, h, n)
    assert np.allclose(g2, g, rtol=0, atol=1e-12)


def test_periodic_field_of_a_single_mode_is_the_poisson_solution():
    """Node masses M0 (1 + A cos(k x)): phi = -4 pi G A (M0 / h^3) cos(k x) / k^2 and
    dphi/dx = 4 pi G A (M0 / h^3) sin(k x) / k, exactly on the nodes; no mean term."""
    n, h = 16, 0.25
    L = n * h
    x = np.arange(n) * h
    for mode, A in [(1, 0.3), (3, -0.1)]:
        k = 2 * np.pi * mode / L
        M0 = 1e11
        mass = np.broadcast_to((M0 * (1 + A * np.cos(k * x)))[:, None, None], (n, n, n)).copy()
        f = pm.periodic_field(mass, h)
        G = orc.G_over_c2()
        amp = 4 * np.pi * G * A * M0 / h ** 3
        tol = 1e-12 * abs(amp)
        assert np.allclose(f[0][:, 3, 5], -amp * np.cos(k * x) / k ** 2, rtol=0, atol=tol / k ** 2)
        assert np.allclose(f[1][:, 3, 5], amp * np.sin(k * x) / k, rtol=0, atol=tol / k)
        assert np.max(np.abs(f[2])) < tol / k and np.max(np.abs(f[3])) < tol / k
    rng = np.random.default_rng(3)
    f = pm.periodic_field(rng.uniform(0, 1e10, (n, n, n)), h)
    assert abs(f[0].mean()) < 1e-12 * np.abs(f[0]).max()


def test_periodic_spline_is_scipys_periodic_spline():
    rng = np.random.default_rng(5)
    y = rng.normal(size=(2, 12))
    h = 0.3
    y2 = pm.spline_y2_periodic(y, h)
    x = np.arange(13) * h
    for r in range(2):
        cs = CubicSpline(x, np.append(y[r], y[r][0]), bc_type="periodic")
        assert np.allclose(y2[r], cs(x[:-1], 2), rtol=0, atol=1e-10)


def test_periodic_appb_wraps_and_is_exact_on_nodes():
    n, h, origin = 12, 0.25, np.array([-1.5, -1.5, 40.0])
    rng = np.random.default_rng(6)
    F = np.stack([rng.normal(size=(n, n, n)) for _ in range(4)])
    F2 = pm.spline_y2_periodic(F, h)
    for n_int in (1, 2, 3):
        for ijk in [(0, 0, 0), (11, 5, 11), (3, 0, 7)]:
            p = origin + h * np.array(ijk)
            assert np.allclose(pm.appb_eval_periodic(F, F2, origin, h, n_int, p), F[(slice(None),) + ijk],
                               rtol=0, atol=1e-12)
        for _ in range(5):
            p = origin + rng.uniform(0, n, 3) * h
            a = pm.appb_eval_periodic(F, F2, origin, h, n_int, p)
            b = pm.appb_eval_periodic(F, F2, origin, h, n_int, p + n * h * np.array([1, -2, 3]))
            assert np.allclose(a, b, rtol=0, atol=1e-12)
    # a smooth periodic field is interpolated to second order
    L = n * h
    fn = lambda X, Y, Z: np.sin(2 * np.pi * (X - origin[0]) / L) * np.cos(2 * np.pi * (Z - origin[2]) / L)
    errs = []
    for nn in (16, 32):
        hh = L / nn
        G = np.stack([_grid_of(fn, nn, hh, origin)] * 4)
        G2 = pm.spline_y2_periodic(G, hh)
        pts = origin + np.random.default_rng(1).uniform(0, L, (20, 3))
        errs.append(max(abs(pm.appb_eval_periodic(G, G2, origin, hh, 2, q)[0] - fn(*q)) for q in pts))
    assert 3.2 < errs[0] / errs[1] < 20
