"""Pins of the oracle's geodesic integration (Sec. 3.2, 3.4, App. A) and of the
lensing it produces (App. C, Sec. 3.1).

Christoffel symbols are re-derived symbolically from the metric; the z-form RK4
is checked against an independent adaptive integrator in the affine parameter,
against its own convergence order and invariant, and against the physics: the
point-mass deflection 4GM/(c^2 b), the Schwarzschild image magnification and
straight rays in an empty universe.
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy.integrate import solve_ivp

import oracle as orc
from paper_1110_4894_amd import workloads as wl
from tests.oracle_run import oracle_run, oracle_fields

C0 = orc.cosmo(0.3, 0.7, 0.7)
G = orc.G_over_c2()


# --------------------------------------------------------------------------- Christoffels
def _symbolic_accel():
    """A^alpha = Gamma^alpha_{beta gamma} k^beta k^gamma for eq. expandingmetric with
    psi = phi / a, differentiated by sympy."""
    t, x, y, z = sp.symbols("t x y z")
    A = sp.Function("a")(t)
    P = sp.Function("phi")(x, y, z)
    X = [t, x, y, z]
    g = sp.diag(-(1 + 2 * P / A), A ** 2 * (1 - 2 * P / A), A ** 2 * (1 - 2 * P / A), A ** 2 * (1 - 2 * P / A))
    ginv = g.inv()
    k = sp.symbols("k0:4")
    acc = []
    for al in range(4):
        s = 0
        for be in range(4):
            for ga in range(4):
                Gam = sum(ginv[al, de] * (sp.diff(g[de, ga], X[be]) + sp.diff(g[de, be], X[ga]) -
                                          sp.diff(g[be, ga], X[de])) for de in range(4)) / 2
                s += Gam * k[be] * k[ga]
        acc.append(s)
    av, adv, pv, gx, gy, gz = sp.symbols("av adv pv gx gy gz")
    subs = {sp.Derivative(A, t): adv, sp.Derivative(P, x): gx, sp.Derivative(P, y): gy, sp.Derivative(P, z): gz}
    out = []
    for e in acc:
        e = e.subs(subs).subs({A: av, P: pv})
        out.append(sp.lambdify((av, adv, pv, gx, gy, gz) + k, sp.simplify(e), "mpmath"))
    return out


def test_christoffel_contraction_matches_symbolic_metric():
    import mpmath as mp
    mp.mp.dps = 30
    fns = _symbolic_accel()
    rng = np.random.default_rng(11)
    for t in [0.0, 300.0, 1500.0]:
        a, adot = orc.scale_factor(C0, t)
        for _ in range(3):
            phi = rng.uniform(-1e-3, 1e-3)
            g = rng.normal(size=3) * 1e-3
            k = np.array([1.0, *(rng.normal(size=3) * 0.5)])
            got = orc.accel(C0, t, k, phi, g)
            for al in range(4):
                ref = float(fns[al](a, adot, phi, *g, *k))
                scale = abs(adot) * (k @ k) + np.abs(g).max() * (k @ k)
                assert abs(got[al] - ref) <= 1e-13 * scale


def test_first_order_appendix_symbol_differs_only_at_order_phi():
    """App. A prints Gamma^t_ij = adot (a + phi); the exact form is adot (a - phi) / (1 + 2 phi / a).
    With a point-like k = (1, 0, 0, 1) and g = 0 they differ by O(adot phi)."""
    a, adot = orc.scale_factor(C0, 100.0)
    phi = 1e-5
    At = orc.accel(C0, 100.0, [1.0, 0.0, 0.0, 1.0], phi, [0.0, 0.0, 0.0])[0]
    exact = (-adot * phi / a ** 2 + adot * (a - phi)) / (1 + 2 * phi / a)
    printed = -adot * phi / a ** 2 + adot * (a + phi)
    assert abs(At - exact) < 1e-15 * abs(exact)
    assert abs(At - printed) > 1e-6 * abs(adot) * phi


def test_z_derivative_is_the_reparametrised_geodesic():
    """dY/dz = (dY/dlambda) / kz for Y = (t, x, y, kt, kx, ky, kz)."""
    Y = np.array([120.0, 0.3, -0.1, 1.02, 1e-4, -2e-4, 0.98])
    g = np.array([1e-8, -2e-8, 3e-9])
    dY = orc.derivs(C0, Y, -1e-6, g)
    A = orc.accel(C0, Y[0], Y[3:], -1e-6, g)
    lam = np.array([Y[3], Y[4], Y[5], -A[0], -A[1], -A[2], -A[3]])
    assert np.allclose(dY, lam / Y[6], rtol=1e-15, atol=0)


# --------------------------------------------------------------------------- integrator
def _point_mass_workload(x_list, mass=1e12, eps=0.0, n_fine=1000, half=1.0, q=1.1, radius_arcsec=1e-3):
    w = wl.schwarzschild(n_radii=1, n_azimuth=1, mass=mass, n_fine=n_fine, half_width=half, q=q,
                         radius_arcsec=radius_arcsec)
    f = w.fields[0]
    th_e = f.meta["theta_E"]
    x = np.asarray(x_list, float)
    ang = 0.3 + 0.7 * np.arange(len(x))
    f.theta = np.stack([x * th_e * np.cos(ang), x * th_e * np.sin(ang)])
    f.meta["x"] = x
    f.sets[0].softening = eps
    return w


def _solve_lambda(c, pset, theta, chi_s):
    """Independent adaptive (DOP853) integration of the geodesic in the affine
    parameter, stopped where x^3 reaches chi_s."""
    tx, ty = theta
    n = np.array([tx, ty, 1.0]) / math.sqrt(tx * tx + ty * ty + 1)
    phi0, _ = orc.field_at(c, pset, [0.0, 0.0, 0.0])
    a0, _ = orc.scale_factor(c, 0.0)
    kk = n * math.sqrt((1 + 2 * phi0 / a0) / (a0 * a0 - 2 * a0 * phi0))
    y0 = np.array([0.0, 0.0, 0.0, 0.0, 1.0, *kk])

    def rhs(lam, y):
        phi, g = orc.field_at(c, pset, y[1:4])
        A = orc.accel(c, y[0], y[4:8], phi, g)
        return np.concatenate([y[4:8], -A])

    ev = lambda lam, y: y[3] - chi_s
    ev.terminal = True
    sol = solve_ivp(rhs, (0, 3 * chi_s), y0, method="DOP853", rtol=1e-12, atol=1e-14, events=ev,
                    first_step=1e-3, max_step=2.0)
    return sol.y_events[0][0]


def test_rk4_in_z_agrees_with_adaptive_lambda_integration():
    w = _point_mass_workload([1.5, 4.0], eps=0.003, n_fine=2000)
    r = oracle_run(w)
    c, chi_s, fields, theta = oracle_fields(w)
    pset = fields[0].sets[0]
    for b in range(2):
        ref = _solve_lambda(c, pset, theta[:, b], chi_s)
        i = 9 * b
        defl = math.hypot(r["rays"][1, i] - theta[0, b] * chi_s, r["rays"][2, i] - theta[1, b] * chi_s)
        assert abs(r["rays"][1, i] - ref[1]) < 1e-7 * defl
        assert abs(r["rays"][2, i] - ref[2]) < 1e-7 * defl
        # lookback time: limited by RK4 on the outer steps of up to ~90 Mpc
        assert abs(r["rays"][0, i] / ref[0] - 1) < 1e-8


def test_rk4_fourth_order_convergence():
    """Halving every step cuts the exit-position error by about 16."""
    def exit_pos(n_fine):
        w = _point_mass_workload([0.8], eps=0.004, n_fine=n_fine, half=0.05, q=1.2)
        return oracle_run(w)["rays"][1:3, 0]
    ref = exit_pos(1600)
    e1 = np.linalg.norm(exit_pos(25) - ref)
    e2 = np.linalg.norm(exit_pos(50) - ref)
    assert 13.0 < e1 / e2 < 19.0


def test_null_invariant_is_conserved():
    """g(k, k) = -E kt^2 + F |k|^2 stays 0 along the path (exact Christoffels)."""
    w = _point_mass_workload([0.7, 3.0])
    r = oracle_run(w)
    c = r["cosmo"]
    pset = r["fields"][0].sets[0]
    for i in range(r["rays"].shape[1]):
        t, x, y, z, kt, kx, ky, kz = r["rays"][:, i]
        a, _ = orc.scale_factor(c, t)
        phi, _ = orc.field_at(c, pset, [x, y, z])
        E = 1 + 2 * phi / a
        F = a * a - 2 * a * phi
        inv = -E * kt * kt + F * (kx * kx + ky * ky + kz * kz)
        assert abs(inv) < 1e-8 * kt * kt


def test_scale_factor_at_source_on_the_axis():
    """The axial ray reaches z = chi_s at lookback time t(z_s): a = 1/(1+z_s)."""
    w = wl.empty(n_bundles=1)
    w.fields[0].theta[:] = 0.0
    r = oracle_run(w)
    a, _ = orc.scale_factor(r["cosmo"], r["rays"][0, 0])
    assert abs(a * (1 + w.z_source) - 1) < 1e-8
    # the ring rays are 1e-3 arcsec off axis: same to 1e-15
    assert np.all(np.abs(r["rays"][3] - r["chi_s"]) == 0)


def test_empty_universe_straight_rays_and_unit_magnification():
    w = wl.empty(n_bundles=12)
    r = oracle_run(w)
    chi_s = r["chi_s"]
    th = r["theta"]
    rays = r["rays"]
    # anchor exit = theta * chi_s
    assert np.max(np.abs(rays[1, ::9] - th[0] * chi_s)) < 1e-12
    assert np.max(np.abs(rays[2, ::9] - th[1] * chi_s)) < 1e-12
    assert np.max(np.abs(r["mu"] - 1)) < 1e-8
    assert np.max(np.abs(r["jac"])) < 1e-8
    assert not r["flags"].any()


# --------------------------------------------------------------------------- physics
@pytest.mark.parametrize("x", [0.5, 1.0, 2.0, 5.0, 10.0])
def test_point_mass_deflection(x):
    """Total bending of the anchor ray is 4GM/(c^2 b) with b the physical impact
    parameter at the lens (comoving b / (1 + z_l))."""
    w = _point_mass_workload([x])
    r = oracle_run(w)
    f = w.fields[0]
    th = r["theta"][:, 0]
    kx, ky, kz = r["rays"][5:8, 0]
    dth = np.array([kx / kz, ky / kz]) - th
    chi_l = f.meta["chi_l"]
    # impact parameter from the ray's own transverse position at the lens node
    b_com = np.linalg.norm(th) * chi_l
    alpha = 4 * G * f.meta["mass"] / (b_com / (1 + f.meta["z_l"]))
    assert abs(np.linalg.norm(dth) / alpha - 1) < 1e-4
    # bending is towards the mass
    assert dth @ th < 0


def _mu_schw(x):
    return 1.0 / (1.0 - x ** -4)


def test_schwarzschild_magnification():
    """App. C, eq. schwmu: the image at x = theta / theta_E has mu = (1 - x^-4)^-1."""
    xs = np.array([0.5, 0.9, 1.1, 1.5, 2.0, 3.0, 5.0, 10.0])
    w = _point_mass_workload(xs)
    r = oracle_run(w)
    c = r["cosmo"]
    zl, zs = w.fields[0].meta["z_l"], w.z_source
    cl, cs = orc.comoving_distance(c, zl), r["chi_s"]
    th_e = math.sqrt(4 * G * 1e12 * (cs - cl) / (1 + zs) / (cl / (1 + zl) * cs / (1 + zs)))
    xv = np.linalg.norm(r["theta"], axis=0) / th_e
    for x, mu in zip(xv, r["mu"]):
        want = _mu_schw(x)
        if x >= 2.0:
            assert abs(mu / want - 1) < 1e-5, (x, mu, want)
        elif x > 1.2:
            assert abs(mu / want - 1) < 2e-4, (x, mu, want)
        else:
            inv_want = 1 - x ** -4
            assert abs(1 / mu - inv_want) < 3e-4 * max(1.0, abs(inv_want)), (x, mu, want)
    # parity flip inside the Einstein ring
    assert np.all(r["mu"][xv < 1] < 0) and np.all(r["mu"][xv > 1] > 0)


def test_schwarzschild_scale_invariance_and_isotropy():
    """mu depends only on x = theta / theta_E (scale invariance in the mass, Sec. 4.1)
    and not on the azimuth."""
    x = 2.5
    w1 = _point_mass_workload([x, x, x], mass=1e12)
    w2 = _point_mass_workload([x], mass=1e13)
    m1 = oracle_run(w1)["mu"]
    m2 = oracle_run(w2)["mu"]
    assert np.ptp(m1) < 1e-7
    assert abs(m1[0] / m2[0] - 1) < 2e-5
    # convergence is zero outside a point mass, shear = x^-2 (App. C, read with the exponent
    # that eq. schwmu and eq. magnification imply)
    r = oracle_run(w1)
    kap, g1, g2, om = r["jac"][:, 0]
    assert abs(kap) < 1e-4 * abs(math.hypot(g1, g2))
    assert abs(math.hypot(g1, g2) / x ** -2 - 1) < 1e-3
