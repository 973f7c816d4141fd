"""Particle-mesh field of Sec. 3.3 and the interpolation scheme of App. B, in plain
FP64 numpy.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.
It shares no code with the product library.

What is computed (isolated lenses, the zero-padded case of Sec. 3.3):

1. Cloud-in-Cell deposit of the particle masses onto the n^3 nodes
   x_ijk = origin + h (i, j, k) of a cubic grid (Sec. 3.3).  Mass whose cloud
   falls outside the grid is dropped.
2. The potential and its three derivatives at the nodes, by convolving the node
   masses with the Plummer kernels of eq. psi and eq. derivs on a grid
   zero-padded to (2n)^3, so that the FFT product is the exact linear
   convolution:  phi = -(G/c^2) sum_n' M_n' (d^2 + eps^2)^(-1/2) and
   dphi/dx = (G/c^2) sum_n' M_n' d_x (d^2 + eps^2)^(-3/2), d = x_n - x_n'.
   With eps = 0 the self term (d = 0) is left out.
3. App. B: natural cubic-spline second derivatives of each grid along the line
   of sight x^3, once per grid; at a point, (2 n_int)^2 spline evaluations along
   x^3, then 2 n_int local natural splines along x^1 through those values, then
   one local natural spline along x^2.  The local windows hold n_int nodes on
   each side of the point, shifted inwards at the grid's edges; outside the
   node range the field is zero.

Periodic boxes (the cosmological case of Sec. 3.3): the n^3 nodes tile a box of
side L = n h; the deposit wraps; the mean node mass is subtracted; the
potential solves Poisson's equation with the continuum Green's function,
phi_k = -4 pi (G/c^2) rho_k / k^2 (k = 0 removed), and dphi/dx_j has the
transform i k_j phi_k; the x^3 spline is the periodic cubic spline; App. B's
windows wrap around instead of shifting, and every point of space is inside.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from . import G_over_c2


def cic_deposit(xyz: np.ndarray, m: np.ndarray, origin, h: float, n: int) -> np.ndarray:
    """Node masses [n, n, n] (index order x^1, x^2, x^3) by Cloud-in-Cell (Sec. 3.3)."""
    u = (np.asarray(xyz, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) / h
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    grid = np.zeros((n, n, n))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                w = ((f[:, 0] if a else 1 - f[:, 0]) * (f[:, 1] if b else 1 - f[:, 1]) *
                     (f[:, 2] if c else 1 - f[:, 2]))
                idx = i0 + np.array([a, b, c])
                ok = np.all((idx >= 0) & (idx < n), axis=1)
                np.add.at(grid, (idx[ok, 0], idx[ok, 1], idx[ok, 2]), (m * w)[ok])
    return grid


def isolated_field(mass: np.ndarray, h: float, eps: float) -> np.ndarray:
    """[4, n, n, n]: phi, dphi/dx^1, dphi/dx^2, dphi/dx^3 at the nodes (eq. psi, derivs),
    by FFT convolution on the zero-padded (2n)^3 grid (Sec. 3.3)."""
    n = mass.shape[0]
    M = 2 * n
    G = G_over_c2()
    d = np.arange(M)
    d = np.where(d < n, d, d - M) * h           # displacement of padded index i (index n unused)
    dx, dy, dz = np.meshgrid(d, d, d, indexing="ij")
    r2 = dx * dx + dy * dy + dz * dz + eps * eps
    with np.errstate(divide="ignore"):
        k1 = np.where(r2 > 0, 1.0 / np.sqrt(r2), 0.0)
    k3 = k1 ** 3
    kernels = [-G * k1, G * dx * k3, G * dy * k3, G * dz * k3]
    padded = np.zeros((M, M, M))
    padded[:n, :n, :n] = mass
    fm = np.fft.fftn(padded)
    out = np.empty((4, n, n, n))
    for q, K in enumerate(kernels):
        out[q] = np.real(np.fft.ifftn(fm * np.fft.fftn(K)))[:n, :n, :n]
    return out


def spline_y2_line(y: np.ndarray, h: float) -> np.ndarray:
    """Natural cubic-spline second derivatives through equally spaced values y[..., k]
    (App. B; y2 = 0 at both ends, y2[k-1] + 4 y2[k] + y2[k+1] = 6 (y[k+1] - 2 y[k] + y[k-1]) / h^2)."""
    m = y.shape[-1]
    lead = y.shape[:-1]
    y2 = np.zeros_like(y)
    if m < 3:
        return y2
    rhs = 6.0 * (y[..., 2:] - 2.0 * y[..., 1:-1] + y[..., :-2]) / (h * h)
    ab = np.zeros((3, m - 2))
    ab[0, 1:] = 1.0
    ab[1, :] = 4.0
    ab[2, :-1] = 1.0
    sol = solve_banded((1, 1), ab, rhs.reshape(-1, m - 2).T)
    y2[..., 1:-1] = sol.T.reshape(lead + (m - 2,))
    return y2


def spline_eval(yk, yk1, y2k, y2k1, A, h):
    """Cubic spline between two nodes (App. B); A = (x_{k+1} - x) / h."""
    B = 1.0 - A
    return A * yk + B * yk1 + ((A ** 3 - A) * y2k + (B ** 3 - B) * y2k1) * (h * h) / 6.0


def z_second_derivatives(fields: np.ndarray, h: float) -> np.ndarray:
    """The once-per-grid spline of App. B along x^3, for each of the four grids."""
    return spline_y2_line(fields, h)


def _window(u: float, n: int, n_int: int):
    k = min(max(int(np.floor(u)), 0), n - 2)
    start = min(max(k - n_int + 1, 0), n - 2 * n_int)
    return np.arange(start, start + 2 * n_int)


def _local_spline(nodes: np.ndarray, vals: np.ndarray, u: float, h: float) -> float:
    """Natural cubic spline through vals at integer nodes (spacing h), evaluated at u."""
    y2 = spline_y2_line(vals, h)
    k = min(max(int(np.floor(u)) - nodes[0], 0), len(nodes) - 2)
    A = (nodes[0] + k + 1) - u
    return spline_eval(vals[k], vals[k + 1], y2[k], y2[k + 1], A, h)


def appb_eval(fields: np.ndarray, fields_y2z: np.ndarray, origin, h: float, n_int: int, p) -> np.ndarray:
    """The four grid quantities at point p by the scheme of App. B; zero outside the nodes."""
    n = fields.shape[1]
    u = (np.asarray(p, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) / h
    if np.any(u < 0) or np.any(u > n - 1):
        return np.zeros(4)
    wx, wy = _window(u[0], n, n_int), _window(u[1], n, n_int)
    kz = min(int(np.floor(u[2])), n - 2)
    Az = (kz + 1) - u[2]
    out = np.empty(4)
    for q in range(4):
        F, F2 = fields[q], fields_y2z[q]
        # step 1: along x^3 on the (2 n_int)^2 lines of the window
        v = np.empty((2 * n_int, 2 * n_int))
        for a, i in enumerate(wx):
            for b, j in enumerate(wy):
                v[a, b] = spline_eval(F[i, j, kz], F[i, j, kz + 1], F2[i, j, kz], F2[i, j, kz + 1], Az, h)
        # steps 2-3: local splines along x^1, one per x^2 node of the window
        w = np.array([_local_spline(wx, v[:, b], u[0], h) for b in range(2 * n_int)])
        # steps 4-5: one local spline along x^2
        out[q] = _local_spline(wy, w, u[1], h)
    return out


def cic_deposit_periodic(xyz: np.ndarray, m: np.ndarray, origin, h: float, n: int) -> np.ndarray:
    """Cloud-in-Cell on the n^3 nodes of a periodic box of side n h (Sec. 3.3)."""
    u = (np.asarray(xyz, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) / h
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    grid = np.zeros((n, n, n))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                w = ((f[:, 0] if a else 1 - f[:, 0]) * (f[:, 1] if b else 1 - f[:, 1]) *
                     (f[:, 2] if c else 1 - f[:, 2]))
                idx = np.mod(i0 + np.array([a, b, c]), n)
                np.add.at(grid, (idx[:, 0], idx[:, 1], idx[:, 2]), m * w)
    return grid


def periodic_field(mass: np.ndarray, h: float) -> np.ndarray:
    """[4, n, n, n]: phi and its gradient at the nodes of a periodic box: the density
    contrast (mean node mass removed) through the continuum Green's function of
    Poisson's equation, derivatives as i k_j (Sec. 3.3, eq. psi, derivs)."""
    n = mass.shape[0]
    G = G_over_c2()
    rho = (mass - mass.mean()) / h ** 3
    rk = np.fft.fftn(rho)
    k = 2 * np.pi * np.fft.fftfreq(n, d=h)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    with np.errstate(divide="ignore", invalid="ignore"):
        phik = np.where(k2 > 0, -4 * np.pi * G * rk / k2, 0.0)
    out = np.empty((4, n, n, n))
    out[0] = np.real(np.fft.ifftn(phik))
    for q, kq in enumerate((kx, ky, kz)):
        out[1 + q] = np.real(np.fft.ifftn(1j * kq * phik))
    return out


def spline_y2_periodic(y: np.ndarray, h: float) -> np.ndarray:
    """Periodic cubic-spline second derivatives along the last axis: the circulant
    system y2[k-1] + 4 y2[k] + y2[k+1] = 6 (y[k+1] - 2 y[k] + y[k-1]) / h^2, indices mod n."""
    from scipy.linalg import solve_circulant
    m = y.shape[-1]
    col = np.zeros(m)
    col[0], col[1], col[-1] = 4.0, 1.0, 1.0
    rhs = 6.0 * (np.roll(y, -1, axis=-1) - 2.0 * y + np.roll(y, 1, axis=-1)) / (h * h)
    flat = rhs.reshape(-1, m)
    sol = np.array([solve_circulant(col, r) for r in flat])
    return sol.reshape(y.shape)


def appb_eval_periodic(fields: np.ndarray, fields_y2z: np.ndarray, origin, h: float, n_int: int, p) -> np.ndarray:
    """App. B on a periodic grid: the point is wrapped into the box, the x^3 segment and the
    x^1, x^2 windows (n_int nodes on each side) are taken modulo n."""
    n = fields.shape[1]
    u = np.mod((np.asarray(p, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) / h, n)
    fl = np.floor(u).astype(np.int64)
    wx = fl[0] - n_int + 1 + np.arange(2 * n_int)
    wy = fl[1] - n_int + 1 + np.arange(2 * n_int)
    kz = fl[2]
    Az = (kz + 1) - u[2]
    out = np.empty(4)
    for q in range(4):
        F, F2 = fields[q], fields_y2z[q]
        v = np.empty((2 * n_int, 2 * n_int))
        for a, i in enumerate(wx % n):
            for b, j in enumerate(wy % n):
                v[a, b] = spline_eval(F[i, j, kz % n], F[i, j, (kz + 1) % n], F2[i, j, kz % n],
                                      F2[i, j, (kz + 1) % n], Az, h)
        w = np.array([_local_spline(wx, v[:, b], u[0], h) for b in range(2 * n_int)])
        out[q] = _local_spline(wy, w, u[1], h)
    return out


def pm_field(xyz, m, eps, origin, h, n, n_int, points):
    """phi [P] and grad [3, P] of the particle-mesh field at points [3, P]."""
    fields = isolated_field(cic_deposit(xyz, m, origin, h, n), h, eps)
    y2 = z_second_derivatives(fields, h)
    pts = np.asarray(points, dtype=np.float64)
    res = np.array([appb_eval(fields, y2, origin, h, n_int, pts[:, i]) for i in range(pts.shape[1])]).T
    return res[0], res[1:]


def trace_pm(c, nodes, rays, fields, fields_y2z, origin, h, n_int, step_begin=0, step_end=2 ** 31 - 1):
    """trace_pm_steps with one isolated grid used at every step."""
    grid = (fields, fields_y2z, origin, h, False)
    return trace_pm_steps(c, nodes, rays, [grid], np.zeros(len(nodes) - 1, dtype=np.int64), n_int, step_begin,
                          step_end)


def trace_pm_steps(c, nodes, rays, grids, step_grid, n_int, step_begin=0, step_end=2 ** 31 - 1):
    """Classical RK4 in z over the given nodes (Sec. 3.4 with x^3 as the independent
    variable); all four stages of step s take the field of grid step_grid[s] by App. B
    (none for -1).  grids: list of (fields [4,n,n,n], x^3 splines [4,n,n,n], origin, h,
    periodic).  Same flags as the direct oracle: 1 non-finite, 2 k^z <= 0 (both freeze the
    ray), 4 |phi|/a > 1e-2.  rays [8, R] are updated in place; returns (rays, flags)."""
    from . import derivs, scale_factor
    n_steps = len(nodes) - 1
    flags = np.zeros(rays.shape[1], dtype=np.uint8)
    for r in range(rays.shape[1]):
        Y = rays[[0, 1, 2, 4, 5, 6, 7], r].copy()
        z = rays[3, r]
        for s in range(step_begin, min(step_end, n_steps)):
            Z0, Z1 = nodes[s], nodes[s + 1]
            hs = Z1 - Z0
            gi = int(step_grid[s])

            def f(Yv, zz):
                if gi < 0:
                    q = np.zeros(4)
                else:
                    F, F2, org, hh, periodic = grids[gi]
                    ev = appb_eval_periodic if periodic else appb_eval
                    q = ev(F, F2, org, hh, n_int, [Yv[1], Yv[2], zz])
                return derivs(c, Yv, q[0], q[1:]), q[0]

            k1, phi0 = f(Y, Z0)
            if abs(phi0) / scale_factor(c, Y[0])[0] > 1e-2:
                flags[r] |= 4
            k2, _ = f(Y + 0.5 * hs * k1, Z0 + 0.5 * hs)
            k3, _ = f(Y + 0.5 * hs * k2, Z0 + 0.5 * hs)
            k4, _ = f(Y + hs * k3, Z1)
            Yn = Y + hs / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            if not np.all(np.isfinite(Yn)):
                flags[r] |= 1
                break
            if not Yn[6] > 0.0:
                flags[r] |= 2
                break
            Y, z = Yn, Z1
        rays[[0, 1, 2, 4, 5, 6, 7], r] = Y
        rays[3, r] = z
    return rays, flags


def trace_pm_lambda(c, chi_s, rays, fields, fields_y2z, origin, h, n_int, f_rk, max_steps):
    """trace_pm_lambda_slabs with one isolated grid as the field everywhere."""
    grid = (fields, fields_y2z, origin, h, False)
    return trace_pm_lambda_slabs(c, chi_s, rays, [grid], np.array([-np.inf, np.inf]), np.zeros(1, np.int64), h,
                                 n_int, f_rk, max_steps)


def slab_field(grids, bounds, slab_grid, n_int, p) -> np.ndarray:
    """(phi, grad) at p from the grid of the slab holding p[2]: bounds[k] <= p[2] < bounds[k + 1]
    takes grid slab_grid[k] (none for -1); zero outside [bounds[0], bounds[-1])."""
    z = p[2]
    if not (bounds[0] <= z < bounds[-1]):
        return np.zeros(4)
    k = int(np.searchsorted(bounds, z, side="right")) - 1
    gi = int(slab_grid[k])
    if gi < 0:
        return np.zeros(4)
    F, F2, org, hh, periodic = grids[gi]
    ev = appb_eval_periodic if periodic else appb_eval
    return ev(F, F2, org, hh, n_int, p)


def trace_pm_lambda_slabs(c, chi_s, rays, grids, bounds, slab_grid, h, n_int, f_rk, max_steps):
    """The paper's own integrator (Sec. 3.4, eq. RKstepsize): classical RK4 in the affine
    parameter with the fixed step  d_lambda = f_RK h / kz_0  (h: the Fourier-grid spacing,
    L_box / n_FFT; kz_0: the ray's dz/dlambda at the observer), repeated until z reaches chi_s;
    the step that overshoots is replaced by the linear interpolation between the previous and
    the current state at z = chi_s.  State (t, x, y, z, kt, kx, ky, kz), d/dlambda = (kt, kx,
    ky, kz, -A^t, -A^x, -A^y, -A^z) with the Christoffel contraction A of the z-form.

    The field at a point is looked up by its own x^3 (Sec. 5.2: the space between observer and
    source is filled by a stack of cubes along the line of sight, each with its own grid): the
    slabs bounds[k] <= x^3 < bounds[k + 1] take grid slab_grid[k] (none for -1), by App. B; a
    point outside [bounds[0], bounds[-1]) sees no field.  grids: list of (fields [4,n,n,n],
    x^3 splines [4,n,n,n], origin, h, periodic).
    Flags: 1 non-finite, 2 kz <= 0 (both freeze the ray), 4 |phi|/a > 1e-2, 8 chi_s not
    reached within max_steps.  rays [8, R] are updated in place; returns (rays, flags, steps)."""
    from . import accel, scale_factor
    bounds = np.asarray(bounds, dtype=np.float64)
    flags = np.zeros(rays.shape[1], dtype=np.uint8)
    steps = np.zeros(rays.shape[1], dtype=np.int64)

    def f(Y):
        q = slab_field(grids, bounds, slab_grid, n_int, Y[1:4])
        A = accel(c, Y[0], Y[4:8], q[0], q[1:])
        return np.concatenate([Y[4:8], -A]), q[0]

    for r in range(rays.shape[1]):
        Y = rays[:, r].copy()
        dl = f_rk * h / Y[7]
        done = not Y[3] < chi_s
        for s in range(0 if done else max_steps):
            k1, phi0 = f(Y)
            if abs(phi0) / scale_factor(c, Y[0])[0] > 1e-2:
                flags[r] |= 4
            k2, _ = f(Y + 0.5 * dl * k1)
            k3, _ = f(Y + 0.5 * dl * k2)
            k4, _ = f(Y + dl * k3)
            Yn = Y + dl / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            steps[r] = s + 1
            if not np.all(np.isfinite(Yn)):
                flags[r] |= 1
                done = True
                break
            if not Yn[7] > 0.0:
                flags[r] |= 2
                done = True
                break
            if Yn[3] >= chi_s:
                w = (chi_s - Y[3]) / (Yn[3] - Y[3])
                Y = Y + w * (Yn - Y)
                done = True
                break
            Y = Yn
        if not done:
            flags[r] |= 8
        rays[:, r] = Y
    return rays, flags, steps
