"""Flexion of a ray bundle, in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.
It shares no code with the product library.

Sec. 6 names flexion, the gradient of the shear and the third-order effect of
lensing, as the next use of ray bundles.  A bundle's ring carries it at second
order: with the offsets D_k = x_k - x_anchor of the eight ring rays at the
source plane (comoving, chi_s times the source-plane angle beta), the lens map
about the anchor reads

    beta(theta_c + d) - beta(theta_c) = A d + 1/2 Dm(d, d) + O(|d|^3),

d = r (cos 2 pi k / 8, sin 2 pi k / 8) for ring ray k, A the Jacobian of
eq. lensmap and Dm_ijl = d A_ij / d theta_l (symmetric in j, l).  The oracle
fits A (4 numbers) and Dm (6 numbers) to the 16 ring coordinates by linear
least squares.  With kappa, gamma1, gamma2 read from A as in the bundle
magnification (kappa = 1 - (A11 + A22) / 2, gamma1 = (A22 - A11) / 2,
gamma2 = -(A12 + A21) / 2), the first flexion is F = grad kappa and the second
G = (d1 gamma1 - d2 gamma2, d2 gamma1 + d1 gamma2) (complex d = d1 + i d2 applied
to gamma), both in rad^-1; for a lens potential psi, Dm_ijl = -psi_ijl and these
are the usual F = (psi_111 + psi_122, psi_112 + psi_222) / 2,
G = (psi_111 - 3 psi_122, 3 psi_112 - psi_222) / 2.
"""
from __future__ import annotations

import numpy as np

# Dm components, in output order
D_NAMES = ("D111", "D112", "D122", "D211", "D212", "D222")


def _design(radius: float) -> np.ndarray:
    """Least-squares matrix of the ring model for unknowns scaled to O(1):
    a_ij = A_ij r chi_s and m_i(jl) = Dm_ijl r^2 chi_s, in the order
    a11 a12 a21 a22 m111 m112 m122 m211 m212 m222; rows (k, i) = ring ray k, coordinate i."""
    M = np.zeros((16, 10))
    for k in range(8):
        c, s = np.cos(2 * np.pi * k / 8), np.sin(2 * np.pi * k / 8)
        for i in range(2):
            row = M[2 * k + i]
            row[2 * i + 0] = c
            row[2 * i + 1] = s
            row[4 + 3 * i + 0] = 0.5 * c * c
            row[4 + 3 * i + 1] = c * s          # Dm_i12 and Dm_i21 together
            row[4 + 3 * i + 2] = 0.5 * s * s
    return M


def bundle_flexion(chi_s: float, rays: np.ndarray, radius: float):
    """rays [8, 9 B] at the source plane (rows x, y are 1 and 2; ray 9 b is bundle b's anchor,
    9 b + 1 + k its ring ray k).  Returns (F [2, B], G [2, B], Dm [6, B] in D_NAMES order,
    A [4, B] = A11 A12 A21 A22)."""
    rays = np.asarray(rays, dtype=np.float64)
    nb = rays.shape[1] // 9
    M = _design(radius)
    F = np.zeros((2, nb))
    G = np.zeros((2, nb))
    Dm = np.zeros((6, nb))
    A = np.zeros((4, nb))
    for b in range(nb):
        x = rays[1, 9 * b: 9 * b + 9]
        y = rays[2, 9 * b: 9 * b + 9]
        rhs = np.empty(16)
        rhs[0::2] = x[1:] - x[0]
        rhs[1::2] = y[1:] - y[0]
        p, *_ = np.linalg.lstsq(M, rhs, rcond=None)
        A[:, b] = p[:4] / (radius * chi_s)
        d111, d112, d122, d211, d212, d222 = p[4:] / (radius * radius * chi_s)
        Dm[:, b] = (d111, d112, d122, d211, d212, d222)
        # kappa = 1 - (A11 + A22) / 2, gamma1 = (A22 - A11) / 2, gamma2 = -(A12 + A21) / 2,
        # differentiated along theta_1 and theta_2 (A_ij,l = Dm_ijl, Dm_ijl = Dm_ilj)
        dk = (-0.5 * (d111 + d212), -0.5 * (d112 + d222))
        dg1 = (0.5 * (d212 - d111), 0.5 * (d222 - d112))
        dg2 = (-0.5 * (d112 + d211), -0.5 * (d122 + d212))
        F[:, b] = dk
        G[:, b] = (dg1[0] - dg2[1], dg1[1] + dg2[0])
    return F, G, Dm, A
