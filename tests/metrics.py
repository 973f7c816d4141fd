"""Error statistics of the measurement contract, shared by the GPU tests, the
smoke check and the benchmark.

Mixed-precision (or any) magnification against a reference: the relative error
|mu - mu_ref| / |mu_ref| for bundles with |mu_ref| <= 100, and the error of the
inverse, |1/mu - 1/mu_ref|, for the rest (near critical curves mu = 1/det A is
ill-conditioned and 1/mu is the well-conditioned quantity).  The gate at
tolerance tol is: relative error <= tol, and inverse error <= tol / 100 (the two
agree at |mu| = 100).
"""
from __future__ import annotations

import numpy as np

MU_BIG = 100.0


def mu_errors(mu, ref):
    """Per-bundle error in the gate's units: relative error for |ref| <= 100, and
    100 |d(1/mu)| beyond (equal to the relative error at |ref| = 100)."""
    mu, ref = np.asarray(mu, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    big = np.abs(ref) > MU_BIG
    err = np.abs(mu - ref) / np.abs(ref)
    err[big] = MU_BIG * np.abs(1.0 / mu[big] - 1.0 / ref[big])
    return err


def mu_stats(mu, ref):
    """max / p99 / p50 of the relative error over |ref| <= 100, the largest inverse
    error over |ref| > 100, and counts."""
    mu, ref = np.asarray(mu, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    big = np.abs(ref) > MU_BIG
    rel = np.abs(mu - ref) / np.abs(ref)
    r = rel[~big]
    q = lambda a, p: float(np.percentile(a, p)) if a.size else 0.0
    inv = np.abs(1.0 / mu[big] - 1.0 / ref[big])
    return {"max_rel": float(r.max()) if r.size else 0.0, "p99_rel": q(r, 99), "p50_rel": q(r, 50),
            "max_inv_big": float(inv.max()) if inv.size else 0.0, "n": int(mu.size), "n_big": int(big.sum()),
            "max_abs_mu": float(np.abs(ref).max()) if ref.size else 0.0}


def mu_gate(mu, ref, tol=1e-4):
    """True when every bundle meets the gate at tol."""
    return bool(np.all(mu_errors(mu, ref) <= tol))
