"""Parity at the workloads' full sizes (full particle sets and full RK4
schedules), on sampled bundles that the CPU oracle traces one by one.

* point lens (32 x 32 bundles, 1225 steps): every bundle against the oracle (FP64
  and mixed), the Schwarzschild magnification, and mixed against GPU FP64;
* NFW halo (1e5 particles, 2236 steps): the 7168-bundle band through the halo
  centre, mixed against GPU FP64 on every bundle, 16 bundles against the oracle;
* Zel'dovich boxes (2^18 and 2^20 particles in 14 replicas, 2000 steps, 1e-3
  arcsec bundles): mixed against GPU FP64 on 1024 / 504 bundles, the oracle on
  one or two;
* 64 uneven fields in one launch (bundle grids reduced to 8 x 8 per field):
  mixed against FP64 over every bundle and the oracle on one bundle of several fields;
* the largest sets: the field of a 7.2e8-particle set (offsets beyond 2^31 elements).
Tolerances as in test_gpu_parity.py; mixed against FP64 is the measurement gate at
1e-4 (relative mu error for |mu| <= 100, |d(1/mu)| <= 1e-6 beyond).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from paper_1110_4894_amd import rt
from paper_1110_4894_amd import workloads as wl
from tests.oracle_run import oracle_run
from tests.metrics import mu_errors
from tests.test_gpu_parity import _check_fp32, _check_fp64

pytestmark = pytest.mark.gpu

FP64, FP32K = rt.RT_FP64, rt.RT_FP32_KAHAN


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def _with_theta(w, theta_per_field):
    fields = [wl.FieldSpec(f.name, f.sets, np.ascontiguousarray(th), f.schedule, f.replica_box, dict(f.meta))
              for f, th in zip(w.fields, theta_per_field)]
    return wl.Workload(w.name, w.cosmology, w.z_source, w.bundle_radius, fields, dict(w.meta))


def _say(msg):
    print("    [fullsize] %s" % msg, flush=True)


def _oracle(w):
    _say("oracle: %d bundles" % w.n_bundles)
    o = oracle_run(w)
    _say("oracle done")
    return o


def _gpu_run(w, prec, tune=False):
    from paper_1110_4894_amd.runner import GpuRun
    _say("gpu %s: %d bundles" % ("fp64" if prec == FP64 else "fp32k", w.n_bundles))
    g = GpuRun(w)
    if tune:
        g.build_bundles()
        rt.rt_autotune(g.cosmo, w.z_source, g.table, prec, g.max_steps // 2, 6, g.n_bundles, g.rays)
    out = g.run(prec)
    _say("gpu done")
    return out


def _sub(g, idx):
    """The bundles idx of a GpuRun result."""
    idx = np.asarray(idx)
    r = (9 * idx[:, None] + np.arange(9)).ravel()
    out = {"mu": g["mu"][idx], "flags": g["flags"][r], "rays": g["rays"][:, r], "chi_s": g["chi_s"]}
    if "jac" in g:
        out["jac"] = g["jac"][:, idx]
    return out


def _mixed_vs_fp64(g32, g64, what):
    err = mu_errors(g32["mu"], g64["mu"])
    _say("%s: mixed vs FP64 over %d bundles: max %.3e, p99 %.3e (|mu| <= %.2f)"
         % (what, err.size, err.max(), np.percentile(err, 99), np.abs(g64["mu"]).max()))
    assert np.array_equal(g32["flags"], g64["flags"])
    assert err.max() <= 1e-4, what


def test_point_lens_full():
    w = wl.schwarzschild()
    o = _oracle(w)
    g = _gpu_run(w, FP64)
    _check_fp64(g, o, o["theta"])
    x = w.fields[0].meta["x"]
    want = 1 / (1 - x ** -4)
    far = x >= 2
    assert np.max(np.abs(g["mu"][far] / want[far] - 1)) < 1e-5
    near = x <= 1.1
    assert np.all(np.abs(1 / g["mu"][near] - (1 - x[near] ** -4)) < 3e-4 * np.maximum(1, np.abs(1 - x[near] ** -4)))
    # mixed precision: every bundle against the oracle and the GPU FP64 run
    g32 = _gpu_run(w, FP32K)
    _check_fp32(g32, o, o["theta"])
    _mixed_vs_fp64(g32, g, "point lens")


def test_nfw_central_band_as_benchmarked():
    """The band of 7168 bundles through the halo centre (rows 114-141 of the 256 x 256 grid),
    traced as bench.py traces a band (FP32 pair terms, autotuned plan): every bundle against
    the GPU FP64 run, and 16 bundles (the most magnified and a spread of others) against the
    oracle in both precisions."""
    w = wl.nfw()
    f = w.fields[0]
    band = 7168
    start = 128 * 256 - band // 2
    th = f.theta[:, start:start + band]
    wb = _with_theta(w, [th])
    g32 = _gpu_run(wb, FP32K, tune=True)
    g64 = _gpu_run(wb, FP64)
    _mixed_vs_fp64(g32, g64, "NFW central band")
    assert np.abs(g64["mu"]).max() > 3                  # the band holds the strongly lensed core
    order = np.argsort(-np.abs(g64["mu"]))
    sample = np.unique(np.concatenate([order[:8], np.linspace(0, band - 1, 8).astype(int)]))
    ws = _with_theta(w, [th[:, sample]])
    o = _oracle(ws)
    _check_fp32(_sub(g32, sample), o, o["theta"])
    _check_fp64(_sub(g64, sample), o, o["theta"])


@pytest.mark.parametrize("log2n,n_side", [(18, 128), (20, 512)])
def test_box_full(log2n, n_side):
    """Zel'dovich boxes with 1e-3 arcsec bundles through all 14 replicas: mixed vs GPU FP64 on
    1024 bundles (8 central rows) of the 2^18 box and 504 bundles spread over the 512 x 512
    grid of the 2^20 box, and one or two bundles against the oracle."""
    _say("building the 2^%d box" % log2n)
    w = wl.box(n_part_log2=log2n, n_side=n_side)
    f = w.fields[0]
    if log2n == 18:
        mid = n_side // 2
        th = f.theta[:, (mid - 4) * n_side: (mid + 4) * n_side]
        sample = np.array([3, th.shape[1] // 2 + 7])
    else:
        th = f.theta[:, ::f.n_bundles // 504][:, :504]
        sample = np.array([250])
    wb = _with_theta(w, [th])
    g32 = _gpu_run(wb, FP32K)
    g64 = _gpu_run(wb, FP64)
    _mixed_vs_fp64(g32, g64, "box 2^%d" % log2n)
    ws = _with_theta(w, [th[:, sample]])
    o = _oracle(ws)
    _check_fp32(_sub(g32, sample), o, o["theta"])
    _check_fp64(_sub(g64, sample), o, o["theta"])
    # mean-density subtraction keeps the box weakly lensing
    assert np.all(np.abs(g64["mu"] - 1) < 0.5)


def test_uneven_fields_one_launch():
    _say("building the 64 fields")
    w = wl.batched(side_override=8)
    g32 = _gpu_run(w, FP32K)
    info = rt.rt_last_trace_info()
    assert info["n_items"] >= 64
    g64 = _gpu_run(w, FP64)
    _mixed_vs_fp64(g32, g64, "64 uneven fields")
    # oracle on one bundle of a few fields of each kind (the cheaper ones)
    order = {"points": [], "nfw": [], "box": []}
    for i, f in enumerate(w.fields):
        order[f.meta["kind"]].append((sum(len(s.m) for s in f.sets), i))
    chosen = [i for k in order for _, i in sorted(order[k])[:2]]
    off = np.cumsum([0] + [f.n_bundles for f in w.fields])
    keep = [off[i] + 27 for i in chosen]
    ws = wl.Workload(w.name, w.cosmology, w.z_source, w.bundle_radius,
                     [wl.FieldSpec(w.fields[i].name, w.fields[i].sets,
                                   np.ascontiguousarray(w.fields[i].theta[:, 27:28]),
                                   w.fields[i].schedule, w.fields[i].replica_box, {}) for i in chosen])
    o = _oracle(ws)
    keep = np.array(keep)
    rays_idx = (9 * keep[:, None] + np.arange(9)).ravel()
    sub64 = {"mu": g64["mu"][keep], "flags": g64["flags"][rays_idx], "rays": g64["rays"][:, rays_idx],
             "jac": g64["jac"][:, keep], "chi_s": g64["chi_s"]}
    _check_fp64(sub64, o, o["theta"])
    sub32 = {"mu": g32["mu"][keep], "flags": g32["flags"][rays_idx], "rays": g32["rays"][:, rays_idx],
             "chi_s": g32["chi_s"]}
    _check_fp32(sub32, o, o["theta"])


def test_set_beyond_32bit_offsets():
    """The largest sets: 7.2e8 particles, so that the z and mass columns of the caller's
    [4][n] array start beyond 2^31 elements.  The last 1000 particles carry mass and the rest
    none (their terms are exactly zero in either precision), so the oracle sums the massive
    ones only; the field at 63 points against it, FP64 and FP32."""
    n, k = 720_000_000, 1000
    assert 3 * n > 2 ** 31
    rng = np.random.default_rng(np.random.SeedSequence(wl.MASTER_SEED + 7))
    xyz = rng.normal(size=(k, 3)) * 0.3 + np.array([0.1, -0.2, 1000.0])
    m = rng.uniform(1e9, 1e11, k)
    pts = rng.normal(size=(3, 63)) * 0.2 + np.array([[0.0], [0.0], [1000.0]])
    eps = 0.01
    c = orc.cosmo()
    ps = orc.ParticleSet(xyz=xyz, m=m, softening=eps)
    ref_phi = np.zeros(63)
    ref_g = np.zeros((3, 63))
    for i in range(63):
        ref_phi[i], ref_g[:, i] = orc.field_at(c, ps, pts[:, i])
    dev = torch.device("cuda")
    _say("allocating a [4][%d] set (%.1f GB)" % (n, 32e-9 * n))
    xyzm = torch.empty((4, n), dtype=torch.float64, device=dev)
    xyzm[0].fill_(0.1)
    xyzm[1].fill_(-0.2)
    xyzm[2].fill_(1000.0)
    xyzm[3].zero_()
    xyzm[:, n - k:] = torch.from_numpy(np.ascontiguousarray(np.concatenate([xyz.T, m[None]], 0))).to(dev)
    pset = rt.make_particle_set(xyzm, eps)
    P = torch.from_numpy(np.ascontiguousarray(pts)).to(dev)
    for prec, tol in ((FP64, 1e-12), (FP32K, 3e-5)):
        phi = torch.empty(63, dtype=torch.float64, device=dev)
        grad = torch.empty((3, 63), dtype=torch.float64, device=dev)
        rt.rt_field_eval(rt.cosmology(), pset, prec, 63, P, phi, grad)
        rt.rt_sync()
        _say("field over %d particles, precision %d: done" % (n, prec))
        gphi, gg = phi.cpu().numpy(), grad.cpu().numpy()
        assert np.all(np.abs(gphi - ref_phi) <= tol * np.abs(ref_phi)), prec
        scale = np.linalg.norm(ref_g, axis=0)
        assert np.all(np.abs(gg - ref_g) <= tol * scale + 1e-30), prec
    del xyzm
    torch.cuda.empty_cache()


def test_benchmark_launch_against_the_oracle():
    """The launch bench.py times by default: the first 28672-bundle band of the 2^20 box's
    512 x 512 grid through the first 25-step window, with the plan the autotuner picks for it
    (one wavefront per 7 bundles, 2304-particle tiles, 512 workgroups).  16 seeded bundles of the
    band against the oracle traced through the same window: positions and directions, each
    relative to its change from the straight ray (a straight ray keeps x = (kx / kz) z).  (The
    bundles' own lensing signal, the ring-minus-anchor offsets, is still below 1e-12 Mpc this
    close to the observer; the whole-schedule tests compare it through mu.)"""
    from paper_1110_4894_amd.runner import GpuRun
    _say("building the 2^20 box")
    w = wl.box(n_part_log2=20, n_side=512)
    f = w.fields[0]
    band, window = 28672, 25
    wb = _with_theta(w, [f.theta[:, :band]])
    plans = [i for i in range(rt.rt_plan_count(FP32K))
             if rt.rt_plan_describe(FP32K, i)["waves_per_group"] == 1
             and rt.rt_plan_describe(FP32K, i)["tile"] == 2304 and rt.rt_plan_describe(FP32K, i)["waves_per_block"] == 8]
    assert plans
    rt.rt_force_plan(FP32K, plans[0])
    try:
        _say("gpu fp32k: %d bundles, RK4 steps [0, %d)" % (band, window))
        g = GpuRun(wb)
        g.build_bundles()
        g.trace(FP32K, 0, window)
        torch.cuda.synchronize()
        info = rt.rt_last_trace_info()
        assert info["plan_id"] == plans[0] and info["grid_blocks"] == 512
        rays = g.rays.cpu().numpy()
        assert not g.flags.cpu().numpy().any()
    finally:
        rt.rt_force_plan(FP32K, -1)
    idx = np.sort(np.random.default_rng(2811).choice(band, 16, replace=False))
    ws = _with_theta(w, [f.theta[:, idx]])
    _say("oracle: 16 bundles, RK4 steps [0, %d)" % window)
    o = oracle_run(ws, step_begin=0, step_end=window)
    c, _, ofields, theta = o["cosmo"], o["chi_s"], o["fields"], o["theta"]
    r0 = orc.build_bundles(c, ofields, theta, w.bundle_radius)
    got = rays[:, (9 * idx[:, None] + np.arange(9)).ravel()]
    want = o["rays"]
    assert np.allclose(got[3], want[3], rtol=1e-13, atol=0)   # both on the window's last node (own schedules)
    z = want[3]
    for comp, kc in ((1, 5), (2, 6)):
        straight = r0[kc] / r0[7] * z
        defl = want[comp] - straight
        assert np.all(np.abs(got[comp] - want[comp]) <= 1e-4 * np.abs(defl) + 1e-13)
        bend = want[kc] / want[7] - r0[kc] / r0[7]
        assert np.all(np.abs(got[kc] / got[7] - want[kc] / want[7]) <= 1e-4 * np.abs(bend) + 1e-16)
