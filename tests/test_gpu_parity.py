"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Element-by-element comparisons on the same seeded inputs, at sizes the oracle
finishes in seconds while spanning several particle tiles with ragged tails.
Tolerances:
  * FP64 GPU vs oracle: mu within 1e-7 relative (1/mu within 1e-7 when |mu| > 100),
    exit positions within 1e-7 of the deflection plus 1e-12 Mpc, lookback
    time and wave vector within 1e-12 relative.  (The stated contract is 1e-4;
    observed differences are round-off amplified along the path.)
  * FP32+Kahan GPU vs oracle: the measurement gate at 1e-4 -- relative mu error
    <= 1e-4 for |mu| <= 100 and |d(1/mu)| <= 1e-6 beyond (tests/metrics.py);
    exit positions within 1e-4 of the deflection plus 1e-12 Mpc.
"""
import dataclasses
import math
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from paper_1110_4894_amd import rt
from paper_1110_4894_amd import workloads as wl
from tests.metrics import mu_errors
from tests.oracle_run import oracle_run

pytestmark = pytest.mark.gpu

FP64, FP32K = rt.RT_FP64, rt.RT_FP32_KAHAN


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()
    yield
    rt.rt_force_plan(FP64, -1)
    rt.rt_force_plan(FP32K, -1)


def _run(w, precision, **kw):
    from paper_1110_4894_amd.runner import GpuRun
    g = GpuRun(w)
    return g.run(precision, **kw), g


def _check_fp64(g, o, theta):
    assert np.array_equal(g["flags"], o["flags"])
    assert np.max(mu_errors(g["mu"], o["mu"])) < 1e-7
    gr, orr = g["rays"], o["rays"]
    th = np.repeat(theta, 9, axis=1)
    defl = np.hypot(orr[1] - th[0] * o["chi_s"], orr[2] - th[1] * o["chi_s"])
    d = np.hypot(gr[1] - orr[1], gr[2] - orr[2])
    assert np.all(d <= 1e-7 * defl + 1e-12)
    # z = the last node, i.e. each side's own chi_s (they differ in the last bits)
    assert np.all(np.abs(gr[3] - orr[3]) <= 1e-14 * orr[3])
    for c in (0, 4, 5, 6, 7):
        scale = np.max(np.abs(orr[c])) if c in (5, 6) else np.abs(orr[c])
        assert np.all(np.abs(gr[c] - orr[c]) <= 1e-12 * scale + 1e-300), c
    assert np.allclose(g["jac"], o["jac"], rtol=0, atol=1e-7 * max(1.0, np.abs(o["jac"]).max()))


def _check_fp32(g, o, theta, tol_mu=1e-4):
    assert np.array_equal(g["flags"], o["flags"])
    err = mu_errors(g["mu"], o["mu"])
    assert np.max(err) <= tol_mu, (np.max(err), int(np.argmax(err)), o["mu"][np.argmax(err)])
    gr, orr = g["rays"], o["rays"]
    th = np.repeat(theta, 9, axis=1)
    defl = np.hypot(orr[1] - th[0] * o["chi_s"], orr[2] - th[1] * o["chi_s"])
    d = np.hypot(gr[1] - orr[1], gr[2] - orr[2])
    assert np.all(d <= 1e-4 * defl + 1e-12)


# --------------------------------------------------------------------------- field kernel
def _set_for(n, eps, seed=3, background=False, masses="random"):
    """masses: "random" (the general FP32 loop), "equal" (the equal-mass loop) or
    "equal_but_last" (equal except a 50x heavier last particle: the general loop)."""
    rng = np.random.default_rng(seed)
    xyz = rng.normal(size=(n, 3)) * 0.5 + np.array([0.1, -0.2, 1000.0])
    m = rng.uniform(1e9, 1e11, n)
    if masses != "random":
        m = np.full(n, 3e10)
    if masses == "equal_but_last":
        m[-1] *= 50.0
    lo, hi = (-3.0, -3.0, 997.0), (3.0, 3.0, 1003.0)
    return xyz, m, eps, background, lo, hi


@pytest.mark.parametrize("n", [1, 63, 256, 1000, 4099])
@pytest.mark.parametrize("background", [False, True])
@pytest.mark.parametrize("masses", ["random", "equal", "equal_but_last"])
def test_field_eval_parity(n, background, masses):
    if masses == "equal_but_last" and n == 1:
        pytest.skip("one particle: its masses are equal")
    xyz, m, eps, bg, lo, hi = _set_for(n, 0.01, background=background, masses=masses)
    c = orc.cosmo()
    ps = orc.ParticleSet(xyz=xyz, m=m, softening=eps, background=bg, lo=lo, hi=hi)
    rng = np.random.default_rng(n)
    pts = rng.normal(size=(3, 300)) * 0.3 + np.array([[0.0], [0.0], [1000.0]])
    ref_phi = np.zeros(300)
    ref_g = np.zeros((3, 300))
    scale_phi = np.zeros(300)
    scale_g = np.zeros(300)
    bare = orc.ParticleSet(xyz=xyz, m=m, softening=eps)
    for i in range(300):
        ref_phi[i], ref_g[:, i] = orc.field_at(c, ps, pts[:, i])
        p0, g0 = orc.field_at(c, bare, pts[:, i])
        # FP32 errors scale with the particle sum, which the cuboid term may cancel
        scale_phi[i] = max(abs(p0), abs(ref_phi[i]))
        scale_g[i] = max(np.linalg.norm(g0), np.linalg.norm(ref_g[:, i]))
    dev = torch.device("cuda")
    xyzm = torch.from_numpy(np.ascontiguousarray(np.concatenate([xyz.T, m[None]], 0))).to(dev)
    pset = rt.make_particle_set(xyzm, eps, bg, lo, hi)
    P = torch.from_numpy(np.ascontiguousarray(pts)).to(dev)
    for prec, tol in ((FP64, 1e-12), (FP32K, 3e-5)):
        phi = torch.empty(300, dtype=torch.float64, device=dev)
        grad = torch.empty((3, 300), dtype=torch.float64, device=dev)
        rt.rt_field_eval(rt.cosmology(), pset, prec, 300, P, phi, grad)
        rt.rt_sync()                         # the library's own wait on the caller's stream
        gphi, gg = phi.cpu().numpy(), grad.cpu().numpy()
        assert np.all(np.abs(gphi - ref_phi) <= tol * scale_phi), prec
        assert np.all(np.abs(gg - ref_g) <= tol * scale_g + 1e-30), prec


def _bundle_points(rng, n_groups, z, spread, ring, centre=(0.0, 0.0)):
    """Groups of 9 points shaped like bundles at one height z: an anchor spread
    around `centre` and 8 points at distance `ring` (deformed by a random linear map),
    as a bundle's rays are at a stage."""
    anchors = rng.normal(size=(n_groups, 2)) * spread + np.asarray(centre)
    k = np.arange(8)
    u = np.stack([np.cos(np.pi * k / 4), np.sin(np.pi * k / 4)], 1) * ring
    pts = []
    for a in anchors:
        A = np.eye(2) + rng.normal(size=(2, 2)) * 0.3
        pts.append(np.vstack([a, a + u @ A.T]))
    xy = np.concatenate(pts, 0)
    return np.stack([xy[:, 0], xy[:, 1], np.full(len(xy), z)])


@pytest.mark.parametrize("case", ["halo_equal", "halo_random", "box_background", "point_near", "points_mixed"])
def test_bundle_field_differences(case):
    """FP32 field at bundle-shaped points (the trace kernel's arithmetic: moments about
    each group's first point, near pairs summed per point) against the FP64 oracle.
    The ring-minus-anchor field differences carry the lensing signal: they must keep
    1e-5 of their own size, far below what one FP32 rounding of a particle-point
    displacement would leave (the ring is 5 pc, the particles up to Mpc away)."""
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    z = 1000.0
    ring = 5e-6
    lo, hi, bg = (-3.0, -3.0, 997.0), (3.0, 3.0, 1003.0), False
    if case.startswith("halo"):
        n = 3000
        xyz = rng.normal(size=(n, 3)) * 0.1 + np.array([0.0, 0.0, z + 0.01])
        m = np.full(n, 3e10) if case == "halo_equal" else rng.uniform(1e9, 1e11, n)
        eps, spread = 0.0025, 0.05
    elif case == "box_background":
        n = 4000
        xyz = rng.uniform(-3, 3, size=(n, 3)) + np.array([0.0, 0.0, z])
        m = np.full(n, 4.5e11)
        eps, spread, bg = 0.0714, 1.0, True
    elif case == "point_near":
        # one unsoftened mass; the groups pass at 20 pc to 20 kpc, so that some pairs
        # are within 256 ring radii and take the direct per-point sum
        xyz = np.array([[0.0, 0.0, z + 0.003]])
        m = np.array([1e12])
        eps, spread = 0.0, 0.005
    else:
        # a few unsoftened masses of very different size among softened-free groups
        k = 6
        xyz = rng.normal(size=(k, 3)) * 0.01 + np.array([0.0, 0.0, z])
        m = 10 ** rng.uniform(10, 13, k)
        eps, spread = 0.0, 0.01
    n_groups = 7 * 6 + 3                                # several wavefronts and a ragged last one
    pts = _bundle_points(rng, n_groups, z, spread, ring)
    npts = pts.shape[1]
    c = orc.cosmo()
    ps = orc.ParticleSet(xyz=xyz, m=m, softening=eps, background=bg, lo=lo, hi=hi)
    bare = orc.ParticleSet(xyz=xyz, m=m, softening=eps)
    ref_phi = np.zeros(npts)
    ref_g = np.zeros((3, npts))
    scale_phi = np.zeros(npts)
    scale_g = np.zeros(npts)
    for i in range(npts):
        ref_phi[i], ref_g[:, i] = orc.field_at(c, ps, pts[:, i])
        p0, g0 = orc.field_at(c, bare, pts[:, i])
        # FP32 errors scale with the particle sum, which the cuboid term may cancel
        scale_phi[i] = max(abs(p0), abs(ref_phi[i]))
        scale_g[i] = max(np.linalg.norm(g0), np.linalg.norm(ref_g[:, i]))
    dev = torch.device("cuda")
    xyzm = torch.from_numpy(np.ascontiguousarray(np.concatenate([xyz.T, m[None]], 0))).to(dev)
    pset = rt.make_particle_set(xyzm, eps, bg, lo, hi)
    P = torch.from_numpy(np.ascontiguousarray(pts)).to(dev)
    phi = torch.empty(npts, dtype=torch.float64, device=dev)
    grad = torch.empty((3, npts), dtype=torch.float64, device=dev)
    rt.rt_field_eval(rt.cosmology(), pset, FP32K, npts, P, phi, grad)
    rt.rt_sync()
    gphi, gg = phi.cpu().numpy(), grad.cpu().numpy()
    # absolute field: FP32 accuracy
    assert np.all(np.abs(gphi - ref_phi) <= 3e-6 * scale_phi), case
    assert np.all(np.abs(gg - ref_g) <= 3e-6 * scale_g[None, :]), case
    # ring-minus-anchor differences, per group, against their own size
    worst = 0.0
    for gi in range(n_groups):
        a, r = 9 * gi, slice(9 * gi + 1, 9 * gi + 9)
        d_ref = ref_g[:, r] - ref_g[:, a:a + 1]
        d_got = gg[:, r] - gg[:, a:a + 1]
        size = np.max(np.linalg.norm(d_ref, axis=0))
        worst = max(worst, np.max(np.linalg.norm(d_got - d_ref, axis=0)) / size)
        p_ref = ref_phi[r] - ref_phi[a]
        p_got = gphi[r] - gphi[a]
        assert np.max(np.abs(p_got - p_ref)) <= 1e-5 * np.max(np.abs(p_ref)) + 1e-14 * abs(ref_phi[a]), (case, gi)
    print("%s: worst ring-difference error %.2e of its size" % (case, worst), flush=True)
    assert worst <= 1e-5, case


# --------------------------------------------------------------------------- bundles
def test_build_bundles_parity():
    w = wl.schwarzschild(n_radii=3, n_azimuth=5)
    # a mass near the observer so that phi_obs matters
    w.fields[0].sets[0].xyz = np.array([[0.002, 0.001, 0.05]])
    from tests.oracle_run import oracle_fields
    c, chi_s, fields, theta = oracle_fields(w)
    ref = orc.build_bundles(c, fields, theta, w.bundle_radius)
    from paper_1110_4894_amd.runner import GpuRun
    g = GpuRun(w)
    g.build_bundles()
    torch.cuda.synchronize()
    got = g.rays.cpu().numpy()
    assert np.allclose(got, ref, rtol=1e-15, atol=0)


# --------------------------------------------------------------------------- trace
def _schw(nb=12):
    w = wl.schwarzschild(n_radii=4, n_azimuth=3)
    return w


def test_schwarzschild_fp64_parity():
    w = _schw()
    o = oracle_run(w)
    g, _ = _run(w, FP64)
    _check_fp64(g, o, o["theta"])


def _small_nfw(n_part=3001, n_side=4, n_fine=150, radius=1e-3):
    w = wl.nfw(n_side=n_side, n_part=n_part, n_fine=n_fine, radius_arcsec=radius)
    return w


def test_nfw_fp64_and_fp32_parity():
    w = _small_nfw()
    o = oracle_run(w)
    g64, _ = _run(w, FP64)
    _check_fp64(g64, o, o["theta"])
    g32, _ = _run(w, FP32K)
    _check_fp32(g32, o, o["theta"])


def _unequal_masses(w, seed=11):
    """The same workload with every particle mass scaled by a seeded factor in [0.5, 1.5]
    (the FP32 path then takes its general-mass loop)."""
    rng = np.random.default_rng(seed)
    fields = [dataclasses.replace(f, sets=[dataclasses.replace(s, m=s.m * rng.uniform(0.5, 1.5, len(s.m)))
                                           for s in f.sets]) for f in w.fields]
    return dataclasses.replace(w, fields=fields)


@pytest.mark.parametrize("prec,masses", [(FP64, "equal"), (FP64, "unequal"), (FP32K, "equal"), (FP32K, "unequal")])
def test_every_plan_passes_parity(prec, masses):
    w = _small_nfw(n_part=2049, n_side=5, n_fine=60)
    if masses == "unequal":
        w = _unequal_masses(w)
    o = oracle_run(w)
    try:
        for pid in range(rt.rt_plan_count(prec)):
            rt.rt_force_plan(prec, pid)
            g, _ = _run(w, prec)
            (_check_fp64 if prec == FP64 else _check_fp32)(g, o, o["theta"])
    finally:
        rt.rt_force_plan(prec, -1)


def _small_box():
    return wl.box(n_part_log2=12, n_side=3, n_steps=150)


def test_box_parity_with_background():
    w = _small_box()
    o = oracle_run(w)
    g64, _ = _run(w, FP64)
    _check_fp64(g64, o, o["theta"])
    g32, _ = _run(w, FP32K)
    _check_fp32(g32, o, o["theta"])


def test_empty_replicas_keep_their_background():
    """Degenerate sets: every other replica of the box holds no particles (n = 0), so only
    its uniform-cuboid term acts there (an empty, underdense region)."""
    w = _small_box()
    f = w.fields[0]
    sets = [dataclasses.replace(s, xyz=np.zeros((0, 3)), m=np.zeros(0)) if k % 2 == 0 else s
            for k, s in enumerate(f.sets)]
    w2 = dataclasses.replace(w, fields=[dataclasses.replace(f, sets=sets)])
    o = oracle_run(w2)
    assert np.all(o["mu"] < 1.0)
    g64, _ = _run(w2, FP64)
    _check_fp64(g64, o, o["theta"])
    g32, _ = _run(w2, FP32K)
    _check_fp32(g32, o, o["theta"])


def test_particle_array_shared_by_two_frames():
    """One particle array in two fields, with and without its background cuboid:
    the two sets have different FP32 frames, so each gets its own FP32 copy."""
    w = _small_box()
    f = w.fields[0]
    bare = dataclasses.replace(f, name="bare", sets=[dataclasses.replace(s, background=False) for s in f.sets])
    assert bare.sets[0].xyz is f.sets[0].xyz          # uploaded once, shared on the device
    w2 = dataclasses.replace(w, fields=[f, bare])
    o = oracle_run(w2)
    g64, _ = _run(w2, FP64)
    _check_fp64(g64, o, o["theta"])
    g32, _ = _run(w2, FP32K)
    _check_fp32(g32, o, o["theta"])


def test_one_configuration_on_two_streams_is_serialised():
    """Two launches of one cached configuration on different streams, with no host wait
    between them, give what the same two launches give on one stream (they share the
    work queue and the FP32 copies, so the second waits for the first)."""
    from paper_1110_4894_amd.runner import GpuRun
    w = _small_nfw(n_part=900, n_side=3, n_fine=60)
    g = GpuRun(w)
    g.run(FP32K)                               # builds and captures the configuration
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def twice(a, b):
        g.build_bundles()
        torch.cuda.synchronize()
        g.trace(FP32K, stream=a)
        g.trace(FP32K, stream=b)
        torch.cuda.synchronize()
        assert rt.rt_last_trace_info()["graph_reused"] == 1
        return g.rays.cpu().numpy()

    same = twice(s1, s1)
    assert np.array_equal(twice(s1, s2), same)
    assert np.array_equal(twice(s2, s1), same)


def test_graph_replay_follows_new_masses():
    """The equal-mass test runs inside the captured graph: a replay after the masses
    changed in place (same pointers, so the graph is reused) takes the general loop."""
    from paper_1110_4894_amd.runner import GpuRun
    w = _small_nfw(n_part=1500, n_side=3, n_fine=80)
    uploads = {}
    g = GpuRun(w, uploads=uploads)
    o = oracle_run(w)
    _check_fp32(g.run(FP32K), o, o["theta"])
    w2 = _unequal_masses(w)
    dev_xyzm = uploads[id(w.fields[0].sets[0].xyz)]
    dev_xyzm[3].copy_(torch.from_numpy(w2.fields[0].sets[0].m))
    o2 = oracle_run(w2)
    g2 = g.run(FP32K)
    assert rt.rt_last_trace_info()["graph_reused"] == 1
    _check_fp32(g2, o2, o2["theta"])
    assert np.max(np.abs(g2["mu"] - o["mu"])) > 100 * np.max(np.abs(g2["mu"] - o2["mu"]))


def test_empty_field_unit_magnification():
    w = wl.empty(n_bundles=30)
    g, _ = _run(w, FP64)
    assert np.max(np.abs(g["mu"] - 1)) < 1e-8
    g, _ = _run(w, FP32K)
    assert np.max(np.abs(g["mu"] - 1)) < 1e-8


def test_several_uneven_fields_in_one_launch():
    a = wl.schwarzschild(n_radii=2, n_azimuth=3)
    b = _small_nfw(n_part=777, n_side=3, n_fine=80)
    e = wl.empty(n_bundles=4)
    w = wl.Workload("mix", a.cosmology, a.z_source, a.bundle_radius, a.fields + b.fields + e.fields)
    o = oracle_run(w)
    g, _ = _run(w, FP64)
    _check_fp64(g, o, o["theta"])
    g, _ = _run(w, FP32K)
    _check_fp32(g, o, o["theta"])


def test_resume_is_bitwise_identical_and_deterministic():
    w = _small_nfw(n_part=1500, n_side=3, n_fine=100)
    from paper_1110_4894_amd.runner import GpuRun
    for prec in (FP64, FP32K):
        g = GpuRun(w)
        full = g.run(prec)["rays"]
        again = g.run(prec)["rays"]
        assert np.array_equal(full, again)
        g.build_bundles()
        g.trace(prec, 0, 37)
        g.trace(prec, 37, 2 ** 31 - 1)
        torch.cuda.synchronize()
        assert np.array_equal(g.rays.cpu().numpy(), full)


def test_graph_replay_matches_eager_each_time():
    """The captured graph is replayed with host work and synchronisation in between;
    every replay reproduces the first result."""
    w = _small_nfw(n_part=900, n_side=3, n_fine=60)
    from paper_1110_4894_amd.runner import GpuRun
    g = GpuRun(w)
    first = g.run(FP32K)
    for _ in range(3):
        g.build_bundles()
        g.trace(FP32K)
        info = rt.rt_last_trace_info()
        assert info["graph_reused"] == 1
        g.magnification()
        torch.cuda.synchronize()
        assert np.array_equal(g.mu.cpu().numpy(), first["mu"])


def test_magnification_and_histogram_parity():
    # magnification of oracle-traced rays
    w = _small_nfw(n_part=1000, n_side=4, n_fine=80)
    o = oracle_run(w)
    dev = torch.device("cuda")
    rays = torch.from_numpy(o["rays"]).to(dev)
    nb = o["mu"].shape[0]
    mu = torch.empty(nb, dtype=torch.float64, device=dev)
    jac = torch.empty((4, nb), dtype=torch.float64, device=dev)
    c = rt.cosmology()
    rt.rt_magnification(c, w.z_source, nb, w.bundle_radius, rays, mu, jac)
    torch.cuda.synchronize()
    assert np.allclose(mu.cpu().numpy(), o["mu"], rtol=1e-12, atol=0)
    assert np.allclose(jac.cpu().numpy(), o["jac"], rtol=0, atol=1e-12)
    # histogram of a wide synthetic mu sample, including excluded and out-of-range values
    rng = np.random.default_rng(4)
    mus = np.concatenate([np.exp(rng.normal(0, 0.08, 20011)), [-1.0, 0.0, 0.3, 7.0]])
    ref_pdf, ref_mom = orc.mu_histogram(mus, 200, -0.1, 0.3)
    m = torch.from_numpy(mus).to(dev)
    pdf = torch.empty(200, dtype=torch.float64, device=dev)
    mom = torch.empty(6, dtype=torch.float64, device=dev)
    rt.rt_mu_histogram(len(mus), m, 200, -0.1, 0.3, pdf, mom)
    torch.cuda.synchronize()
    assert np.allclose(pdf.cpu().numpy(), ref_pdf, rtol=1e-12, atol=1e-14)
    assert np.allclose(mom.cpu().numpy(), ref_mom, rtol=1e-12, atol=0)
    # shear PDF of the oracle-traced bundles' Jacobians
    ref_pdf, ref_mom = orc.shear_histogram(o["mu"], o["jac"], 40, 0.0, 0.2)
    pdf = torch.empty(40, dtype=torch.float64, device=dev)
    rt.rt_shear_histogram(nb, torch.from_numpy(o["mu"]).to(dev), torch.from_numpy(o["jac"]).to(dev), 40, 0.0, 0.2,
                          pdf, mom)
    torch.cuda.synchronize()
    assert np.allclose(pdf.cpu().numpy(), ref_pdf, rtol=1e-12, atol=1e-14)
    assert np.allclose(mom.cpu().numpy(), ref_mom, rtol=1e-12, atol=0)


def test_result_independent_of_grid_size():
    """The persistent launch drains one work queue: any number of workgroups gives
    bitwise identical rays."""
    w = _small_nfw(n_part=1200, n_side=6, n_fine=40)
    from paper_1110_4894_amd.runner import GpuRun
    try:
        for prec in (FP64, FP32K):
            rt.rt_set_grid_limit(0)
            ref = GpuRun(w).run(prec)["rays"]
            for lim in (1, 3, 7):
                rt.rt_set_grid_limit(lim)
                got = GpuRun(w).run(prec)["rays"]
                assert np.array_equal(got, ref), (prec, lim)
    finally:
        rt.rt_set_grid_limit(0)


def test_flags_outside_the_weak_field():
    """A 1e17 Msun point mass: rays at ~50 kpc leave the weak-field regime (flag 4),
    rays aimed at the mass turn back or blow up (flags 1/2) and keep their last good
    state; the same rays are flagged on both sides and nothing faults."""
    w = wl.schwarzschild(n_radii=1, n_azimuth=1, mass=1e17)
    f = w.fields[0]
    chi_l = f.meta["chi_l"]
    b = np.array([50e-3, 80e-3, 1e-4, 2e-5, 300e-3])           # impact parameters, Mpc
    ang = np.arange(len(b)) * 1.1
    f.theta = np.stack([b / chi_l * np.cos(ang), b / chi_l * np.sin(ang)])
    o = oracle_run(w)
    for prec in (FP64, FP32K):
        g, _ = _run(w, prec)
        hard_o = (o["flags"] & 3) != 0
        hard_g = (g["flags"] & 3) != 0
        assert np.array_equal(hard_o, hard_g)
        soft = ~hard_o
        assert np.array_equal(o["flags"][soft] & 4, g["flags"][soft] & 4)
        assert np.all(np.isfinite(g["rays"]))
    assert hard_o.any() and (o["flags"] & 4).any()
