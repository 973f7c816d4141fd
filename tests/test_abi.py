"""CPU checks of librt.so: it loads, exports every symbol include/rt.h declares,
its host-side routines agree with the oracle, and bad arguments are rejected
with the documented status before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as orc
from paper_1110_4894_amd import rt
from paper_1110_4894_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("librt.so not built")
    return rt.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "rt_trace" in names and "rt_build_bundles" in names and "rt_magnification" in names
    raw = C.CDLL(rt.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) <= set(rt.EXPORTS)


def test_comoving_distance_matches_oracle(lib):
    for p in [(0.3, 0.7, 0.7), (0.27, 0.73, 0.71)]:
        for z in [0.1, 0.25, 0.5, 1.0]:
            got = rt.rt_comoving_distance(rt.cosmology(*p), z)
            want = orc.comoving_distance(orc.cosmo(*p), z)
            assert abs(got / want - 1) < 1e-13


def test_schedule_matches_oracle(lib):
    chi_s = orc.comoving_distance(orc.cosmo(), 0.5)
    for args in [(1007.14, 1009.14, 1000, 1.1), (1006.0, 1010.0, 2000, 1.1), (0.0, chi_s, 2000, 1.0),
                 (0.0, 100.0, 37, 1.3), (1800.0, chi_s, 11, 1.05)]:
        a = rt.rt_make_schedule(chi_s, *args)
        b = orc.make_schedule(chi_s, *args)
        assert len(a) == len(b)
        assert np.array_equal(a, b)


def test_replica_step_sets_match_oracle(lib):
    chi_s = orc.comoving_distance(orc.cosmo(), 0.5)
    nodes = orc.make_schedule(chi_s, 0.0, chi_s, 2000, 1.0)
    L = 100 / 0.7
    assert np.array_equal(rt.rt_replica_step_sets(nodes, L, 14), orc.replica_step_sets(nodes, L, 14))
    nodes = np.array([0.0, 20.0])
    assert list(rt.rt_replica_step_sets(nodes, 10.0, 3)) == [1]


def _status(fn, *a):
    try:
        fn(*a)
    except rt.RTError as e:
        return e.status
    return 0


def test_argument_errors(lib):
    c = rt.cosmology()
    assert _status(rt.rt_comoving_distance, rt.cosmology(0.3, 0.6, 0.7), 0.5) == -2
    assert _status(rt.rt_comoving_distance, rt.cosmology(0.3, 0.7, -1.0), 0.5) == -2
    assert _status(rt.rt_comoving_distance, rt.cosmology(float("nan"), 0.7, 0.7), 0.5) == -3
    assert _status(rt.rt_comoving_distance, c, -1.0) == -1
    assert _status(rt.rt_make_schedule, 100.0, 50.0, 40.0, 10, 1.1) == -1
    assert _status(rt.rt_make_schedule, 100.0, 0.0, 100.0, 100, 1.0, 50) == -1
    assert "capacity" in rt.rt_last_error()
    # field tables are validated on the host before any device call
    chi_s = rt.rt_comoving_distance(c, 0.5)
    nodes = rt.rt_make_schedule(chi_s, 0.0, chi_s, 10, 1.0)
    good = {"sets": [], "z_nodes": nodes, "step_set": np.full(10, -1, np.int32), "bundle_offset": 0, "n_bundles": 2}
    fake = 1 << 40   # never dereferenced: validation fails first
    bad_nodes = dict(good, z_nodes=nodes[::-1].copy())
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([bad_nodes]), 0, 0, 10, 2, fake) == -4
    short = dict(good, z_nodes=rt.rt_make_schedule(chi_s * 0.9, 0.0, chi_s * 0.9, 10, 1.0))
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([short]), 0, 0, 10, 2, fake) == -4
    bad_set = dict(good, step_set=np.full(10, 3, np.int32))
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([bad_set]), 0, 0, 10, 2, fake) == -1
    assert "step_set" in rt.rt_last_error()
    overlap = [good, dict(good, bundle_offset=1)]
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable(overlap), 0, 0, 10, 4, fake) == -1
    outside = dict(good, n_bundles=5)
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([outside]), 0, 0, 10, 2, fake) == -1
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([good]), 7, 0, 10, 2, fake) == -1
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([good]), 0, 5, 2, 2, fake) == -1
    assert _status(rt.rt_trace, rt.cosmology(0.3, 0.8, 0.7), 0.5, rt.FieldTable([good]), 0, 0, 10, 2, fake) == -2
    neg = {"xyzm": None, "softening": -1.0}
    with_set = dict(good, sets=[neg], step_set=np.zeros(10, np.int32))
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([with_set]), 0, 0, 10, 2, fake) == -1
    cub = {"xyzm": None, "softening": 0.1, "background": True, "lo": (0, 0, 1), "hi": (1, 1, 0)}
    with_cub = dict(good, sets=[cub], step_set=np.zeros(10, np.int32))
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([with_cub]), 0, 0, 10, 2, fake) == -1
    # the largest set is 2^31 particles (a 32 GB FP32 copy); one more is refused
    class _Huge:
        shape = (4, (1 << 31) + 1)

        def data_ptr(self):
            return fake
    huge = dict(good, sets=[{"xyzm": _Huge(), "softening": 0.0}], step_set=np.zeros(10, np.int32))
    assert _status(rt.rt_trace, c, 0.5, rt.FieldTable([huge]), 0, 0, 10, 2, fake) == -7
    assert "2^31" in rt.rt_last_error()
    assert _status(rt.rt_build_bundles, c, rt.FieldTable([]), 2, fake, 0.1, fake) == -1     # radius too large
    assert _status(rt.rt_build_bundles, c, rt.FieldTable([]), 0, fake, 1e-8, fake) == -1
    assert _status(rt.rt_magnification, c, 0.5, 2, 0.0, fake, fake) == -1
    assert _status(rt.rt_mu_histogram, 10, fake, 0, -0.1, 0.3, fake, fake) == -1
    assert _status(rt.rt_mu_histogram, 10, fake, 10, 0.3, -0.1, fake, fake) == -1
    assert _status(rt.rt_force_plan, 0, 99) == -1
    assert rt.rt_plan_count(0) >= 1 and rt.rt_plan_count(1) >= 1 and rt.rt_plan_count(7) == 0
    info = rt.rt_plan_describe(1, 0)
    assert info["rays_per_block"] == 63 * info["waves_per_block"] // info["waves_per_group"]


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_1110_4894_amd.rt")
    with pytest.raises(RuntimeError):
        mod._lib, saved = None, mod._lib
        try:
            mod.load(str(tmp_path / "missing.so"))
        finally:
            mod._lib = saved


def test_pm_argument_errors(lib):
    """The particle-mesh entry points validate grids, n_int, sets, nodes and the observer's
    position on the host, before any device call."""
    c = rt.cosmology()
    fake = 1 << 40
    g = rt.pm_grid(32, (-1.0, -1.0, 999.0), 0.0625)
    assert rt.rt_pm_workspace_bytes(g) == 32 * 64 ** 3 + 16 * 32
    for bad in [rt.pm_grid(24, (0, 0, 0), 0.1), rt.pm_grid(2, (0, 0, 0), 0.1), rt.pm_grid(1024, (0, 0, 0), 0.1),
                rt.pm_grid(32, (0, 0, 0), 0.0), rt.pm_grid(32, (0, float("inf"), 0), 0.1)]:
        assert _status(rt.rt_pm_workspace_bytes, bad) in (-1, -3)
    pset = rt.make_particle_set(None, softening=0.01)
    assert _status(rt.rt_pm_build, pset, g, fake, fake, 100) == -1          # workspace too small
    assert "workspace" in rt.rt_last_error()
    bg = rt.make_particle_set(None, softening=0.01, background=True, lo=(0, 0, 0), hi=(1, 1, 1))
    assert _status(rt.rt_pm_build, bg, g, fake, fake, 1 << 40) == -7       # isolated lenses only
    assert _status(rt.rt_pm_eval, g, fake, 0, 4, fake, fake, fake) == -1
    assert _status(rt.rt_pm_eval, g, fake, 5, 4, fake, fake, fake) == -1
    assert _status(rt.rt_pm_eval, rt.pm_grid(4, (0, 0, 0), 0.1), fake, 3, 4, fake, fake, fake) == -1
    chi_s = rt.rt_comoving_distance(c, 0.5)
    nodes = rt.rt_make_schedule(chi_s, 0.0, chi_s, 10, 1.0)
    assert _status(rt.rt_trace_pm, c, 0.5, g, fake, 2, nodes[::-1].copy(), 0, 10, 2, fake) == -4
    assert _status(rt.rt_trace_pm, c, 0.5, [g, g], [fake, fake], 2, nodes, 0, 10, 2, fake, None,
                   np.full(10, 2, np.int32)) == -1
    assert "step_grid" in rt.rt_last_error()
    assert _status(rt.rt_trace_pm, c, 0.5, g, fake, 2, nodes * 0.9, 0, 10, 2, fake) == -4
    around = rt.pm_grid(32, (-1.0, -1.0, -1.0), 0.0625)
    assert _status(rt.rt_trace_pm, c, 0.5, around, fake, 2, nodes, 0, 10, 2, fake) == -1
    assert "observer" in rt.rt_last_error()
    assert _status(rt.rt_trace_pm, c, 0.5, g, fake, 2, nodes, 5, 2, 2, fake) == -1
    assert _status(rt.rt_trace_pm_lambda, c, 0.5, g, fake, 2, 0.0, 100, 2, fake) == -1
    assert _status(rt.rt_trace_pm_lambda, c, 0.5, g, fake, 2, float("nan"), 100, 2, fake) == -3
    assert _status(rt.rt_trace_pm_lambda, c, 0.5, g, fake, 2, 0.5, 0, 2, fake) == -1
    assert _status(rt.rt_trace_pm_lambda, c, 0.5, around, fake, 2, 0.5, 100, 2, fake) == -1
    assert _status(rt.rt_trace_pm_lambda, c, 0.5, g, fake, 9, 0.5, 100, 2, fake) == -1
    # periodic boxes: smaller workspace (no padding)
    pg = rt.pm_grid(32, (-1.0, -1.0, 999.0), 0.0625, periodic=True)
    assert rt.rt_pm_workspace_bytes(pg) == 32 * 32 ** 3 + 8 * 32
    bad = rt.pm_grid(32, (0, 0, 0), 0.1)
    bad.periodic = 2
    assert _status(rt.rt_pm_workspace_bytes, bad) == -1
    # the slab stack of the lambda integrator
    sl = rt.rt_trace_pm_lambda_slabs
    b2, s2 = [0.0, 100.0, 200.0], [0, -1]
    assert _status(sl, c, 0.5, [pg], [fake], 2, [0.0], [], 0.5, 100, 2, fake) == -1                 # no slab
    assert _status(sl, c, 0.5, [pg], [fake], 2, [0.0, 100.0, 100.0], s2, 0.5, 100, 2, fake) == -1   # not increasing
    assert _status(sl, c, 0.5, [pg], [fake], 2, [0.0, float("inf"), 300.0], s2, 0.5, 100, 2, fake) == -3
    assert _status(sl, c, 0.5, [pg], [fake], 2, b2, [1, 0], 0.5, 100, 2, fake) == -1                # no grid 1
    assert "slab_grid" in rt.rt_last_error()
    assert _status(sl, c, 0.5, [pg, around], [fake, fake], 2, b2, s2, 0.5, 100, 2, fake) == -1      # observer
    coarse = rt.pm_grid(32, (-1.0, -1.0, 999.0), 0.125, periodic=True)
    assert _status(sl, c, 0.5, [pg, coarse], [fake, fake], 2, b2, s2, 0.5, 100, 2, fake) == -1      # two spacings
    assert ".h" in rt.rt_last_error()
    assert _status(sl, c, 0.5, [pg], [fake], 2, b2, s2, 0.0, 100, 2, fake) == -1
    assert _status(sl, c, 0.5, [pg], [fake], 9, b2, s2, 0.5, 100, 2, fake) == -1


def test_flexion_argument_errors(lib):
    """rt_flexion validates its arguments on the host, before any device call."""
    c = rt.cosmology()
    fake = 1 << 40
    assert _status(rt.rt_flexion, c, 0.5, 0, 1e-8, fake, fake) == -1
    assert _status(rt.rt_flexion, c, 0.5, 4, 0.0, fake, fake) == -1
    assert _status(rt.rt_flexion, c, 0.5, 4, float("nan"), fake, fake) == -3
    assert _status(rt.rt_flexion, c, 0.5, 4, 1e-8, fake, None) == -1
    assert _status(rt.rt_flexion, c, -1.0, 4, 1e-8, fake, fake) == -1
