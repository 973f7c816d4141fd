"""ctypes binding of librt.so (include/rt.h): same names, argument marshalling only.

Device arrays are passed as torch CUDA tensors (or raw integer device
addresses); every step of the lensing path runs in the library's HIP kernels.
There is no CPU fallback: if librt.so is missing or cannot be loaded, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RT_LIB_PATH names another build of the library to load instead (the host-sanitizer test's).
LIB_PATH = os.environ.get("RT_LIB_PATH") or os.path.join(_HERE, "librt.so")

RT_OK = 0
RT_FP64 = 0
RT_FP32_KAHAN = 1
PRECISIONS = {"fp64": RT_FP64, "fp32k": RT_FP32_KAHAN}

FLAG_NONFINITE = 1
FLAG_TURNED_BACK = 2
FLAG_STRONG_FIELD = 4


class RTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("rt status %d: %s" % (status, message))
        self.status = status


class rt_cosmology(C.Structure):
    _fields_ = [("omega_m", C.c_double), ("omega_lambda", C.c_double), ("h", C.c_double)]


class rt_particle_set(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyzm", C.c_void_p), ("softening", C.c_double), ("background", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class rt_field(C.Structure):
    _fields_ = [("n_sets", C.c_int32), ("sets", C.c_void_p), ("n_steps", C.c_int32), ("z_nodes", C.c_void_p),
                ("step_set", C.c_void_p), ("bundle_offset", C.c_int64), ("n_bundles", C.c_int64)]


class rt_plan_info(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("waves_per_group", C.c_int32), ("tile", C.c_int32),
                ("rays_per_block", C.c_int32), ("waves_per_simd", C.c_int32)]


class rt_trace_info(C.Structure):
    _fields_ = [("kernel_ms", C.c_double), ("interactions", C.c_double), ("plan_id", C.c_int32),
                ("grid_blocks", C.c_int32), ("n_items", C.c_int32), ("graph_reused", C.c_int32)]


class rt_pm_grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("origin", C.c_double * 3), ("h", C.c_double), ("periodic", C.c_int32)]


EXPORTS = ["rt_comoving_distance", "rt_make_schedule", "rt_replica_step_sets", "rt_build_bundles", "rt_trace",
           "rt_magnification", "rt_flexion", "rt_mu_histogram", "rt_mu_histogram_noalloc", "rt_shear_histogram", "rt_field_eval",
           "rt_plan_count", "rt_plan_describe",
           "rt_force_plan", "rt_set_grid_limit", "rt_autotune", "rt_enable_timing", "rt_last_trace_info", "rt_last_error",
           "rt_release_caches", "rt_pm_workspace_bytes", "rt_pm_build", "rt_pm_eval", "rt_trace_pm", "rt_trace_pm_lambda",
           "rt_trace_pm_lambda_slabs", "rt_sync"]

_lib = None


def load(path: str = LIB_PATH):
    """Load librt.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librt.so not found at %s; build it with `python -m paper_1110_4894_amd.build`" % path)
    lib = C.CDLL(path)
    d, p, i32, i64, st = C.c_double, C.c_void_p, C.c_int32, C.c_int64, C.c_int
    sigs = {
        "rt_comoving_distance": (st, [p, d, p]),
        "rt_make_schedule": (st, [d, d, d, i32, d, p, i32, p]),
        "rt_replica_step_sets": (st, [p, i32, d, i32, p]),
        "rt_build_bundles": (st, [p, p, i32, i64, p, d, p, p]),
        "rt_trace": (st, [p, d, p, i32, st, i32, i32, i64, p, p, p]),
        "rt_magnification": (st, [p, d, i64, d, p, p, p, p]),
        "rt_flexion": (st, [p, d, i64, d, p, p, p, p]),
        "rt_mu_histogram": (st, [i64, p, i32, d, d, p, p, p]),
        "rt_mu_histogram_noalloc": (st, [i64, p, i32, d, d, p, p, p]),
        "rt_shear_histogram": (st, [i64, p, p, i32, d, d, p, p, p]),
        "rt_field_eval": (st, [p, p, st, i64, p, p, p, p]),
        "rt_plan_count": (i32, [st]),
        "rt_plan_describe": (st, [st, i32, p]),
        "rt_force_plan": (st, [st, i32]),
        "rt_set_grid_limit": (st, [i32]),
        "rt_autotune": (st, [p, d, p, i32, st, i32, i32, i64, p, p, p]),
        "rt_enable_timing": (st, [i32]),
        "rt_last_trace_info": (st, [p]),
        "rt_last_error": (C.c_char_p, []),
        "rt_sync": (st, [p]),
        "rt_release_caches": (None, []),
        "rt_pm_workspace_bytes": (st, [p, p]),
        "rt_pm_build": (st, [p, p, p, p, C.c_size_t, p]),
        "rt_pm_eval": (st, [p, p, i32, i64, p, p, p, p]),
        "rt_trace_pm": (st, [p, d, i32, p, p, i32, i32, p, p, i32, i32, i64, p, p, p]),
        "rt_trace_pm_lambda": (st, [p, d, p, p, i32, d, i32, i64, p, p, p, p]),
        "rt_trace_pm_lambda_slabs": (st, [p, d, i32, p, p, i32, i32, p, p, d, i32, i64, p, p, p, p]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != RT_OK:
        raise RTError(status, load().rt_last_error().decode())


def _dptr(x) -> Optional[int]:
    """Device address of a torch tensor (or an int address), None for None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def cosmology(omega_m: float = 0.3, omega_lambda: float = 0.7, h: float = 0.7) -> rt_cosmology:
    return rt_cosmology(omega_m, omega_lambda, h)


# ----------------------------------------------------------------------------- field tables
class FieldTable:
    """Owns the host-side rt_field / rt_particle_set arrays (and keeps alive the
    arrays they point to).  `sets_per_field[f]` lists (xyzm_tensor [4, n] float64
    on the device, softening, background, lo, hi)."""

    def __init__(self, fields: Sequence[dict]):
        self._keep = []
        self.arr = (rt_field * max(1, len(fields)))()
        for i, f in enumerate(fields):
            sets = (rt_particle_set * max(1, len(f["sets"])))()
            for j, s in enumerate(f["sets"]):
                xyzm = s["xyzm"]
                n = int(xyzm.shape[1]) if xyzm is not None else 0
                sets[j] = rt_particle_set(n, _dptr(xyzm) if n else None, float(s.get("softening", 0.0)),
                                          1 if s.get("background") else 0,
                                          (C.c_double * 3)(*s.get("lo", (0.0, 0.0, 0.0))),
                                          (C.c_double * 3)(*s.get("hi", (0.0, 0.0, 0.0))))
                self._keep.append(xyzm)
            nodes = np.ascontiguousarray(f["z_nodes"], dtype=np.float64)
            ss = np.ascontiguousarray(f["step_set"], dtype=np.int32)
            self._keep += [sets, nodes, ss]
            self.arr[i] = rt_field(len(f["sets"]), C.addressof(sets), len(nodes) - 1, nodes.ctypes.data,
                                   ss.ctypes.data, int(f["bundle_offset"]), int(f["n_bundles"]))
        self.n = len(fields)

    @property
    def ptr(self) -> int:
        return C.addressof(self.arr)


def make_particle_set(xyzm, softening: float = 0.0, background: bool = False, lo=(0, 0, 0), hi=(0, 0, 0)):
    n = int(xyzm.shape[1]) if xyzm is not None else 0
    s = rt_particle_set(n, _dptr(xyzm) if n else None, float(softening), 1 if background else 0,
                        (C.c_double * 3)(*lo), (C.c_double * 3)(*hi))
    s._keep = xyzm
    return s


# ----------------------------------------------------------------------------- entry points
def rt_comoving_distance(cosmo: rt_cosmology, z: float) -> float:
    out = C.c_double()
    _check(load().rt_comoving_distance(C.byref(cosmo), float(z), C.addressof(out)))
    return out.value


def rt_make_schedule(chi_s: float, z_lo: float, z_hi: float, n_fine: int, q: float, capacity: int = 1 << 20):
    nodes = np.zeros(capacity)
    n = C.c_int32()
    _check(load().rt_make_schedule(float(chi_s), float(z_lo), float(z_hi), int(n_fine), float(q), nodes.ctypes.data,
                                   int(capacity), C.addressof(n)))
    return nodes[: n.value + 1].copy()


def rt_replica_step_sets(nodes, box: float, n_replicas: int):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    out = np.zeros(len(nodes) - 1, dtype=np.int32)
    _check(load().rt_replica_step_sets(nodes.ctypes.data, len(nodes) - 1, float(box), int(n_replicas),
                                       out.ctypes.data))
    return out


def rt_build_bundles(cosmo, table: FieldTable, n_bundles: int, theta, radius: float, rays, stream=None):
    _check(load().rt_build_bundles(C.byref(cosmo), table.ptr if table.n else None, table.n, int(n_bundles),
                                   _dptr(theta), float(radius), _dptr(rays), _stream(stream)))


def rt_trace(cosmo, z_source: float, table: FieldTable, precision: int, step_begin: int, step_end: int,
             n_bundles: int, rays, flags=None, stream=None):
    _check(load().rt_trace(C.byref(cosmo), float(z_source), table.ptr if table.n else None, table.n,
                           int(precision), int(step_begin), int(step_end), int(n_bundles), _dptr(rays),
                           _dptr(flags), _stream(stream)))


def rt_magnification(cosmo, z_source: float, n_bundles: int, radius: float, rays, mu, jac=None, stream=None):
    _check(load().rt_magnification(C.byref(cosmo), float(z_source), int(n_bundles), float(radius), _dptr(rays),
                                   _dptr(mu), _dptr(jac), _stream(stream)))


def rt_flexion(cosmo, z_source: float, n_bundles: int, radius: float, rays, flex, dm=None, stream=None):
    _check(load().rt_flexion(C.byref(cosmo), float(z_source), int(n_bundles), float(radius), _dptr(rays),
                             _dptr(flex), _dptr(dm), _stream(stream)))


def rt_mu_histogram(n: int, mu, n_bins: int, log_lo: float, log_hi: float, pdf, moments, stream=None):
    _check(load().rt_mu_histogram(int(n), _dptr(mu), int(n_bins), float(log_lo), float(log_hi), _dptr(pdf),
                                  _dptr(moments), _stream(stream)))


def rt_mu_histogram_noalloc(n: int, mu, n_bins: int, log_lo: float, log_hi: float, pdf, moments, stream=None):
    _check(load().rt_mu_histogram_noalloc(int(n), _dptr(mu), int(n_bins), float(log_lo), float(log_hi), _dptr(pdf),
                                          _dptr(moments), _stream(stream)))


def rt_shear_histogram(n: int, mu, jac, n_bins: int, lo: float, hi: float, pdf, moments, stream=None):
    _check(load().rt_shear_histogram(int(n), _dptr(mu), _dptr(jac), int(n_bins), float(lo), float(hi), _dptr(pdf),
                                     _dptr(moments), _stream(stream)))


def rt_field_eval(cosmo, pset: rt_particle_set, precision: int, n: int, points, phi, grad, stream=None):
    _check(load().rt_field_eval(C.byref(cosmo), C.byref(pset), int(precision), int(n), _dptr(points), _dptr(phi),
                                _dptr(grad), _stream(stream)))


def rt_plan_count(precision: int) -> int:
    return int(load().rt_plan_count(int(precision)))


def rt_plan_describe(precision: int, plan_id: int) -> dict:
    info = rt_plan_info()
    _check(load().rt_plan_describe(int(precision), int(plan_id), C.addressof(info)))
    return {k: getattr(info, k) for k, _ in rt_plan_info._fields_}


def rt_force_plan(precision: int, plan_id: int):
    _check(load().rt_force_plan(int(precision), int(plan_id)))


def rt_set_grid_limit(max_blocks: int):
    _check(load().rt_set_grid_limit(int(max_blocks)))


def rt_autotune(cosmo, z_source: float, table: FieldTable, precision: int, step_begin: int, n_probe_steps: int,
                n_bundles: int, rays, stream=None) -> int:
    best = C.c_int32(-1)
    _check(load().rt_autotune(C.byref(cosmo), float(z_source), table.ptr, table.n, int(precision), int(step_begin),
                              int(n_probe_steps), int(n_bundles), _dptr(rays), C.addressof(best), _stream(stream)))
    return best.value


def rt_enable_timing(on: bool):
    _check(load().rt_enable_timing(1 if on else 0))


def rt_last_trace_info() -> dict:
    info = rt_trace_info()
    _check(load().rt_last_trace_info(C.addressof(info)))
    return {k: getattr(info, k) for k, _ in rt_trace_info._fields_}


def rt_sync(stream=None):
    _check(load().rt_sync(_stream(stream)))


def rt_last_error() -> str:
    return load().rt_last_error().decode()


def rt_release_caches():
    load().rt_release_caches()


def pm_grid(n: int, origin, h: float, periodic: bool = False) -> rt_pm_grid:
    return rt_pm_grid(int(n), (C.c_double * 3)(*[float(v) for v in origin]), float(h), 1 if periodic else 0)


def rt_pm_workspace_bytes(grid: rt_pm_grid) -> int:
    b = C.c_size_t(0)
    _check(load().rt_pm_workspace_bytes(C.byref(grid), C.addressof(b)))
    return int(b.value)


def rt_pm_build(pset: rt_particle_set, grid: rt_pm_grid, fields, workspace, workspace_bytes: int, stream=None):
    _check(load().rt_pm_build(C.byref(pset), C.byref(grid), _dptr(fields), _dptr(workspace), int(workspace_bytes),
                              _stream(stream)))


def rt_pm_eval(grid: rt_pm_grid, fields, n_int: int, n: int, points, phi, grad, stream=None):
    _check(load().rt_pm_eval(C.byref(grid), _dptr(fields), int(n_int), int(n), _dptr(points), _dptr(phi), _dptr(grad),
                             _stream(stream)))


def rt_trace_pm(cosmo, z_source: float, grids, fields, n_int: int, z_nodes, step_begin: int, step_end: int,
                n_bundles: int, rays, ray_flags=None, step_grid=None, stream=None):
    """grids: one rt_pm_grid or a list; fields: the matching built field tensor(s)."""
    if isinstance(grids, rt_pm_grid):
        grids, fields = [grids], [fields]
    garr = (rt_pm_grid * len(grids))(*grids)
    farr = (C.c_void_p * len(fields))(*[_dptr(f) for f in fields])
    nodes = np.ascontiguousarray(z_nodes, dtype=np.float64)
    sg = None if step_grid is None else np.ascontiguousarray(step_grid, dtype=np.int32)
    _check(load().rt_trace_pm(C.byref(cosmo), float(z_source), len(grids), C.addressof(garr), C.addressof(farr),
                              int(n_int), int(nodes.size - 1), nodes.ctypes.data,
                              None if sg is None else sg.ctypes.data, int(step_begin), int(step_end),
                              int(n_bundles), _dptr(rays), _dptr(ray_flags), _stream(stream)))


def rt_trace_pm_lambda(cosmo, z_source: float, grid: rt_pm_grid, fields, n_int: int, f_rk: float, max_steps: int,
                       n_bundles: int, rays, ray_flags=None, ray_steps=None, stream=None):
    _check(load().rt_trace_pm_lambda(C.byref(cosmo), float(z_source), C.byref(grid), _dptr(fields), int(n_int),
                                     float(f_rk), int(max_steps), int(n_bundles), _dptr(rays), _dptr(ray_flags),
                                     _dptr(ray_steps), _stream(stream)))


def rt_trace_pm_lambda_slabs(cosmo, z_source: float, grids, fields, n_int: int, slab_bounds, slab_grid,
                             f_rk: float, max_steps: int, n_bundles: int, rays, ray_flags=None, ray_steps=None,
                             stream=None):
    """grids: list of rt_pm_grid; fields: the matching built field tensors; slab_bounds [n_slabs + 1];
    slab_grid [n_slabs] (grid index per slab, -1 = no field)."""
    garr = (rt_pm_grid * len(grids))(*grids)
    farr = (C.c_void_p * len(fields))(*[_dptr(f) for f in fields])
    b = np.ascontiguousarray(slab_bounds, dtype=np.float64)
    sg = np.ascontiguousarray(slab_grid, dtype=np.int32)
    if b.size != sg.size + 1:
        raise ValueError("slab_bounds must hold one more entry than slab_grid")
    _check(load().rt_trace_pm_lambda_slabs(C.byref(cosmo), float(z_source), len(grids), C.addressof(garr),
                                           C.addressof(farr), int(n_int), int(sg.size), b.ctypes.data,
                                           sg.ctypes.data, float(f_rk), int(max_steps), int(n_bundles), _dptr(rays),
                                           _dptr(ray_flags), _dptr(ray_steps), _stream(stream)))
