"""Benchmark of the ray-bundle lensing hot path on one MI355X.

Workload: the NFW halo (1e5 equal-mass particles from an NFW halo with
M200 = 1e14 Msun, c = 5, truncated at r200, softening 2 kpc physical, z_l = 0.25,
z_s = 0.5) with 256 x 256 bundles (anchor + 8 rays, radius 1e-3 arcsec) over
+-3 r_s and 2000 fine RK4 steps across the halo (2237 steps in all).

One step = one pass of the whole path over one batch of the bundle grid: a
band of 7168 consecutive bundles (64 512 rays) of the row-major grid, sized to
two full rounds of the trace kernel's resident workgroups: bundle
construction, tracing with FP32 pair terms + Kahan sums and FP64 integration
(one captured graph with the persistent kernel), magnification and the muPDF.
Steps walk through the grid band after band.  Inputs (particles, bundle
directions) are resident in HBM before the timed region.

Untimed: every second bundle of the first timed band is also traced in FP64
(4096 bundles, enough to fill the GPU) to give the mixed-vs-FP64 mu error and
the FP64 throughput; the CPU oracle is timed on two bundles of the batch (full
schedule, all particles).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray-particle interactions/s and bundles/s at μ err ≤1e-4 vs FP64 (mixed vs FP64)"
PEAK_FP32 = 157.3      # TFLOP/s, MI355X FP32 vector (published)
# HBM bytes per launch of the FP32 trace kernel on this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs scaled by a 1 GiB copy (factors 2.0 and 1.0),
# keyed by the sha256 prefix of the kernel source they were taken with.
MEASURED_TRAFFIC = {"4c91bd822f7f7084": {"read": 791209081351.7532, "write": 309593045824.0,
                                         "summary": "profiles/trace_kernel_fp32_nfw1e5_band7168.md"}}
PEAK_FP64 = 78.6       # TFLOP/s, MI355X FP64 vector (published)
FLOP_PER_INTERACTION = 20.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--band", type=int, default=7168,
                   help="bundles per step: 7168 bundles = 1024 groups of 7 bundles, i.e. two full rounds of the "
                        "512 workgroups that the trace kernel keeps resident on 256 CUs")
    p.add_argument("--n-side", type=int, default=256)
    p.add_argument("--n-part", type=int, default=100_000)
    p.add_argument("--fp64-stride", type=int, default=2, help="every k-th bundle of one band traced in FP64")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-autotune", action="store_true")
    p.add_argument("--cpu-bundles", type=int, default=2)
    p.add_argument("--plan", type=int, default=-1, help="force a trace plan (skips the autotuner)")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="only copy a buffer of this many MiB (HBM counter calibration) and exit")
    return p.parse_args()


def traffic_bytes(band):
    """Measured HBM bytes per trace launch, or None when the kernel source has changed
    since the counters were taken (or the batch differs from the profiled one)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1110_4894_amd", "csrc", "rt_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    m = MEASURED_TRAFFIC.get(sha)
    if m is None or band != 7168:
        return None
    return m["read"] + m["write"]


def mu_stats(mu, ref):
    mu, ref = np.asarray(mu), np.asarray(ref)
    rel = np.abs(mu - ref) / np.abs(ref)
    cond = np.abs(mu - ref) / (np.abs(ref) * np.maximum(1.0, np.abs(ref)))
    weak = np.abs(ref - 1) < 0.5
    q = lambda a, p: float(np.percentile(a, p)) if a.size else 0.0
    return {"max_rel": float(rel.max()), "p99_rel": q(rel, 99), "p50_rel": q(rel, 50),
            "max_rel_weak": float(rel[weak].max()) if weak.any() else 0.0,
            "max_cond": float(cond.max()), "max_inv_mu": float(np.max(np.abs(1 / mu - 1 / ref))),
            "n": int(mu.size), "n_weak": int(weak.sum()), "max_abs_mu": float(np.abs(ref).max())}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this path is measured per GPU (bundles shard across GPUs "
              "with no communication while tracing); --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1110_4894_amd import rt, workloads
    from paper_1110_4894_amd.runner import GpuRun

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}), flush=True)
        return
    rt.load()

    t_setup = time.time()
    w = workloads.nfw(n_side=a.n_side, n_part=a.n_part)
    f = w.fields[0]
    nb_all = f.n_bundles
    band = a.band
    n_bands = -(-nb_all // band)
    # consecutive bands of the row-major bundle grid, wrapping around at its end
    bands = [np.ascontiguousarray(f.theta[:, (np.arange(i * band, (i + 1) * band) % nb_all)])
             for i in range(n_bands)]
    w_batch = workloads.Workload(w.name, w.cosmology, w.z_source, w.bundle_radius,
                                 [workloads.FieldSpec(f.name, f.sets, bands[0], f.schedule, f.replica_box, {})])
    uploads = {}
    g = GpuRun(w_batch, uploads=uploads)
    theta_dev = [torch.from_numpy(b).to(dev) for b in bands]
    stream = torch.cuda.current_stream()
    n_steps_path = g.max_steps
    inter_per_step = g.interactions()
    print("setup: %d bundles per step, %d RK4 steps, %d particles, %.3e interactions per step (%.1f s)"
          % (band, n_steps_path, a.n_part, inter_per_step, time.time() - t_setup), file=sys.stderr, flush=True)

    tuned = None
    if a.plan >= 0:
        rt.rt_force_plan(rt.RT_FP32_KAHAN, a.plan)
        tuned = a.plan
    elif not a.no_autotune:
        g.build_bundles()
        mid = n_steps_path // 2
        tuned = rt.rt_autotune(g.cosmo, w.z_source, g.table, rt.RT_FP32_KAHAN, mid, 6, g.n_bundles, g.rays)
        print("autotune: plan %d %s" % (tuned, rt.rt_plan_describe(rt.RT_FP32_KAHAN, tuned)), file=sys.stderr,
              flush=True)

    def one_step(i):
        g.set_theta(theta_dev[i % n_bands])
        g.build_bundles()
        g.trace(rt.RT_FP32_KAHAN)
        g.magnification()
        return g.histogram()

    rt.rt_enable_timing(True)
    for i in range(a.warmup):
        one_step(i)
        torch.cuda.synchronize()
        print("warmup step %d done" % i, file=sys.stderr, flush=True)

    kernel_ms = []
    mu32 = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        one_step(a.warmup + i)
        info = rt.rt_last_trace_info()      # waits for this step's trace graph (events on its stream)
        kernel_ms.append(info["kernel_ms"])
        mu32[(a.warmup + i) % n_bands] = g.mu.clone()
        print("step %d: trace %.1f ms, plan %d, grid %d, graph reused %d" % (
            i, info["kernel_ms"], info["plan_id"], info["grid_blocks"], info["graph_reused"]), file=sys.stderr,
            flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rt.rt_enable_timing(False)
    elapsed = t1 - t0
    total_inter = inter_per_step * a.steps
    value = total_inter / elapsed
    bundles_per_s = band * a.steps / elapsed
    ms_per_step = 1e3 * elapsed / a.steps
    k_ms = float(np.mean(kernel_ms))
    achieved = FLOP_PER_INTERACTION * inter_per_step / (k_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value": value, "unit": "ray-particle interactions/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "nfw-halo 1e5 particles (M200 1e14 Msun, c 5, z_l 0.25, z_s 0.5), 256x256 "
                               "bundles over +-3 r_s, r_b 1e-3 arcsec, 2000 fine RK4 steps (%d in all); "
                               "one step = one band of %d consecutive bundles" % (n_steps_path, band),
                   "bundles_per_step": band, "rays_per_step": 9 * band, "rk4_steps": n_steps_path,
                   "particles": a.n_part, "precision": "fp32-kahan field, fp64 integration",
                   "parallelism": "single GPU", "plan": tuned},
        "bundles_per_s": bundles_per_s,
        "interactions_per_step": inter_per_step,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic_bytes(band),
                     "traffic_unit": "HBM bytes per launch (read + write)",
                     "kernel": "trace_kernel (fp32)", "kernel_ms": k_ms,
                     "flop_per_interaction": FLOP_PER_INTERACTION},
    }

    # ---------------------------------------------------------------- FP64 reference on a subsample
    if not a.no_fp64:
        errs = []
        f64_ms, f64_inter = [], 0.0
        for bi, m32 in sorted(mu32.items())[:1]:
            sub = np.ascontiguousarray(bands[bi][:, ::a.fp64_stride])
            ws = workloads.Workload(w.name, w.cosmology, w.z_source, w.bundle_radius,
                                    [workloads.FieldSpec(f.name, f.sets, sub, f.schedule, f.replica_box, {})])
            gs = GpuRun(ws, uploads=uploads)
            gs.build_bundles()
            rt.rt_enable_timing(True)
            gs.trace(rt.RT_FP64)
            info = rt.rt_last_trace_info()
            rt.rt_enable_timing(False)
            gs.magnification()
            torch.cuda.synchronize()
            f64_ms.append(info["kernel_ms"])
            f64_inter += gs.interactions()
            errs.append((m32.cpu().numpy()[::a.fp64_stride], gs.mu.cpu().numpy()))
        m32c = np.concatenate([e[0] for e in errs])
        m64c = np.concatenate([e[1] for e in errs])
        result["mu_err_vs_fp64"] = mu_stats(m32c, m64c)
        fp64_rate = f64_inter / (sum(f64_ms) * 1e-3)
        result["fp64"] = {"interactions_per_s": fp64_rate, "bundles": int(m64c.size),
                          "tflops": FLOP_PER_INTERACTION * fp64_rate / 1e12,
                          "frac_of_fp64_peak": FLOP_PER_INTERACTION * fp64_rate / 1e12 / PEAK_FP64,
                          "mixed_speedup": (FLOP_PER_INTERACTION * inter_per_step / (k_ms * 1e-3)) /
                                           (FLOP_PER_INTERACTION * fp64_rate)}
        print("fp64 reference: %s" % json.dumps(result["mu_err_vs_fp64"]), file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- CPU oracle baseline
    if not a.no_cpu_baseline:
        import oracle as orc
        from tests.oracle_run import oracle_fields
        sub = np.ascontiguousarray(bands[0][:, : a.cpu_bundles * 37: 37][:, : a.cpu_bundles])
        ws = workloads.Workload(w.name, w.cosmology, w.z_source, w.bundle_radius,
                                [workloads.FieldSpec(f.name, f.sets, sub, f.schedule, f.replica_box, {})])
        c, chi_s, fields, theta = oracle_fields(ws)
        rays = orc.build_bundles(c, fields, theta, ws.bundle_radius)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        tc0 = time.perf_counter()
        orc.trace(c, fields, rays, n_threads=threads)
        tc = time.perf_counter() - tc0
        n_inter = 9.0 * sub.shape[1] * 4.0 * sum(len(s.xyz) for s in f.sets) * n_steps_path
        result["cpu_baseline"] = {"value": n_inter / tc, "unit": "ray-particle interactions/s", "cores": threads,
                                  "kind": "oracle", "seconds": tc,
                                  "sample": "%d bundles (%d rays) of the first band, full %d-step schedule, all %d "
                                            "particles, FP64" % (sub.shape[1], 9 * sub.shape[1], n_steps_path,
                                                                 a.n_part)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
