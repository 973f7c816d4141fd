"""Drive a workload through librt: upload inputs, build the schedules with the
library's own host routines, and call the entry points in order.

Orchestration only: schedules, replica selection, bundles, tracing,
magnification and the muPDF are all computed by librt.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from . import rt
from .workloads import Workload


class GpuRun:
    def __init__(self, w: Workload, device: str = "cuda", uploads: Optional[Dict[int, torch.Tensor]] = None):
        self.w = w
        self.device = torch.device(device)
        c = w.cosmology
        self.cosmo = rt.cosmology(c.omega_m, c.omega_lambda, c.h)
        self.chi_s = rt.rt_comoving_distance(self.cosmo, w.z_source)
        self.radius = w.bundle_radius
        uploaded: Dict[int, torch.Tensor] = uploads if uploads is not None else {}
        fields = []
        thetas = []
        off = 0
        self.n_steps = []
        for f in w.fields:
            sched = f.schedule
            if "uniform" in sched:
                nodes = rt.rt_make_schedule(self.chi_s, 0.0, self.chi_s, int(sched["uniform"]), 1.0)
            else:
                nodes = rt.rt_make_schedule(self.chi_s, sched["z_lo"], sched["z_hi"], int(sched["n_fine"]),
                                            sched["q"])
            if not f.sets:
                step_set = np.full(len(nodes) - 1, -1, dtype=np.int32)
            elif f.replica_box is not None:
                step_set = rt.rt_replica_step_sets(nodes, f.replica_box, len(f.sets))
            else:
                step_set = np.zeros(len(nodes) - 1, dtype=np.int32)
            sets = []
            for s in f.sets:
                key = id(s.xyz)
                if key not in uploaded:
                    host = np.ascontiguousarray(np.concatenate([s.xyz.T, s.m[None, :]], axis=0), dtype=np.float64)
                    uploaded[key] = torch.from_numpy(host).to(self.device)
                sets.append({"xyzm": uploaded[key], "softening": s.softening, "background": s.background,
                             "lo": tuple(float(v) for v in s.lo), "hi": tuple(float(v) for v in s.hi)})
            fields.append({"sets": sets, "z_nodes": nodes, "step_set": step_set, "bundle_offset": off,
                           "n_bundles": f.n_bundles})
            self.n_steps.append(len(nodes) - 1)
            thetas.append(f.theta)
            off += f.n_bundles
        self.fields = fields
        self.table = rt.FieldTable(fields)
        self.n_bundles = off
        self.theta = torch.from_numpy(np.ascontiguousarray(np.concatenate(thetas, axis=1))).to(self.device)
        self.rays = torch.empty((8, 9 * off), dtype=torch.float64, device=self.device)
        self.flags = torch.zeros(9 * off, dtype=torch.uint8, device=self.device)
        self.mu = torch.empty(off, dtype=torch.float64, device=self.device)
        self.jac = torch.empty((4, off), dtype=torch.float64, device=self.device)

    def set_theta(self, theta):
        """Point the same fields at another set of bundle directions (device copy)."""
        self.theta.copy_(theta)

    @property
    def max_steps(self) -> int:
        return max(self.n_steps)

    def interactions(self, step_begin: int = 0, step_end: int = 2 ** 31 - 1) -> float:
        tot = 0.0
        for f in self.fields:
            ss = f["step_set"][step_begin:step_end]
            npart = np.array([f["sets"][s]["xyzm"].shape[1] if s >= 0 else 0 for s in ss], dtype=np.float64)
            tot += 9.0 * f["n_bundles"] * 4.0 * npart.sum()
        return tot

    def build_bundles(self, stream=None):
        rt.rt_build_bundles(self.cosmo, self.table, self.n_bundles, self.theta, self.radius, self.rays, stream)
        self.flags.zero_()

    def trace(self, precision: int, step_begin: int = 0, step_end: int = 2 ** 31 - 1, stream=None):
        rt.rt_trace(self.cosmo, self.w.z_source, self.table, precision, step_begin, step_end, self.n_bundles,
                    self.rays, self.flags, stream)

    def magnification(self, stream=None):
        rt.rt_magnification(self.cosmo, self.w.z_source, self.n_bundles, self.radius, self.rays, self.mu, self.jac,
                            stream)

    def histogram(self, n_bins: int = 200, log_lo: float = -0.1, log_hi: float = 0.3, stream=None):
        pdf = torch.empty(n_bins, dtype=torch.float64, device=self.device)
        mom = torch.empty(6, dtype=torch.float64, device=self.device)
        rt.rt_mu_histogram(self.n_bundles, self.mu, n_bins, log_lo, log_hi, pdf, mom, stream)
        return pdf, mom

    def run(self, precision: int, step_begin: int = 0, step_end: int = 2 ** 31 - 1) -> dict:
        self.build_bundles()
        self.trace(precision, step_begin, step_end)
        self.magnification()
        torch.cuda.synchronize()
        return {"rays": self.rays.cpu().numpy(), "flags": self.flags.cpu().numpy(), "mu": self.mu.cpu().numpy(),
                "jac": self.jac.cpu().numpy(), "chi_s": self.chi_s}
