"""Run a workload through the CPU oracle (test infrastructure).

The oracle builds its own schedules, replica selection and source distance;
only the particle positions, masses and bundle directions come from the
shared input generators.
"""
from __future__ import annotations

import numpy as np

import oracle as orc
from paper_1110_4894_amd.workloads import Workload


def oracle_cosmo(w: Workload):
    c = w.cosmology
    return orc.cosmo(c.omega_m, c.omega_lambda, c.h)


def oracle_schedule(chi_s: float, sched: dict) -> np.ndarray:
    if "uniform" in sched:
        return orc.make_schedule(chi_s, 0.0, chi_s, int(sched["uniform"]), 1.0)
    return orc.make_schedule(chi_s, sched["z_lo"], sched["z_hi"], int(sched["n_fine"]), sched["q"])


def oracle_fields(w: Workload):
    c = oracle_cosmo(w)
    chi_s = orc.comoving_distance(c, w.z_source)
    fields, thetas, off = [], [], 0
    for f in w.fields:
        nodes = oracle_schedule(chi_s, f.schedule)
        if not f.sets:
            step_set = np.full(len(nodes) - 1, -1, dtype=np.int32)
        elif f.replica_box is not None:
            step_set = orc.replica_step_sets(nodes, f.replica_box, len(f.sets))
        else:
            step_set = np.zeros(len(nodes) - 1, dtype=np.int32)
        sets = [orc.ParticleSet(xyz=s.xyz, m=s.m, softening=s.softening, background=s.background, lo=s.lo,
                                hi=s.hi) for s in f.sets]
        fields.append(orc.Field(sets, nodes, step_set, off, f.n_bundles))
        thetas.append(f.theta)
        off += f.n_bundles
    theta = np.ascontiguousarray(np.concatenate(thetas, axis=1))
    return c, chi_s, fields, theta


def oracle_run(w: Workload, n_threads: int = 0, step_begin: int = 0, step_end: int = 2 ** 31 - 1):
    """Returns dict(rays, flags, mu, jac, chi_s, fields, theta)."""
    c, chi_s, fields, theta = oracle_fields(w)
    rays = orc.build_bundles(c, fields, theta, w.bundle_radius)
    rays, flags = orc.trace(c, fields, rays, step_begin, step_end, n_threads=n_threads)
    mu, jac = orc.magnification(chi_s, rays, w.bundle_radius)
    return dict(rays=rays, flags=flags, mu=mu, jac=jac, chi_s=chi_s, fields=fields, theta=theta, cosmo=c)
