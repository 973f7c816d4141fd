"""GPU parity of rt_flexion (Sec. 6: flexion through ray bundles) against the oracle's
least-squares ring fit: on the same seeded source-plane rays, and through whole traces of a
point lens (GPU trace and flexion against the oracle's trace and flexion)."""
import math

import numpy as np
import pytest
import torch

import oracle as orc
from oracle import flexion as ofx
from paper_1110_4894_amd import rt
from tests.oracle_run import oracle_run
from tests.test_oracle_geodesic import _point_mass_workload

pytestmark = pytest.mark.gpu

RING = np.array([[math.cos(2 * math.pi * k / 8), math.sin(2 * math.pi * k / 8)] for k in range(8)])


def _synthetic_rays(nb, seed, chi_s, radius):
    """Seeded source-plane rays: per bundle a random anchor and a random map about it of first,
    second and third order (the sizes of a weakly lensed 1e-3 arcsec bundle: second-order part
    ~1e-4 of the ring offsets)."""
    rng = np.random.default_rng(seed)
    anchor = rng.normal(size=(2, nb)) * 0.01 * chi_s
    A = np.eye(2)[:, :, None] + 0.05 * rng.normal(size=(2, 2, nb))
    D = rng.normal(size=(2, 2, 2, nb)) * 2e4
    D = 0.5 * (D + D.transpose(0, 2, 1, 3))
    C = rng.normal(size=(2, 2, 2, 2, nb)) * 1e9
    rays = np.zeros((8, 9 * nb))
    rays[1, 0::9], rays[2, 0::9] = anchor
    for k, e in enumerate(RING):
        d = radius * e
        off = (np.einsum("ijb,j->ib", A, d) + 0.5 * np.einsum("ijlb,j,l->ib", D, d, d)
               + np.einsum("ijlmb,j,l,m->ib", C, d, d, d) / 6.0)
        rays[1, 1 + k::9] = anchor[0] + chi_s * off[0]
        rays[2, 1 + k::9] = anchor[1] + chi_s * off[1]
    return rays


def _gpu_flexion(cosmo, z_s, radius, rays):
    dev = torch.device("cuda")
    nb = rays.shape[1] // 9
    R = torch.from_numpy(rays).to(dev)
    flex = torch.full((4, nb), float("nan"), dtype=torch.float64, device=dev)
    dm = torch.full((6, nb), float("nan"), dtype=torch.float64, device=dev)
    rt.rt_flexion(cosmo, z_s, nb, radius, R, flex, dm)
    torch.cuda.synchronize()
    return flex.cpu().numpy(), dm.cpu().numpy()


@pytest.mark.parametrize("nb", [1, 7, 29, 1001])
def test_flexion_matches_oracle_on_the_same_rays(nb):
    print("    [flexion] %d synthetic bundles" % nb, flush=True)
    c = rt.cosmology()
    z_s = 0.5
    chi_s = rt.rt_comoving_distance(c, z_s)
    radius = 1e-3 * math.pi / 180 / 3600
    rays = _synthetic_rays(nb, 100 + nb, chi_s, radius)
    flex, dm = _gpu_flexion(c, z_s, radius, rays)
    F, G, Dm, _ = ofx.bundle_flexion(chi_s, rays, radius)
    scale = np.abs(Dm).max(axis=0)
    assert np.all(np.isfinite(flex)) and np.all(np.isfinite(dm))
    assert np.all(np.abs(dm - Dm) <= 1e-8 * scale)
    assert np.all(np.abs(flex[:2] - F) <= 1e-8 * scale)
    assert np.all(np.abs(flex[2:] - G) <= 1e-8 * scale)


def test_flexion_full_size_sampled():
    """All 262144 bundles of a 512 x 512 grid in one launch: every output finite, 512 sampled
    bundles against the oracle."""
    c = rt.cosmology()
    z_s = 0.5
    chi_s = rt.rt_comoving_distance(c, z_s)
    radius = 1e-3 * math.pi / 180 / 3600
    nb = 512 * 512
    print("    [flexion] %d synthetic bundles, full grid" % nb, flush=True)
    rays = _synthetic_rays(nb, 7, chi_s, radius)
    flex, dm = _gpu_flexion(c, z_s, radius, rays)
    assert np.all(np.isfinite(flex)) and np.all(np.isfinite(dm))
    idx = np.random.default_rng(1).choice(nb, 512, replace=False)
    sub = rays.reshape(8, nb, 9)[:, idx].reshape(8, -1)
    F, G, Dm, _ = ofx.bundle_flexion(chi_s, sub, radius)
    scale = np.abs(Dm).max(axis=0)
    assert np.all(np.abs(dm[:, idx] - Dm) <= 1e-8 * scale)
    assert np.all(np.abs(flex[2:, idx] - G) <= 1e-8 * scale)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_traced_point_lens_flexion_matches_oracle(precision):
    """A point lens (Sec. 4.1) at x = theta / theta_E = 1.2 ... 5, bundles of radius 0.01 theta_E:
    the GPU trace and rt_flexion against the oracle's trace and fit (G and F relative to |G|);
    both within 1e-4 of the thin-lens G = 4 theta_E^2 / conj(theta)^3."""
    from paper_1110_4894_amd.runner import GpuRun
    xs = [1.2, 1.5, 2.0, 3.0, 5.0]
    th_e = _point_mass_workload([1.5]).fields[0].meta["theta_E"]
    w = _point_mass_workload(xs, radius_arcsec=0.01 * th_e * 180 / math.pi * 3600)
    print("    [flexion] point lens, %s trace" % precision, flush=True)
    g = GpuRun(w)
    out = g.run(rt.RT_FP64 if precision == "fp64" else rt.RT_FP32_KAHAN)
    assert not out["flags"].any()
    flex, dm = _gpu_flexion(g.cosmo, w.z_source, w.bundle_radius, out["rays"])
    r = oracle_run(w)
    F, G, Dm, _ = ofx.bundle_flexion(r["chi_s"], r["rays"], w.bundle_radius)
    gn = np.hypot(*G)
    tol = 1e-7 if precision == "fp64" else 1e-4
    assert np.all(np.hypot(*(flex[2:] - G)) <= tol * gn)
    assert np.all(np.hypot(*(flex[:2] - F)) <= tol * gn)
    th = r["theta"]
    tn, ph = np.linalg.norm(th, axis=0), np.arctan2(th[1], th[0])
    want = 4 * th_e ** 2 / tn ** 3 * np.stack([np.cos(3 * ph), np.sin(3 * ph)])
    assert np.all(np.hypot(*(flex[2:] - want)) <= 1e-4 * np.hypot(*want))
