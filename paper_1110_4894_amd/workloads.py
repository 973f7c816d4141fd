"""Seeded synthetic inputs for the ray-bundle lensing path.

This module only builds inputs: particle positions and masses, bundle
directions and the geometry numbers needed to place them.  It holds none of
the lensing method's arithmetic (no field sums, no geodesics, no schedules, no
magnifications), and both the GPU library and the CPU oracle consume what it
returns.  It stands in for the paper's GADGET2 simulations and fake-GADGET NFW
haloes (Sec. 4.2 and 5.1), which are not available.

Workloads (cosmology Omega_m = 0.3, Omega_Lambda = 0.7, h = 0.7 throughout):
  * ``schwarzschild``: one 1e12 Msun point mass at z_l = 0.25, z_s = 0.5;
    32 x 32 bundles at 0.5-10 Einstein radii, 1e-3 arcsec bundle radius.
  * ``nfw``: 1e5 equal-mass particles drawn from a truncated NFW halo
    (M200 = 1e14 Msun, c = 5) at z_l = 0.25; 256 x 256 bundles over +-3 r_s.
  * ``box``: a Zel'dovich-displaced periodic box (100 Mpc/h, P(k) ~ k^-1.5,
    sigma_8 = 0.8), replicated along the line of sight with random periodic
    shifts and 90-degree rotations (Sec. 5.2), 2^18 or 2^20 particles;
    128 x 128 or 512 x 512 bundles of radius 1e-3 arcsec over 1 deg.
  * ``batched``: 64 uneven fields (point-mass groups, NFW haloes, box
    sub-volumes), bundle radius 1e-3 arcsec.

Seeds: master seed 1110; each object draws from its own child of
``numpy.random.SeedSequence(seed)``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np
from scipy import integrate

MASTER_SEED = 1110
ARCSEC = math.pi / (180.0 * 3600.0)

# Geometry constants used only to place inputs (published values).
_GM_SUN = 1.32712440018e20
_C_SI = 299792458.0
_MPC = 3.0856775814913673e22
_C_KMS = 299792.458


@dataclass(frozen=True)
class Cosmology:
    omega_m: float = 0.3
    omega_lambda: float = 0.7
    h: float = 0.7

    @property
    def hubble0(self) -> float:           # Mpc^-1, c = 1
        return 100.0 * self.h / _C_KMS

    def e_of_z(self, z: float) -> float:
        return math.sqrt(self.omega_m * (1.0 + z) ** 3 + self.omega_lambda)

    def comoving(self, z: float) -> float:
        val, _ = integrate.quad(lambda x: 1.0 / self.e_of_z(x), 0.0, z, epsabs=0, epsrel=1e-13, limit=200)
        return val / self.hubble0

    def rho_crit(self, z: float = 0.0) -> float:   # Msun / Mpc^3
        G = _GM_SUN / _C_SI ** 2 / _MPC
        return 3.0 * (self.hubble0 * self.e_of_z(z)) ** 2 / (8.0 * math.pi * G)


G_OVER_C2 = _GM_SUN / _C_SI ** 2 / _MPC


@dataclass
class ParticleSetSpec:
    """One lens volume: positions [n, 3] (comoving Mpc, observer frame), masses [n]."""
    xyz: np.ndarray
    m: np.ndarray
    softening: float
    background: bool = False
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclass
class FieldSpec:
    """One independent lens field: its particle sets, bundle directions and the
    parameters from which each side builds its own step schedule."""
    name: str
    sets: List[ParticleSetSpec]
    theta: np.ndarray               # [2, n_bundles] radians (gnomonic)
    schedule: dict                  # {"z_lo", "z_hi", "n_fine", "q"} or {"uniform": n}
    replica_box: Optional[float] = None   # box length when step sets follow replicas
    meta: dict = field(default_factory=dict)

    @property
    def n_bundles(self) -> int:
        return self.theta.shape[1]


@dataclass
class Workload:
    name: str
    cosmology: Cosmology
    z_source: float
    bundle_radius: float            # radians
    fields: List[FieldSpec]
    meta: dict = field(default_factory=dict)

    @property
    def n_bundles(self) -> int:
        return sum(f.n_bundles for f in self.fields)


def _children(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# ----------------------------------------------------------------------------- compact lenses
def einstein_angle(cos: Cosmology, mass: float, z_l: float, z_s: float) -> float:
    """Point-lens Einstein angle (App. C, eq. Eangle) for placing bundles."""
    cl, cs = cos.comoving(z_l), cos.comoving(z_s)
    d_d, d_s, d_ds = cl / (1 + z_l), cs / (1 + z_s), (cs - cl) / (1 + z_s)
    return math.sqrt(4.0 * G_OVER_C2 * mass * d_ds / (d_d * d_s))


def schwarzschild(n_radii: int = 32, n_azimuth: int = 32, mass: float = 1e12, z_l: float = 0.25,
                  z_s: float = 0.5, radius_arcsec: float = 1e-3, x_min: float = 0.5, x_max: float = 10.0,
                  n_fine: int = 1000, half_width: float = 1.0, q: float = 1.1) -> Workload:
    cos = Cosmology()
    chi_l = cos.comoving(z_l)
    th_e = einstein_angle(cos, mass, z_l, z_s)
    xs = np.geomspace(x_min, x_max, n_radii)
    az = 2 * np.pi * (np.arange(n_azimuth) + 0.5) / n_azimuth
    xx, aa = np.meshgrid(xs, az, indexing="ij")
    theta = np.stack([(xx * th_e * np.cos(aa)).ravel(), (xx * th_e * np.sin(aa)).ravel()])
    pset = ParticleSetSpec(xyz=np.array([[0.0, 0.0, chi_l]]), m=np.array([mass]), softening=0.0)
    f = FieldSpec("point-mass", [pset], theta,
                  {"z_lo": chi_l - half_width, "z_hi": chi_l + half_width, "n_fine": n_fine, "q": q},
                  meta={"x": xx.ravel(), "theta_E": th_e, "chi_l": chi_l, "mass": mass, "z_l": z_l})
    return Workload("schwarzschild", cos, z_s, radius_arcsec * ARCSEC, [f], meta={"theta_E": th_e})


def nfw_radii(rng: np.random.Generator, n: int, conc: float) -> np.ndarray:
    """Radii (units of r_s) from the NFW enclosed-mass profile truncated at c,
    by inverting m(x) = ln(1+x) - x/(1+x) with bisection."""
    mfun = lambda x: np.log1p(x) - x / (1.0 + x)
    target = rng.random(n) * mfun(conc)
    lo, hi = np.zeros(n), np.full(n, conc)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        below = mfun(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)


def nfw_halo_spec(cos: Cosmology, m200: float, conc: float, z_l: float, n_part: int, rng: np.random.Generator,
                  center: Tuple[float, float, float]) -> Tuple[np.ndarray, np.ndarray, dict]:
    """Equal-mass particles of an NFW halo truncated at r200 (Sec. 4.2, eq. nfwprof),
    placed at ``center`` in comoving Mpc.  r200 uses 200 rho_c(z_l)."""
    r200 = (3.0 * m200 / (4.0 * math.pi * 200.0 * cos.rho_crit(z_l))) ** (1.0 / 3.0)   # physical Mpc
    rs = r200 / conc
    r = nfw_radii(rng, n_part, conc) * rs * (1.0 + z_l)      # comoving
    xyz = isotropic(rng, n_part) * r[:, None] + np.asarray(center)[None, :]
    m = np.full(n_part, m200 / n_part)
    return xyz, m, {"r200_phys": r200, "rs_phys": rs, "conc": conc, "m200": m200, "z_l": z_l}


def nfw(n_side: int = 256, n_part: int = 100_000, m200: float = 1e14, conc: float = 5.0, z_l: float = 0.25,
        z_s: float = 0.5, soft_phys_kpc: float = 2.0, radius_arcsec: float = 1e-3, fov_rs: float = 3.0,
        n_fine: int = 2000, q: float = 1.1, seed: int = MASTER_SEED) -> Workload:
    cos = Cosmology()
    chi_l = cos.comoving(z_l)
    (rng,) = _children(seed, 1)
    xyz, m, meta = nfw_halo_spec(cos, m200, conc, z_l, n_part, rng, (0.0, 0.0, chi_l))
    d_d = chi_l / (1 + z_l)
    half = fov_rs * meta["rs_phys"] / d_d                      # radians
    pitch = 2 * half / n_side
    g = -half + pitch * (np.arange(n_side) + 0.5)
    ty, tx = np.meshgrid(g, g, indexing="ij")
    theta = np.stack([tx.ravel(), ty.ravel()])
    r200c = meta["r200_phys"] * (1 + z_l)
    soft = soft_phys_kpc * 1e-3 * (1 + z_l)
    pset = ParticleSetSpec(xyz=xyz, m=m, softening=soft)
    meta.update(chi_l=chi_l, d_d=d_d, pitch=pitch, half=half)
    f = FieldSpec("nfw", [pset], theta,
                  {"z_lo": chi_l - r200c, "z_hi": chi_l + r200c, "n_fine": n_fine, "q": q}, meta=meta)
    return Workload("nfw", cos, z_s, radius_arcsec * ARCSEC, [f], meta=meta)


# ----------------------------------------------------------------------------- cosmological box
def _tophat(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    s = x > 1e-4
    xs = x[s]
    out[s] = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return out


def power_amplitude(n_index: float, sigma8: float, r8: float) -> float:
    """A such that P(k) = A k^n has the continuum top-hat sigma(r8) = sigma8."""
    f = lambda k: k ** (2.0 + n_index) * _tophat(k * r8) ** 2
    val, _ = integrate.quad(f, 0.0, np.inf, limit=2000)
    return sigma8 ** 2 * 2.0 * math.pi ** 2 / val


def zeldovich_positions(n_mesh: int, box: float, rng: np.random.Generator, n_index: float = -1.5,
                        sigma8: float = 0.8, h: float = 0.7) -> np.ndarray:
    """Lattice of n_mesh^3 points displaced by the Zel'dovich field of a seeded
    Gaussian density with P(k) = A k^n, periodic wrap into [0, box)^3."""
    amp = power_amplitude(n_index, sigma8, 8.0 / h)
    white = rng.standard_normal((n_mesh,) * 3)
    wk = np.fft.rfftn(white)
    kf = 2 * np.pi / box
    kx = np.fft.fftfreq(n_mesh, d=1.0 / n_mesh) * kf
    kz = np.fft.rfftfreq(n_mesh, d=1.0 / n_mesh) * kf
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[0, 0, 0] = 1.0
    pk = amp * k2 ** (n_index / 2.0)
    dk = wk * np.sqrt(pk * n_mesh ** 3 / box ** 3)
    dk[0, 0, 0] = 0.0
    cell = box / n_mesh
    q = (np.arange(n_mesh) + 0.5) * cell
    QX, QY, QZ = np.meshgrid(q, q, q, indexing="ij")
    pos = np.empty((n_mesh ** 3, 3))
    for i, (K, Q) in enumerate(((KX, QX), (KY, QY), (KZ, QZ))):
        s = np.fft.irfftn(1j * K / k2 * dk, s=(n_mesh,) * 3, axes=(0, 1, 2))
        pos[:, i] = np.mod((Q + s).ravel(), box)
    return pos


def proper_rotations() -> List[np.ndarray]:
    """The 24 signed permutation matrices with determinant +1."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3))
            for i, p in enumerate(perm):
                R[i, p] = signs[i]
            if np.linalg.det(R) > 0:
                out.append(R)
    return out


def box_replicas(pos: np.ndarray, box: float, n_rep: int, rng: np.random.Generator) -> List[np.ndarray]:
    """Copies of a periodic box stacked along the line of sight (Sec. 5.2): each is
    shifted periodically at random, rotated by one of the 24 proper 90-degree
    rotations about the box centre, and placed at x, y in [-L/2, L/2), z in
    [rL, (r+1)L)."""
    rots = proper_rotations()
    reps = []
    for r in range(n_rep):
        shift = rng.uniform(0.0, box, 3)
        p = np.mod(pos + shift[None, :], box) - 0.5 * box
        R = rots[int(rng.integers(0, len(rots)))]
        p = p @ R.T
        p = np.mod(p + 0.5 * box, box)          # back into [0, L) after rotation
        p[:, 0] -= 0.5 * box
        p[:, 1] -= 0.5 * box
        p[:, 2] += r * box
        reps.append(p)
    return reps


def box(n_part_log2: int = 18, n_side: int = 128, z_s: float = 0.5, fov_deg: float = 1.0,
        radius_arcsec: float = 1e-3, n_steps: int = 2000, box_mpc_h: float = 100.0,
        soft_kpc_h: float = 50.0, seed: int = MASTER_SEED, n_replicas: Optional[int] = None) -> Workload:
    cos = Cosmology()
    L = box_mpc_h / cos.h
    chi_s = cos.comoving(z_s)
    n_rep = n_replicas if n_replicas is not None else int(math.ceil(chi_s / L))
    rng_field, rng_half, rng_rep = _children(seed, 3)
    if n_part_log2 % 3 == 0:
        n_mesh = 2 ** (n_part_log2 // 3)
        pos = zeldovich_positions(n_mesh, L, rng_field, h=cos.h)
    else:
        # a seeded random subset of the next cubic lattice (e.g. half of 128^3 for 2^20)
        n_mesh = 2 ** ((n_part_log2 + 2) // 3)
        pos = zeldovich_positions(n_mesh, L, rng_field, h=cos.h)
        keep = rng_half.choice(pos.shape[0], size=2 ** n_part_log2, replace=False)
        pos = pos[np.sort(keep)]
    n = pos.shape[0]
    m_p = cos.omega_m * cos.rho_crit(0.0) * L ** 3 / n
    reps = box_replicas(pos, L, n_rep, rng_rep)
    soft = soft_kpc_h * 1e-3 / cos.h
    sets = [ParticleSetSpec(xyz=p, m=np.full(n, m_p), softening=soft, background=True,
                            lo=(-0.5 * L, -0.5 * L, r * L), hi=(0.5 * L, 0.5 * L, (r + 1) * L))
            for r, p in enumerate(reps)]
    half = 0.5 * fov_deg * math.pi / 180.0
    pitch = 2 * half / n_side
    g = -half + pitch * (np.arange(n_side) + 0.5)
    ty, tx = np.meshgrid(g, g, indexing="ij")
    theta = np.stack([tx.ravel(), ty.ravel()])
    f = FieldSpec("box", sets, theta, {"uniform": n_steps}, replica_box=L,
                  meta={"L": L, "n_mesh": n_mesh, "m_p": m_p, "n_rep": n_rep})
    return Workload("box", cos, z_s, radius_arcsec * ARCSEC, [f], meta={"L": L, "m_p": m_p})


def empty(n_bundles: int = 16, z_s: float = 0.5, radius_arcsec: float = 1e-3, n_steps: int = 200,
          seed: int = MASTER_SEED) -> Workload:
    """No mass at all: bundles at random directions within 10 arcmin."""
    cos = Cosmology()
    (rng,) = _children(seed, 1)
    theta = rng.uniform(-1, 1, (2, n_bundles)) * 10 * 60 * ARCSEC
    f = FieldSpec("empty", [], theta, {"uniform": n_steps})
    return Workload("empty", cos, z_s, radius_arcsec * ARCSEC, [f])


def subsample(w: Workload, stride: int, offset: int = 0, max_bundles: Optional[int] = None) -> Workload:
    """Every ``stride``-th bundle of every field (same particles and schedules)."""
    fields = []
    for f in w.fields:
        th = f.theta[:, offset::stride]
        if max_bundles is not None:
            th = th[:, :max_bundles]
        meta = dict(f.meta)
        for k, v in f.meta.items():
            if isinstance(v, np.ndarray) and v.shape == (f.n_bundles,):
                meta[k] = v[offset::stride][: th.shape[1]]
        fields.append(FieldSpec(f.name, f.sets, np.ascontiguousarray(th), f.schedule, f.replica_box, meta))
    return Workload(w.name, w.cosmology, w.z_source, w.bundle_radius, fields, dict(w.meta))


# ----------------------------------------------------------------------------- batched uneven fields
def batched(n_sides=(64, 128, 256), side_override: Optional[int] = None, z_s: float = 0.5,
            radius_arcsec: float = 1e-3, n_fine: int = 500, q: float = 1.1, seed: int = MASTER_SEED,
            n_point: int = 16, n_nfw: int = 32, n_box: int = 16, nfw_np_range=(10_000, 1_000_000),
            box_sub_mpc_h: float = 25.0) -> Workload:
    """64 independent lens fields of very uneven cost, in this order:
    16 groups of 1-8 point masses (log-uniform 1e11-1e13 Msun, z_l ~ U[0.1, 0.4]);
    32 NFW haloes (N_p log-uniform in [1e4, 1e6], M200 log-uniform in [1e13, 1e15] Msun,
    c ~ U[4, 8], z_l ~ U[0.1, 0.4], softening 2 kpc physical);
    16 sub-volumes (25 Mpc/h cubes) cut from the 2^20-particle Zel'dovich box and
    placed at a seeded distance, with their uniform-cuboid background.
    Each field gets a seeded 64^2, 128^2 or 256^2 bundle grid (``side_override``
    replaces the side, to run reduced versions) and 500 fine steps across its mass."""
    cos = Cosmology()
    chi_s = cos.comoving(z_s)
    rng_master = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    rngs = [np.random.default_rng(s) for s in np.random.SeedSequence(seed + 5).spawn(n_point + n_nfw + n_box + 1)]
    fields: List[FieldSpec] = []

    def grid(half: float, side: int):
        pitch = 2 * half / side
        g = -half + pitch * (np.arange(side) + 0.5)
        ty, tx = np.meshgrid(g, g, indexing="ij")
        return np.stack([tx.ravel(), ty.ravel()])

    def pick_side(r):
        s = int(r.choice(np.asarray(n_sides)))
        return side_override if side_override is not None else s

    for i in range(n_point):
        r = rngs[i]
        k = int(r.integers(1, 9))
        masses = 10 ** r.uniform(11, 13, k)
        z_l = r.uniform(0.1, 0.4)
        chi_l = cos.comoving(z_l)
        th_e = einstein_angle(cos, masses.sum(), z_l, z_s)
        pos = np.zeros((k, 3))
        pos[:, :2] = r.normal(size=(k, 2)) * th_e * chi_l
        pos[:, 2] = chi_l + r.uniform(-0.5, 0.5, k)
        side = pick_side(r)
        half = 3 * th_e
        fields.append(FieldSpec("points-%d" % i, [ParticleSetSpec(pos, masses, 0.0)], grid(half, side),
                                {"z_lo": chi_l - 1.0, "z_hi": chi_l + 1.0, "n_fine": n_fine, "q": q},
                                meta={"kind": "points", "n": k}))
    lo_np, hi_np = nfw_np_range
    for i in range(n_nfw):
        r = rngs[n_point + i]
        n_part = int(round(10 ** r.uniform(np.log10(lo_np), np.log10(hi_np))))
        m200 = 10 ** r.uniform(13, 15)
        conc = r.uniform(4, 8)
        z_l = r.uniform(0.1, 0.4)
        chi_l = cos.comoving(z_l)
        xyz, m, meta = nfw_halo_spec(cos, m200, conc, z_l, n_part, r, (0.0, 0.0, chi_l))
        d_d = chi_l / (1 + z_l)
        r200c = meta["r200_phys"] * (1 + z_l)
        side = pick_side(r)
        half = 3 * meta["rs_phys"] / d_d
        fields.append(FieldSpec("nfw-%d" % i, [ParticleSetSpec(xyz, m, 2e-3 * (1 + z_l))], grid(half, side),
                                {"z_lo": chi_l - r200c, "z_hi": chi_l + r200c, "n_fine": n_fine, "q": q},
                                meta=dict(meta, kind="nfw", n=n_part)))
    # the parent box of the sub-volumes: 2^20 particles of the 128^3 Zel'dovich field
    L = 100.0 / cos.h
    r_box = rngs[-1]
    pos = zeldovich_positions(128, L, r_box, h=cos.h)
    keep = r_box.choice(pos.shape[0], size=2 ** 20, replace=False)
    pos = pos[np.sort(keep)]
    m_p = cos.omega_m * cos.rho_crit(0.0) * L ** 3 / pos.shape[0]
    sub = box_sub_mpc_h / cos.h
    n_cells = int(round(L / sub))
    for i in range(n_box):
        r = rngs[n_point + n_nfw + i]
        cx, cy, cz = (int(v) for v in r.integers(0, n_cells, 3))
        lo = np.array([cx, cy, cz]) * sub
        sel = np.all((pos >= lo) & (pos < lo + sub), axis=1)
        p = pos[sel] - lo - 0.5 * sub                 # centred cube
        z0 = r.uniform(0.2, 0.8) * chi_s              # near face of the slab
        p[:, 2] += z0 + 0.5 * sub
        side = pick_side(r)
        half = 0.4 * sub / (z0 + sub)                 # 0.8 x the cube's angular width at its far face
        fields.append(FieldSpec("box-%d" % i, [ParticleSetSpec(p, np.full(len(p), m_p), 0.05 / cos.h, True,
                                                               (-0.5 * sub, -0.5 * sub, z0),
                                                               (0.5 * sub, 0.5 * sub, z0 + sub))],
                                grid(half, side), {"z_lo": z0, "z_hi": z0 + sub, "n_fine": n_fine, "q": q},
                                meta={"kind": "box", "n": int(len(p))}))
    return Workload("batched", cos, z_s, radius_arcsec * ARCSEC, fields, meta={"chi_s": chi_s})
