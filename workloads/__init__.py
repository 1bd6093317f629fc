"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module only draws numbers: Gaussian parameters, scanner angles and
distances, detector and grid sizes, upstream gradients and measured target
images.  It holds none of the method's arithmetic (no projection, no
rectification, no splatting, no voxelisation), so the HIP path and the oracle
can both consume its output without sharing any computation.

The paper's datasets (real CT volumes projected with a CT toolbox, and the
FIPS scans) are not available; ellipsoid phantoms with the same workload shapes
stand in for them (512^2 projections over a full circle, 256^3 target volumes,
75/50/25 views, density threshold 0.05, density scale 0.15, nearest-neighbour
scales; paper Sec. 4.1 "Implementation details" and App. B).

Every draw uses ``numpy.random.default_rng(seed)`` in FP64 in a fixed order and
is cast once to FP32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Cone-beam scanner of the paper's synthetic data (App. B): source-object
# 1000 mm, source-detector 1500 mm, a 384 mm detector.  Lengths are normalised
# by UNIT_MM = R_fov / sqrt(3), R_fov being the radius of the circle that every
# ray of the detector's field of view covers at the rotation centre, so that a
# centre anywhere in [-1, 1]^3 projects onto the detector at every angle.
L_SO_MM = 1000.0
L_SD_MM = 1500.0
DETECTOR_MM = 384.0
UNIT_MM = L_SO_MM * math.sin(math.atan((DETECTOR_MM / 2) / L_SD_MM)) / math.sqrt(3.0)


@dataclass
class Gaussians:
    """Structure-of-arrays Gaussian set, FP32, C-contiguous.

    mean [M,3], scale [M,3] (post-activation, > 0), quat [M,4] as (w,x,y,z),
    not necessarily unit length, density [M].
    """
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    density: np.ndarray

    @property
    def n(self) -> int:
        return int(self.density.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(*(np.ascontiguousarray(a[idx]) for a in
                           (self.mean, self.scale, self.quat, self.density)))


@dataclass
class ConeScan:
    """Circular cone-beam scan: gantry angles plus distances and detector size."""
    thetas: np.ndarray          # [V] float64 radians
    src_obj: float              # L_SO
    src_det: float              # L_SD
    width: int
    height: int
    pitch: float


@dataclass
class ParallelScan:
    """Parallel-beam scan: explicit world->view rotations (rows u, v, ray)."""
    rots: np.ndarray            # [V,3,3] float64
    width: int
    height: int
    pitch: float


@dataclass
class Grid:
    """Voxel grid: counts, min corner, spacing.  Voxel (i,j,k) centre is
    origin + ((i+1/2)hx, (j+1/2)hy, (k+1/2)hz); volumes are [nz][ny][nx]."""
    nx: int
    ny: int
    nz: int
    origin: tuple
    spacing: tuple


@dataclass
class Workload:
    name: str
    gaussians: Gaussians
    scan: object
    grid: Grid
    cutoff: float = 3.0
    extra: dict = field(default_factory=dict)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def random_quats(rng, m):
    """Uniform random rotations: four i.i.d. N(0,1) numbers, normalised."""
    q = rng.standard_normal((m, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _rot_from_quat_np(q):
    # Only used to orient phantom ellipsoids (data generation, not the method).
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@dataclass
class Ellipsoid:
    centre: np.ndarray   # [3]
    axes: np.ndarray     # [3] semi-axes
    rot: np.ndarray      # [3,3] columns = principal directions in world
    density: float


def phantom_value(ells, pts, clip=False, box=False):
    """f(x) = sum_k d_k 1[x in E_k] at points [N,3] (FP64)."""
    f = np.zeros(pts.shape[0])
    for e in ells:
        loc = (pts - e.centre) @ e.rot / e.axes
        f += e.density * (np.einsum("ij,ij->i", loc, loc) <= 1.0)
    if box:
        f = np.where(np.all(np.abs(pts) <= 1.0, axis=1), f, 0.0)
    if clip:
        f = np.maximum(f, 0.0)
    return f


def ellipsoids_c2(rng):
    """Ten random ellipsoids: centres U[-0.5,0.5]^3, semi-axes U[0.1,0.6]^3,
    uniform random orientation, densities U[0.1,1]."""
    out = []
    for _ in range(10):
        c = rng.uniform(-0.5, 0.5, 3)
        a = rng.uniform(0.1, 0.6, 3)
        r = _rot_from_quat_np(random_quats(rng, 1)[0])
        d = rng.uniform(0.1, 1.0)
        out.append(Ellipsoid(c, a, r, d))
    return out


def ellipsoids_shepp_logan_style(rng):
    """Twelve-ellipsoid head-like phantom (not the standard table): an outer
    shell, a 0.92-scaled inner ellipsoid of negative density, and ten small
    ellipsoids in a ball of radius 0.55 rotated about z."""
    out = []
    a0 = rng.uniform(0.8, 0.9, 3)
    out.append(Ellipsoid(np.zeros(3), a0, np.eye(3), 1.0))
    out.append(Ellipsoid(np.zeros(3), 0.92 * a0, np.eye(3), -0.8))
    for _ in range(10):
        while True:
            c = rng.uniform(-0.55, 0.55, 3)
            if np.linalg.norm(c) <= 0.55:
                break
        a = rng.uniform(0.05, 0.3, 3)
        ang = rng.uniform(0.0, math.pi)
        ca, sa = math.cos(ang), math.sin(ang)
        r = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
        d = rng.uniform(-0.2, 0.3)
        out.append(Ellipsoid(c, a, r, d))
    return out


def rejection_sample(rng, ells, m, tau, clip, box, batch=200_000):
    pts = []
    have = 0
    while have < m:
        cand = rng.uniform(-1.0, 1.0, (batch, 3))
        keep = cand[phantom_value(ells, cand, clip=clip, box=box) > tau]
        pts.append(keep)
        have += keep.shape[0]
    return np.concatenate(pts)[:m]


def nn_scale(pts, k=3):
    """RMS distance to the k nearest other centres (the paper's nearest
    neighbour scale initialisation, Sec. 3.1 "Initialization")."""
    from scipy.spatial import cKDTree
    d, _ = cKDTree(pts).query(pts, k=k + 1)
    return np.sqrt(np.mean(d[:, 1:] ** 2, axis=1))


def cone_scan(n_views, width, height, pitch_mm):
    thetas = 2.0 * math.pi * np.arange(n_views) / n_views
    return ConeScan(thetas=thetas, src_obj=L_SO_MM / UNIT_MM, src_det=L_SD_MM / UNIT_MM,
                    width=width, height=height, pitch=pitch_mm / UNIT_MM)


# --------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------

def c1_forward(seed=0, m=2000):
    """2,000 Gaussians in [-1,1]^3; one parallel view along +z onto a 128^2
    detector spanning [-1.5,1.5]^2; a 64^3 grid over [-1,1]^3; 3-sigma cutoff."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, (m, 3))
    s = np.exp(rng.uniform(math.log(0.02), math.log(0.1), (m, 3)))
    q = random_quats(rng, m)
    rho = rng.uniform(0.0, 1.0, m)
    g = Gaussians(_f32(p), _f32(s), _f32(q), _f32(rho))
    scan = ParallelScan(rots=np.eye(3)[None].copy(), width=128, height=128, pitch=3.0 / 128)
    grid = Grid(64, 64, 64, (-1.0, -1.0, -1.0), (1 / 32, 1 / 32, 1 / 32))
    return Workload("c1_parallel_2k_128px_64vox", g, scan, grid)


def c2_cone(seed=0, m=50_000, n_views=75, det=256, pitch_mm=1.5, tv=128):
    """Ten-ellipsoid phantom sampled by rejection (f > 0), rho = 0.15 f(p),
    anisotropic scales sigma_NN * exp(U[-0.5,0.5]) per axis, 75 cone views of
    256^2 at 1.5 mm, TV grid 128^3 over [-1,1]^3."""
    rng = np.random.default_rng(seed)
    ells = ellipsoids_c2(rng)
    p = rejection_sample(rng, ells, m, 0.0, clip=False, box=True)
    f = phantom_value(ells, p, box=True)
    s = nn_scale(p)[:, None] * np.exp(rng.uniform(-0.5, 0.5, (m, 3)))
    q = random_quats(rng, m)
    rho = 0.15 * f
    g = Gaussians(_f32(p), _f32(s), _f32(q), _f32(rho))
    scan = cone_scan(n_views, det, det, pitch_mm)
    h = 2.0 / tv
    grid = Grid(tv, tv, tv, (-1.0, -1.0, -1.0), (h, h, h))
    return Workload(f"c2_cone_{m // 1000}k_{n_views}x{det}px_tv{tv}", g, scan, grid,
                    extra={"ellipsoids": ells})


def c3_iteration(seed=0, m=200_000, n_views=75, det=512, pitch_mm=0.75, full=256, block=64):
    """Shepp-Logan-style 12-ellipsoid phantom, 200k centres where f > 0.05,
    rho = 0.15 f, scales sigma_NN * exp(U[-0.3,0.3]), 75 cone views of 512^2 at
    0.75 mm, TV on a random 64^3 block of a 256^3 grid over [-1,1]^3."""
    rng = np.random.default_rng(seed)
    ells = ellipsoids_shepp_logan_style(rng)
    p = rejection_sample(rng, ells, m, 0.05, clip=True, box=False)
    f = phantom_value(ells, p, clip=True)
    s = nn_scale(p)[:, None] * np.exp(rng.uniform(-0.3, 0.3, (m, 3)))
    q = random_quats(rng, m)
    rho = 0.15 * f
    g = Gaussians(_f32(p), _f32(s), _f32(q), _f32(rho))
    scan = cone_scan(n_views, det, det, pitch_mm)
    h = 2.0 / full
    grid = Grid(block, block, block, (-1.0, -1.0, -1.0), (h, h, h))
    return Workload(f"c3_iter_{m // 1000}k_{n_views}x{det}px_tv{block}of{full}", g, scan, grid,
                    extra={"ellipsoids": ells, "full": full, "block": block})


def c5_large(seed=0, m=1_000_000, n_views=150, det=1024, pitch_mm=0.375, vol=512):
    """1,000,000 Gaussians on the 12-ellipsoid phantom with prolate,
    volume-preserving anisotropy up to 20:1 (r ~ exp(U[0, ln 20]), scales
    sigma_NN (r^(2/3), r^(-1/3), r^(-1/3))), 150 cone views of 1024^2 at
    0.375 mm, a 512^3 grid over [-1,1]^3."""
    rng = np.random.default_rng(seed)
    ells = ellipsoids_shepp_logan_style(rng)
    p = rejection_sample(rng, ells, m, 0.05, clip=True, box=False, batch=1_000_000)
    f = phantom_value(ells, p, clip=True)
    r = np.exp(rng.uniform(0.0, math.log(20.0), m))
    s = nn_scale(p)[:, None] * np.stack([r ** (2 / 3), r ** (-1 / 3), r ** (-1 / 3)], 1)
    q = random_quats(rng, m)
    rho = 0.15 * f
    g = Gaussians(_f32(p), _f32(s), _f32(q), _f32(rho))
    scan = cone_scan(n_views, det, det, pitch_mm)
    h = 2.0 / vol
    grid = Grid(vol, vol, vol, (-1.0, -1.0, -1.0), (h, h, h))
    return Workload(f"c5_large_{m // 1000}k_{n_views}x{det}px_vox{vol}", g, scan, grid,
                    extra={"ellipsoids": ells})


def sub_grid(grid: Grid, i0, j0, k0, nx, ny, nz) -> Grid:
    """The voxels [k0:k0+nz, j0:j0+ny, i0:i0+nx] of `grid` as a grid of their own."""
    h = grid.spacing
    o = grid.origin
    return Grid(nx, ny, nz, (o[0] + i0 * h[0], o[1] + j0 * h[1], o[2] + k0 * h[2]), h)


def phantom_model(seed, m, tau=0.05, jitter=0.3):
    """A resident model for serving: C3-style phantom Gaussians (seeded)."""
    rng = np.random.default_rng(seed)
    ells = ellipsoids_shepp_logan_style(rng)
    p = rejection_sample(rng, ells, m, tau, clip=True, box=False)
    f = phantom_value(ells, p, clip=True)
    s = nn_scale(p)[:, None] * np.exp(rng.uniform(-jitter, jitter, (m, 3)))
    q = random_quats(rng, m)
    return Gaussians(_f32(p), _f32(s), _f32(q), _f32(0.15 * f))


def c4_models(seed=0, n_models=16, lo=20_000, hi=500_000):
    """Sizes log-uniform in [20k, 500k] (seed 0); model j from seed 1000 + j."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_models))).astype(int)
    return [phantom_model(1000 + j, int(m)) for j, m in enumerate(sizes)]


def c4_requests(seed, n, rate, n_models=16, full=256, block=128):
    """Poisson arrivals at `rate` requests/s.  80% projections: 1-64 views
    evenly spaced from a random start angle, 256^2 at 1.5 mm or 512^2 at
    0.75 mm (p = 1/2); 20% volume queries: a 128^3 block of the 256^3 grid over
    [-1,1]^3 at offset U{0..128}^3."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate > 0 else np.zeros(n)
    out = []
    h = 2.0 / full
    for i in range(n):
        model = int(rng.integers(0, n_models))
        if rng.uniform() < 0.8:
            nv = int(rng.integers(1, 65))
            th0 = rng.uniform(0.0, 2 * math.pi)
            det, pitch = (256, 1.5) if rng.uniform() < 0.5 else (512, 0.75)
            scan = cone_scan(nv, det, det, pitch)
            scan.thetas = th0 + scan.thetas
            out.append({"kind": "project", "model": model, "arrival_s": float(t[i]), "scan": scan})
        else:
            off = rng.integers(0, full - block + 1, 3)
            g = Grid(block, block, block, tuple(float(-1.0 + o * h) for o in off), (h, h, h))
            out.append({"kind": "volume", "model": model, "arrival_s": float(t[i]), "grid": g})
    return out


def tv_block_grid(wl: Workload, iteration: int) -> Grid:
    """Random D^3 sub-block of the full TV grid at the target spacing; the
    offset is drawn with seed = iteration."""
    full, block = wl.extra["full"], wl.extra["block"]
    rng = np.random.default_rng(iteration)
    off = rng.integers(0, full - block + 1, 3)
    h = wl.grid.spacing[0]
    origin = tuple(float(-1.0 + o * h) for o in off)
    return Grid(block, block, block, origin, wl.grid.spacing)


def upstream(seed, shape):
    """N(0,1) upstream gradient, FP32."""
    return _f32(np.random.default_rng(seed).standard_normal(shape))


def random_images(seed, n, h, w, smooth=3):
    """Smooth positive random images in [0,1] for loss tests."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n, h, w))
    for _ in range(smooth):
        x = 0.25 * (np.roll(x, 1, 1) + np.roll(x, -1, 1) + np.roll(x, 1, 2) + np.roll(x, -1, 2))
    x = (x - x.min()) / max(x.max() - x.min(), 1e-12)
    return _f32(x)


# --------------------------------------------------------------------------
# Measured projections for the training iteration: exact line integrals of the
# additive ellipsoid phantom along each detector ray (chord length x density),
# clipped at zero.  This plays the role of the CT toolbox in the paper's data
# synthesis and is independent of the Gaussian representation.
# --------------------------------------------------------------------------

def _cone_rays(theta, scan: ConeScan, rows):
    """Source point and unit directions for detector rows `rows` of one view.

    Scanner model of App. A: the source circles the z axis at distance L_SO,
    the flat detector is perpendicular to the central ray at distance L_SD from
    the source, detector columns run along (-sin t, cos t, 0) and rows along -z;
    pixel centres sit at ((a + 1/2 - W/2) h, (b + 1/2 - H/2) h)."""
    c, s = math.cos(theta), math.sin(theta)
    src = scan.src_obj * np.array([c, s, 0.0])
    axis = -np.array([c, s, 0.0])
    u_ax = np.array([-s, c, 0.0])
    v_ax = np.array([0.0, 0.0, -1.0])
    a = (np.arange(scan.width) + 0.5 - scan.width / 2) * scan.pitch
    b = (np.asarray(rows) + 0.5 - scan.height / 2) * scan.pitch
    det = src + scan.src_det * axis
    pts = det[None, None, :] + b[:, None, None] * v_ax + a[None, :, None] * u_ax
    d = pts - src
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return src, d


def phantom_volume(wl: Workload, grid: Grid):
    """Ground-truth density f of the workload's phantom at the voxel centres
    of grid, [nz][ny][nx] FP32 (the volume its measured projections
    integrate)."""
    ells = wl.extra["ellipsoids"]
    ax = [grid.origin[k] + (np.arange(n) + 0.5) * grid.spacing[k]
          for k, n in enumerate((grid.nx, grid.ny, grid.nz))]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    return _f32(phantom_value(ells, pts, clip=True).reshape(grid.nz, grid.ny, grid.nx))


def measured_projections(wl: Workload, rows_per_chunk=64):
    scan = wl.scan
    ells = wl.extra["ellipsoids"]
    out = np.zeros((len(scan.thetas), scan.height, scan.width), np.float32)
    for v, th in enumerate(scan.thetas):
        for r0 in range(0, scan.height, rows_per_chunk):
            rows = np.arange(r0, min(r0 + rows_per_chunk, scan.height))
            src, d = _cone_rays(th, scan, rows)
            acc = np.zeros(d.shape[:2])
            for e in ells:
                o = (src - e.centre) @ e.rot / e.axes
                dd = (d @ e.rot) / e.axes
                aa = np.einsum("...i,...i->...", dd, dd)
                bb = dd @ o
                cc = o @ o - 1.0
                disc = bb * bb - aa * cc
                chord = np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0)) / aa, 0.0)
                acc += e.density * chord
            out[v, rows] = np.maximum(acc, 0.0)
    return out
