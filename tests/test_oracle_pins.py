"""Pins of the FP64 oracle to facts outside the oracle itself.

Each test checks the oracle against closed forms, physical laws, independent
library routines (scipy rotations, quadrature, Gaussian filters, multivariate
normal densities) or finite differences, chosen so that a plausible mistake in
the oracle (dropped rectification factor, wrong sign in the scanner rotation,
transposed rotation, wrong Jacobian row, wrong pixel centre) fails at least one
of them.  No GPU is used.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch
from scipy import integrate
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

import oracle
from tests import scenes

INF = float("inf")


# --------------------------------------------------------------- rotation ---

def test_rotation_matches_scipy_hamilton():
    """The quaternion convention (w,x,y,z), Hamilton, normalised inside the
    operator, agrees with scipy's Rotation (an independent implementation)."""
    rng = np.random.default_rng(0)
    q = rng.standard_normal((50, 4)) * rng.uniform(0.1, 3.0, (50, 1))
    R = oracle.rotation(torch.tensor(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-13)


def test_covariance_and_precision_are_inverse():
    g = scenes.random_scene(1, 20)
    s = torch.tensor(g.scale, dtype=torch.float64)
    q = torch.tensor(g.quat, dtype=torch.float64)
    S = oracle.covariance(s, q).numpy()
    P = oracle.precision(s, q).numpy()
    np.testing.assert_allclose(np.einsum("nij,njk->nik", S, P), np.broadcast_to(np.eye(3), S.shape),
                               atol=1e-10)
    np.testing.assert_allclose(S, scenes.scipy_covariance(g), rtol=1e-12, atol=1e-15)


# ----------------------------------------------------- parallel beam (P1) ---

def test_parallel_equals_exact_line_integral_every_pixel():
    """Parallel beam, no cutoff: the rectified 2D Gaussian sum equals the exact
    line integral of the 3D density at every pixel (Eq. 7 is exact here)."""
    g = scenes.random_scene(3, 6, lo=0.05, hi=0.25)
    rot = Rotation.random(random_state=4).as_matrix()
    view = oracle.parallel_view(rot, 40, 32, 0.04, off_u=0.013, off_v=-0.021)
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    W = view["W"]
    u, v = scenes.pixel_centres(view)
    o = u[None, :, None] * W[0] + v[:, None, None] * W[1]
    d = np.broadcast_to(W[2] / np.linalg.norm(W[2]), o.shape)
    exact = scenes.line_integral(g, o, d)
    np.testing.assert_allclose(img, exact, rtol=1e-6, atol=1e-9 * exact.max())


def test_parallel_against_adaptive_quadrature():
    g = scenes.random_scene(5, 3)
    view = oracle.parallel_view(np.eye(3), 16, 16, 0.06)
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    Sig = scenes.scipy_covariance(g)
    P = np.linalg.inv(Sig)
    u, v = scenes.pixel_centres(view)
    for (b, a) in [(3, 4), (8, 8), (12, 2), (0, 15)]:
        def f(t):
            x = np.array([u[a], v[b], t])
            return sum(float(g.density[i]) * math.exp(-0.5 * (x - g.mean[i]) @ P[i] @ (x - g.mean[i]))
                       for i in range(g.n))
        val, _ = integrate.quad(f, -4, 4, epsabs=1e-13, epsrel=1e-12, limit=200)
        assert abs(img[b, a] - val) <= 1e-9 * max(abs(val), 1e-3)


def test_isotropic_closed_form_parallel():
    """Sigma = s^2 I: image = rho s sqrt(2 pi) exp(-r^2 / (2 s^2))."""
    g = scenes.gaussians([[0.11, -0.07, 0.3]], [[0.15, 0.15, 0.15]], [[0.3, 0.1, -0.5, 0.8]], [0.7])
    view = oracle.parallel_view(np.eye(3), 33, 31, 0.025)
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    u, v = scenes.pixel_centres(view)
    s, p = float(g.scale[0, 0]), g.mean[0].astype(np.float64)
    r2 = (u[None, :] - p[0]) ** 2 + (v[:, None] - p[1]) ** 2
    ref = float(g.density[0]) * s * math.sqrt(2 * math.pi) * np.exp(-r2 / (2 * s * s))
    np.testing.assert_allclose(img, ref, rtol=1e-6, atol=1e-12)


def test_isotropic_mu_any_view():
    """For Sigma = s^2 I the rectification factor is sqrt(2 pi) s for every view."""
    g = scenes.gaussians([[0.2, 0.1, -0.3], [-0.4, 0.3, 0.2]], [[0.1] * 3, [0.05] * 3],
                         [[1, 0, 0, 0], [0.2, 0.4, 0.1, 0.3]], [1.0, 1.0])
    params = [torch.tensor(a, dtype=torch.float64) for a in (g.mean, g.scale, g.quat, g.density)]
    for th in (0.0, 0.4, 2.0, 4.4):
        pr = oracle.project_gaussians(*params, oracle.cone_view(th, 13.6, 20.5, 32, 32, 0.05))
        # the FP32-rounded scanner rotation is orthonormal to ~6e-8 only
        np.testing.assert_allclose(pr["mu"].numpy(), math.sqrt(2 * math.pi) * g.scale[:, 0].astype(np.float64),
                                   rtol=1e-7)


# --------------------------------------------------------- cone beam (P2) ---

def _on_ray_gaussian(view, theta, a, b, lam, scale, quat, rho):
    src, _ = scenes.cone_rays(view, theta)
    src_, dirs = scenes.cone_rays(view, theta)
    p = src_[b, a] + lam * dirs[b, a]
    return scenes.gaussians(p, scale, quat, rho), src_[b, a], dirs[b, a]


@pytest.mark.parametrize("theta", [0.0, 0.9, 2.5, 5.1])
def test_cone_central_ray_equals_exact_integral(theta):
    """A Gaussian centred on the ray through a pixel centre: the pixel value is
    the exact line integral through the centre, rho sqrt(2 pi / (d^T P d)), and
    agrees with adaptive quadrature along the physical ray (App. A scanner)."""
    view = oracle.cone_view(theta, 13.64, 20.46, 48, 40, 0.06)
    a, b = 30, 11
    g, o, d = _on_ray_gaussian(view, theta, a, b, 13.0, [0.08, 0.3, 0.15],
                               [0.9, -0.2, 0.35, 0.1], 0.8)
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    Sig = scenes.scipy_covariance(g)[0]
    P = np.linalg.inv(Sig)
    p = g.mean[0].astype(np.float64)
    f = lambda t: 0.8 * math.exp(-0.5 * (o + t * d - p) @ P @ (o + t * d - p))
    tc = float(d @ (p - o))
    val, _ = integrate.quad(f, tc - 5, tc + 5, epsabs=1e-14, epsrel=1e-12, limit=200)
    assert abs(img[b, a] - val) <= 2e-6 * val


def test_cone_off_centre_within_local_affine_error():
    """Away from the central ray the method uses the local affine (EWA)
    approximation (Eq. 6), so it is not exact; for a small Gaussian the
    relative error against the exact line integral is bounded by O(sigma/L)."""
    theta = 1.3
    view = oracle.cone_view(theta, 13.64, 20.46, 64, 64, 0.01)
    g = scenes.gaussians([[0.05, -0.08, 0.1]], [[0.012, 0.03, 0.02]], [[0.7, 0.3, -0.4, 0.5]], [1.0])
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    o, d = scenes.cone_rays(view, theta)
    exact = scenes.line_integral(g, o, d)
    err = np.abs(img - exact).max() / exact.max()
    assert err < 3e-3, err
    # and the footprint is substantially covered by the detector
    assert exact.sum() > 0.5 * exact.max() * 50


def test_cone_conservation_of_detector_integral():
    """Integral of the projection over the detector plane = mass times the
    magnification of the cone beam at the centre: for a ray bundle from a point
    source, du dt = D^3 / (t^2 L_SD) dV with D the source-to-detector-point
    distance, giving L_SD^2 l / t2^3 for a centre at depth t2 and range l."""
    theta = 0.6
    view = oracle.cone_view(theta, 13.64, 20.46, 96, 96, 0.02)
    g = scenes.gaussians([[0.2, -0.1, 0.15]], [[0.05, 0.08, 0.06]], [[0.6, -0.2, 0.5, 0.3]], [0.9])
    img = oracle.project(g, [view], cutoff=INF)["image"][0]
    src, axis, _, _ = scenes.cone_geometry(theta, view["L_SO"], view["L_SD"])
    p = g.mean[0].astype(np.float64)
    t2 = float((p - src) @ axis)
    l = float(np.linalg.norm(p - src))
    L = view["L_SD"]
    mass = float(g.density[0]) * (2 * math.pi) ** 1.5 * float(np.prod(g.scale[0].astype(np.float64)))
    expect = mass * L * L * l / t2 ** 3
    total = img.sum() * view["hu"] * view["hv"]
    # exact up to the FP32 rounding of the scanner rotation (~6e-8)
    assert abs(total - expect) <= 1e-7 * expect


def test_cutoff_mass_fraction_2d():
    """With cutoff kappa the detector integral is multiplied by the 2D Gaussian
    mass inside q <= kappa^2, 1 - exp(-kappa^2/2) (up to the pixel sum's error)."""
    view = oracle.parallel_view(np.eye(3), 200, 200, 0.005)
    g = scenes.gaussians([[0.0013, -0.0021, 0.0]], [[0.06, 0.09, 0.07]], [[0.8, 0.1, 0.3, -0.2]], [1.0])
    full = oracle.project(g, [view], cutoff=INF)["image"].sum()
    cut = oracle.project(g, [view], cutoff=3.0)["image"].sum()
    assert abs(cut / full - (1 - math.exp(-4.5))) < 2e-4


def test_parallel_limit_of_cone():
    """Cone beam with L_SO, L_SD -> inf at fixed magnification M and pitch
    M*h converges to the parallel projection with pitch h (rays along the
    central axis); the error decays like 1/L."""
    g = scenes.random_scene(8, 4, lo=0.05, hi=0.12, box=0.3)
    theta = 0.8
    M = 1.5
    h = 0.03
    Wc = oracle.cone_view(theta, 1.0, 1.5, 40, 40, M * h)["W"]
    par = oracle.project(g, [oracle.parallel_view(Wc, 40, 40, h)], cutoff=INF)["image"][0]
    errs = []
    for L in (1e2, 1e3, 1e4):
        cone = oracle.project(g, [oracle.cone_view(theta, L, M * L, 40, 40, M * h)], cutoff=INF)["image"][0]
        errs.append(np.abs(cone - par).max() / par.max())
    assert errs[2] < 1e-3 and errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[0] / errs[2] > 30


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def test_rotation_covariance_of_gantry():
    """Rotating the scene by alpha about z and the gantry angle by alpha leaves
    every projection unchanged (fixes the signs of the scanner rotation and the
    quaternion convention)."""
    g = scenes.random_scene(11, 5, lo=0.03, hi=0.15, box=0.4)
    alpha = 0.7
    ca, sa = math.cos(alpha), math.sin(alpha)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1.0]])
    qz = np.array([math.cos(alpha / 2), 0.0, 0.0, math.sin(alpha / 2)])
    g2 = scenes.gaussians(g.mean.astype(np.float64) @ Rz.T, g.scale, _quat_mul(qz, g.quat.astype(np.float64)),
                          g.density)
    for th in (0.3, 2.0):
        i1 = oracle.project(g, [oracle.cone_view(th, 13.64, 20.46, 48, 48, 0.04)], cutoff=INF)["image"]
        i2 = oracle.project(g2, [oracle.cone_view(th + alpha, 13.64, 20.46, 48, 48, 0.04)], cutoff=INF)["image"]
        assert np.abs(i1 - i2).max() <= 1e-5 * i1.max()


def test_linearity_permutation_duplication():
    """Composition is a plain sum: linear in rho, order-free, and a duplicated
    Gaussian doubles its contribution (so halving both copies' density, as the
    densification rule does, preserves the image)."""
    g = scenes.random_scene(12, 7)
    views = [oracle.cone_view(t, 13.64, 20.46, 32, 32, 0.05) for t in (0.1, 1.7)]
    base = oracle.project(g, views)["image"]
    g2 = scenes.gaussians(g.mean, g.scale, g.quat, 2.5 * g.density.astype(np.float64))
    np.testing.assert_allclose(oracle.project(g2, views)["image"], 2.5 * base, rtol=1e-6)
    perm = np.random.default_rng(0).permutation(g.n)
    np.testing.assert_allclose(oracle.project(g.subset(perm), views)["image"], base, rtol=1e-12, atol=1e-15)
    dup = np.concatenate([np.arange(g.n), np.arange(g.n)])
    gd = g.subset(dup)
    gd.density = (gd.density * np.float32(0.5)).astype(np.float32)
    np.testing.assert_allclose(oracle.project(gd, views)["image"], base, rtol=1e-12, atol=1e-15)


def test_cutoff_brute_force_agree():
    g = scenes.random_scene(13, 10)
    views = [oracle.cone_view(0.4, 13.64, 20.46, 40, 36, 0.04)]
    a = oracle.project(g, views, cutoff=3.0)
    b = oracle.project(g, views, cutoff=3.0, brute=True)
    np.testing.assert_array_equal(a["image"], b["image"])
    assert a["npairs"][0] == b["npairs"][0] > 0


# ---------------------------------------------------------- voxelizer (P10) ---

def test_voxel_values_match_scipy_density():
    g = scenes.random_scene(14, 5)
    grd = scenes.grid(12)
    vol = oracle.voxelize(g, grd, cutoff=INF)["volume"]
    Sig = scenes.scipy_covariance(g)
    h = float(np.float32(grd.spacing[0]))   # the interface carries FP32 grid geometry
    c = -1 + (np.arange(12) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    ref = np.zeros(pts.shape[0])
    for i in range(g.n):
        mvn = multivariate_normal(mean=g.mean[i].astype(np.float64), cov=Sig[i])
        ref += float(g.density[i]) * mvn.pdf(pts) * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(Sig[i]))
    np.testing.assert_allclose(vol.reshape(-1), ref, rtol=1e-9, atol=1e-14)


def test_voxel_mass_and_cutoff_fraction():
    """sum V h^3 = mass * F(kappa), F(3) = erf(3/sqrt 2) - sqrt(2/pi) 3 e^{-4.5}."""
    g = scenes.gaussians([[0.011, -0.02, 0.007]], [[0.1, 0.14, 0.12]], [[0.5, 0.5, -0.1, 0.7]], [1.3])
    grd = scenes.grid(96)
    mass = float(g.density[0]) * (2 * math.pi) ** 1.5 * float(np.prod(g.scale[0].astype(np.float64)))
    h3 = float(np.float32(grd.spacing[0])) ** 3
    full = oracle.voxelize(g, grd, cutoff=INF)["volume"].sum() * h3
    cut = oracle.voxelize(g, grd, cutoff=3.0)["volume"].sum() * h3
    F3 = math.erf(3 / math.sqrt(2)) - math.sqrt(2 / math.pi) * 3 * math.exp(-4.5)
    assert abs(full / mass - 1) < 1e-9
    assert abs(cut / mass - F3) < 2e-3


def test_voxel_brute_equals_culled():
    g = scenes.random_scene(15, 12)
    grd = scenes.grid(20)
    a = oracle.voxelize(g, grd, cutoff=3.0)
    b = oracle.voxelize(g, grd, cutoff=3.0, brute=True)
    np.testing.assert_allclose(a["volume"], b["volume"], rtol=1e-13, atol=1e-15)
    assert a["npairs"] == b["npairs"]


# -------------------------------------------------------- gradients (P11) ---

def _fd(fun, g, key, idx, h):
    arrs = {k: getattr(g, k).astype(np.float64).copy() for k in ("mean", "scale", "quat", "density")}
    out = []
    for sgn in (+1, -1):
        a = {k: v.copy() for k, v in arrs.items()}
        a[key][idx] += sgn * h
        out.append(fun(a))
    return (out[0] - out[1]) / (2 * h)


class _G64:
    """Gaussian set carrying float64 arrays (finite differences need steps far
    below FP32 resolution; the oracle widens whatever it is given)."""
    def __init__(self, a):
        self.mean, self.scale, self.quat, self.density = a["mean"], a["scale"], a["quat"], a["density"]
        self.n = self.density.shape[0]


def _params64(g):
    return {k: getattr(g, k).astype(np.float64) for k in ("mean", "scale", "quat", "density")}


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_projection_gradient_matches_finite_differences(beam, monkeypatch):
    monkeypatch.setattr(oracle, "_params",
                        lambda g, requires_grad=False: [torch.tensor(np.asarray(a, np.float64),
                                                                     requires_grad=requires_grad)
                                                        for a in (g.mean, g.scale, g.quat, g.density)])
    g = scenes.random_scene(21, 4, lo=0.06, hi=0.2, box=0.3)
    if beam == "cone":
        views = [oracle.cone_view(t, 4.0, 6.0, 24, 24, 0.08) for t in (0.3, 2.2)]
    else:
        views = [oracle.parallel_view(Rotation.random(random_state=s).as_matrix(), 24, 24, 0.06) for s in (1, 2)]
    G = np.random.default_rng(3).standard_normal((2, 24, 24))
    gr = oracle.project_grad(g, views, G, cutoff=INF)
    f = lambda a: float((oracle.project(_G64(a), views, cutoff=INF)["image"] * G).sum())
    for key, shape in (("mean", (4, 3)), ("scale", (4, 3)), ("quat", (4, 4)), ("density", (4,))):
        for idx in np.ndindex(*shape):
            fd = _fd(f, g, key, idx, 1e-6)
            assert abs(gr[key][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (key, idx, gr[key][idx], fd)


def test_voxel_gradient_matches_finite_differences(monkeypatch):
    monkeypatch.setattr(oracle, "_params",
                        lambda g, requires_grad=False: [torch.tensor(np.asarray(a, np.float64),
                                                                     requires_grad=requires_grad)
                                                        for a in (g.mean, g.scale, g.quat, g.density)])
    g = scenes.random_scene(22, 3, lo=0.08, hi=0.2, box=0.3)
    grd = scenes.grid(10)
    H = np.random.default_rng(4).standard_normal((10, 10, 10))
    gr = oracle.voxelize_grad(g, grd, H, cutoff=INF)
    f = lambda a: float((oracle.voxelize(_G64(a), grd, cutoff=INF)["volume"] * H).sum())
    for key, shape in (("mean", (3, 3)), ("scale", (3, 3)), ("quat", (3, 4)), ("density", (3,))):
        for idx in np.ndindex(*shape):
            fd = _fd(f, g, key, idx, 1e-6)
            assert abs(gr[key][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (key, idx)


def _clean_gaussians(gr, n):
    """Gaussians none of whose pairs lies within the cutoff's ambiguity band
    (|q - kappa^2| <= 1e-3 kappa^2): a central-difference step cannot move one
    of their terms across the cutoff."""
    return [i for i in range(n) if all(np.all(np.asarray(gr["amb"][k])[i] == 0.0)
                                       for k in ("mean", "scale", "quat", "density"))]


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_projection_gradient_with_cutoff_matches_finite_differences(beam, monkeypatch):
    """The cutoff branch (kappa = 3) of the analytic projection gradient: the
    terms inside the cutoff, differentiated with the indicator held fixed,
    equal FP64 central differences of the cutoff sum for every Gaussian whose
    pairs all stay clear of the cutoff (its derivative is zero almost
    everywhere)."""
    monkeypatch.setattr(oracle, "_params",
                        lambda g, requires_grad=False: [torch.tensor(np.asarray(a, np.float64),
                                                                     requires_grad=requires_grad)
                                                        for a in (g.mean, g.scale, g.quat, g.density)])
    g = scenes.random_scene(25, 10, lo=0.04, hi=0.12, box=0.3)
    if beam == "cone":
        views = [oracle.cone_view(t, 4.0, 6.0, 28, 28, 0.07) for t in (0.3, 2.2)]
    else:
        views = [oracle.parallel_view(Rotation.random(random_state=s).as_matrix(), 28, 28, 0.05)
                 for s in (3, 4)]
    G = np.random.default_rng(7).standard_normal((2, 28, 28))
    gr = oracle.project_grad(g, views, G, cutoff=3.0, with_scale=True)
    clean = _clean_gaussians(gr, g.n)
    assert len(clean) >= 3, clean
    f = lambda a: float((oracle.project(_G64(a), views, cutoff=3.0)["image"] * G).sum())
    for i in clean:
        for key, width in (("mean", 3), ("scale", 3), ("quat", 4), ("density", None)):
            for idx in ([(i,)] if width is None else [(i, c) for c in range(width)]):
                fd = _fd(f, g, key, idx, 1e-6)
                assert abs(gr[key][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (key, idx, gr[key][idx], fd)


def test_voxel_gradient_with_cutoff_matches_finite_differences(monkeypatch):
    """The cutoff branch (kappa = 3) of the analytic voxelizer gradient against
    FP64 central differences, for the Gaussians whose voxel pairs all stay
    clear of the cutoff."""
    monkeypatch.setattr(oracle, "_params",
                        lambda g, requires_grad=False: [torch.tensor(np.asarray(a, np.float64),
                                                                     requires_grad=requires_grad)
                                                        for a in (g.mean, g.scale, g.quat, g.density)])
    g = scenes.random_scene(26, 8, lo=0.06, hi=0.15, box=0.3)
    grd = scenes.grid(12)
    H = np.random.default_rng(8).standard_normal((12, 12, 12))
    gr = oracle.voxelize_grad(g, grd, H, cutoff=3.0, with_scale=True)
    clean = _clean_gaussians(gr, g.n)
    assert len(clean) >= 2, clean
    f = lambda a: float((oracle.voxelize(_G64(a), grd, cutoff=3.0)["volume"] * H).sum())
    for i in clean:
        for key, width in (("mean", 3), ("scale", 3), ("quat", 4), ("density", None)):
            for idx in ([(i,)] if width is None else [(i, c) for c in range(width)]):
                fd = _fd(f, g, key, idx, 1e-6)
                assert abs(gr[key][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (key, idx, gr[key][idx], fd)


def test_gradient_scale_bounds_gradient():
    g = scenes.random_scene(23, 6)
    views = [oracle.cone_view(0.5, 13.64, 20.46, 32, 32, 0.05)]
    G = np.random.default_rng(5).standard_normal((1, 32, 32))
    gr = oracle.project_grad(g, views, G, with_scale=True)
    for k in ("mean", "scale", "quat", "density"):
        assert np.all(np.abs(gr[k]) <= gr["S_abs"][k] * (1 + 1e-12) + 1e-300)
        assert np.all(gr["amb"][k] <= gr["S_abs"][k] * (1 + 1e-12) + 1e-300)


def test_gradient_select_subset():
    g = scenes.random_scene(24, 8)
    views = [oracle.cone_view(0.5, 13.64, 20.46, 32, 32, 0.05)]
    G = np.random.default_rng(6).standard_normal((1, 32, 32))
    full = oracle.project_grad(g, views, G)
    sub = oracle.project_grad(g, views, G, select=[1, 5])
    for k in ("mean", "scale", "quat", "density"):
        np.testing.assert_allclose(sub[k][[1, 5]], full[k][[1, 5]], rtol=1e-12, atol=1e-300)
        assert np.all(sub[k][[0, 2, 3, 4, 6, 7]] == 0)


# ----------------------------------------------------------- losses (P12) ---

def test_image_loss_grad_scale_bounds_the_gradient():
    """The per-pixel magnitudes behind the image-loss gradient tolerance: the
    gradient's L1 and D-SSIM parts never exceed them (they are sums of the
    absolute values of the parts' terms), an FP32 evaluation of the loss
    gradient passes the tolerance, and a 1% error in the D-SSIM part fails it."""
    from oracle import parity
    rng = np.random.default_rng(31)
    x = rng.uniform(0, 1, (2, 40, 33)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, None).astype(np.float32)
    _, _, _, g = oracle.image_loss(x, y, 0.25)
    ssim_abs, l1_abs = oracle.image_loss_grad_scale(x, y, 0.25)
    l1_part = np.sign(x.astype(np.float64) - y) / x.size
    assert np.all(np.abs(l1_part) <= l1_abs * (1 + 1e-12))
    assert np.all(np.abs(g - l1_part) <= ssim_abs * (1 + 1e-9) + 1e-300)
    xr = torch.tensor(x, requires_grad=True)
    ym = torch.tensor(y)
    w = oracle.ssim_window().float()[None, None]
    conv = lambda a: torch.nn.functional.conv2d(a[:, None], w, padding=5)[:, 0]
    mx, my = conv(xr), conv(ym)
    sxx, syy, sxy = conv(xr * xr) - mx * mx, conv(ym * ym) - my * my, conv(xr * ym) - mx * my
    S = ((2 * mx * my + 1e-4) * (2 * sxy + 9e-4)) / ((mx * mx + my * my + 1e-4) * (sxx + syy + 9e-4))
    (g32,) = torch.autograd.grad((xr - ym).abs().mean() + 0.25 * (1 - S.mean()), xr)
    assert parity.loss_grad_violation(g32.numpy(), g, (ssim_abs, l1_abs)) <= 1.0
    bad = l1_part + 1.01 * (g - l1_part)
    assert parity.loss_grad_violation(bad, g, (ssim_abs, l1_abs)) > 1.0


def _ssim_scipy(x, y):
    from scipy.ndimage import gaussian_filter
    f = lambda a: gaussian_filter(a, 1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
    vals = []
    for a, b in zip(x, y):
        a = a.astype(np.float64); b = b.astype(np.float64)
        mx, my = f(a), f(b)
        sxx = f(a * a) - mx * mx
        syy = f(b * b) - my * my
        sxy = f(a * b) - mx * my
        c1, c2 = 0.01 ** 2, 0.03 ** 2
        vals.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2)))
    return np.mean(vals)


def test_ssim_matches_scipy_gaussian_filter():
    import workloads
    x = workloads.random_images(1, 3, 40, 37)
    y = workloads.random_images(2, 3, 40, 37)
    total, l1, s, _ = oracle.image_loss(x, y, 0.25)
    assert abs(s - _ssim_scipy(x, y)) < 1e-12
    assert abs(l1 - np.abs(x.astype(np.float64) - y).mean()) < 1e-15
    assert abs(total - (l1 + 0.25 * (1 - s))) < 1e-15


def test_ssim_identity_and_gradient_fd():
    import workloads
    x = workloads.random_images(3, 2, 20, 22)
    _, _, s, _ = oracle.image_loss(x, x, 0.25)
    assert abs(s - 1) < 1e-14
    y = workloads.random_images(4, 2, 20, 22)
    _, _, _, g = oracle.image_loss(x, y, 0.25)
    rng = np.random.default_rng(0)
    xd = x.astype(np.float64)
    # finite differences on a float64 copy (the loss widens its inputs)
    def total(arr):
        r = torch.tensor(arr)
        m = torch.tensor(y, dtype=torch.float64)
        return float((r - m).abs().mean() + 0.25 * (1 - oracle.ssim(r, m)))
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in x.shape)
        h = 1e-6
        a = xd.copy(); a[idx] += h
        b = xd.copy(); b[idx] -= h
        fd = (total(a) - total(b)) / (2 * h)
        assert abs(g[idx] - fd) < 1e-7 + 1e-5 * abs(fd)


def test_tv_closed_forms():
    D = 6
    const = np.full((D, D, D), 0.37, np.float32)
    t, g = oracle.tv_loss(const)
    assert t == 0.0 and np.all(g == 0)
    i = np.arange(D, dtype=np.float64)
    ramp = (0.25 * i[None, None, :] - 0.5 * i[None, :, None] + 0 * i[:, None, None]).astype(np.float32)
    t, g = oracle.tv_loss(np.broadcast_to(ramp, (D, D, D)).copy())
    assert abs(t - 0.75) < 1e-7
    # brute force on a random block
    v = np.random.default_rng(1).standard_normal((4, 5, 6)).astype(np.float32)
    t, g = oracle.tv_loss(v, weight=0.05)
    vd = v.astype(np.float64)
    ref = (np.abs(np.diff(vd, axis=0)).mean() + np.abs(np.diff(vd, axis=1)).mean() +
           np.abs(np.diff(vd, axis=2)).mean())
    assert abs(t - ref) < 1e-13
    gref = np.zeros_like(vd)
    for ax in range(3):
        dsg = np.sign(np.diff(vd, axis=ax)) / np.diff(vd, axis=ax).size
        sl_hi = [slice(None)] * 3; sl_hi[ax] = slice(1, None)
        sl_lo = [slice(None)] * 3; sl_lo[ax] = slice(None, -1)
        gref[tuple(sl_hi)] += dsg
        gref[tuple(sl_lo)] -= dsg
    np.testing.assert_allclose(g, 0.05 * gref, atol=1e-15)


# ------------------------------------------- planted mistakes are caught ---
# Each test plants a plausible mistake in the oracle (on the CPU, by
# monkeypatching) and checks that one of the pins above fails.

def test_pin_catches_dropped_rectification(monkeypatch):
    orig = oracle.project_gaussians

    def unrectified(mean, scale, quat, density, view):
        r = orig(mean, scale, quat, density, view)
        r["rho_hat"] = density * torch.ones_like(r["rho_hat"])
        return r
    monkeypatch.setattr(oracle, "project_gaussians", unrectified)
    with pytest.raises(AssertionError):
        test_parallel_equals_exact_line_integral_every_pixel()


def test_pin_catches_transposed_rotation(monkeypatch):
    orig = oracle.rotation
    monkeypatch.setattr(oracle, "rotation", lambda q: orig(q).transpose(1, 2))
    with pytest.raises(AssertionError):
        test_rotation_covariance_of_gantry()


def test_pin_catches_mirrored_gantry_angle(monkeypatch):
    orig = oracle.cone_view
    monkeypatch.setattr(oracle, "cone_view", lambda th, *a, **k: orig(-th, *a, **k))
    with pytest.raises(AssertionError):
        test_cone_central_ray_equals_exact_integral(0.9)


def test_pin_catches_wrong_third_jacobian_row(monkeypatch):
    """Using the optical axis instead of the ray direction as the third row of
    the local affine Jacobian changes the rectification off-axis."""
    orig = oracle.project_gaussians

    def axis_row(mean, scale, quat, density, view):
        r = orig(mean, scale, quat, density, view)
        if view["beam"] == oracle.BEAM_CONE:
            W = torch.tensor(view["W"], dtype=torch.float64)
            P = oracle.precision(scale, quat)
            d = W[2].expand(mean.shape[0], 3)
            m = torch.einsum("ni,nij,nj->n", d, P, d)
            r["rho_hat"] = torch.sqrt(2 * math.pi / m) * density
        return r
    monkeypatch.setattr(oracle, "project_gaussians", axis_row)
    with pytest.raises(AssertionError):
        test_cone_central_ray_equals_exact_integral(0.9)


# ------------------------------------------------ integration bias (P13) ---

def test_unrectified_projection_is_biased_by_mu():
    """Parallel beam: the unrectified image times mu equals the exact line
    integral (so the unrectified image is the integral divided by a
    view-dependent factor)."""
    g = scenes.gaussians([[0.05, -0.1, 0.2]], [[0.06, 0.2, 0.1]], [[0.7, 0.1, -0.4, 0.3]], [0.9])
    rot = Rotation.random(random_state=12).as_matrix()
    view = oracle.parallel_view(rot, 40, 40, 0.03)
    unrect = oracle.project(g, [view], cutoff=INF, rectify=False)["image"][0]
    rect = oracle.project(g, [view], cutoff=INF)["image"][0]
    mu = oracle.mean_mu(g, [view])[0]
    np.testing.assert_allclose(unrect * mu, rect, rtol=1e-12, atol=1e-15)
    W = view["W"]
    u, v = scenes.pixel_centres(view)
    o = u[None, :, None] * W[0] + v[:, None, None] * W[1]
    exact = scenes.line_integral(g, o, np.broadcast_to(W[2] / np.linalg.norm(W[2]), o.shape))
    np.testing.assert_allclose(unrect * mu, exact, rtol=1e-6, atol=1e-8 * exact.max())


def test_rectification_gives_view_consistent_density():
    """The density recovered from each view's central pixel, I_j(p_hat_j) /
    mu_j, is the same 3D density for every view with rectification; an
    unrectified renderer would need a different density per view (mu_j varies
    with the view for an anisotropic Gaussian)."""
    views, mus, peaks = [], [], []
    for th in np.linspace(0.0, np.pi, 7):
        view = oracle.cone_view(th, 13.64, 20.46, 48, 40, 0.06)
        g, o, d = _on_ray_gaussian(view, th, 30, 11, 13.0, [0.04, 0.2, 0.08], [0.9, -0.2, 0.35, 0.1], 0.8)
        img = oracle.project(g, [view], cutoff=INF)["image"][0]
        peaks.append(img[11, 30])
        mus.append(oracle.mean_mu(g, [view])[0])
    ratio = np.array(peaks) / np.array(mus)
    np.testing.assert_allclose(ratio, 0.8, rtol=2e-6)
    mus = np.array(mus)
    assert mus.std() / mus.mean() > 0.1


def test_integration_bias_least_squares():
    """Sec. 3.2.1 / Sec. 4.3 on a synthetic phantom: fit only the densities of
    a model whose geometry is exact to projections of that model.  Rectified
    kernels recover the true densities exactly (the data lie in their range);
    the unrectified kernels cannot fit all views with one density per Gaussian,
    their density divided by the mean mu is wrong, and dividing by each view's
    mu_j gives a different density per view."""
    g = scenes.lattice()
    views = [oracle.cone_view(t, 13.64, 20.46, 32, 32, 0.06)
             for t in np.linspace(0, np.pi, 6, endpoint=False)]

    def footprints(rectify):
        cols = []
        for i in range(g.n):
            d = np.zeros(g.n, np.float32)
            d[i] = 1.0
            gi = dataclasses.replace(g, density=d)
            cols.append(oracle.project(gi, views, rectify=rectify)["image"].ravel())
        return np.stack(cols, 1)

    rho = g.density.astype(np.float64)
    A_rect, A_un = footprints(True), footprints(False)
    b = A_rect @ rho
    fit_rect = np.linalg.lstsq(A_rect, b, rcond=None)[0]
    np.testing.assert_allclose(fit_rect, rho, atol=1e-9)
    fit_un = np.linalg.lstsq(A_un, b, rcond=None)[0]
    assert np.linalg.norm(A_un @ fit_un - b) / np.linalg.norm(b) > 0.05
    mubar = oracle.mean_mu(g, views)
    assert np.linalg.norm(fit_un / mubar - rho) / np.linalg.norm(rho) > 0.05
    per_view = fit_un[None] / np.stack([oracle.mean_mu(g, [v]) for v in views])
    assert np.median((per_view.max(0) - per_view.min(0)) / rho) > 0.2
