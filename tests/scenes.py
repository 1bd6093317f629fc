"""Small hand-built scenes for the oracle pins and the GPU parity tests."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from workloads import Gaussians, Grid


def gaussians(mean, scale, quat, density):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    return Gaussians(f(np.atleast_2d(mean)), f(np.atleast_2d(scale)), f(np.atleast_2d(quat)),
                     f(np.atleast_1d(density)))


def random_scene(seed, m, lo=0.05, hi=0.2, box=0.5, rho=(0.5, 1.0)):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-box, box, (m, 3))
    scale = rng.uniform(lo, hi, (m, 3))
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    dens = rng.uniform(*rho, m)
    return gaussians(mean, scale, q, dens)


def lattice(seed=7, rot_seed=3, n_side=3, spacing=0.3):
    """Strongly anisotropic Gaussians (axis ratios up to 8:1) on a jittered
    cubic lattice, densities in [0.5, 1]."""
    rng = np.random.default_rng(seed)
    m = n_side ** 3
    ax = (np.arange(n_side) - (n_side - 1) / 2) * spacing
    mean = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    mean = mean + rng.uniform(-0.03, 0.03, (m, 3))
    scale = np.stack([rng.uniform(0.02, 0.04, m), rng.uniform(0.04, 0.08, m),
                      rng.uniform(0.1, 0.16, m)], 1)
    q = Rotation.random(m, random_state=rot_seed).as_quat()[:, [3, 0, 1, 2]]
    return gaussians(mean, scale, q, rng.uniform(0.5, 1.0, m))


def scipy_covariance(g):
    """Sigma = R diag(s^2) R^T with R from scipy (Hamilton, active); quaternions
    are stored (w,x,y,z) and scipy takes (x,y,z,w)."""
    q = g.quat.astype(np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    s2 = g.scale.astype(np.float64) ** 2
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


def line_integral(g, o, d):
    """Exact integral of sum_i rho_i exp(-1/2 (x-p_i)^T Sigma_i^{-1} (x-p_i))
    along the full line o + t d (|d| = 1); o, d [...,3].  Closed form of a
    Gaussian integral: rho sqrt(2 pi / a) exp(-(c - b^2/a)/2), evaluated at the
    line point closest to the centre to avoid cancellation."""
    Sig = scipy_covariance(g)
    P = np.linalg.inv(Sig)
    out = np.zeros(o.shape[:-1])
    for i in range(g.n):
        p = g.mean[i].astype(np.float64)
        a = np.einsum("...i,ij,...j->...", d, P[i], d)
        b = np.einsum("...i,ij,...j->...", d, P[i], o - p)
        o2 = o - (b / a)[..., None] * d
        c = np.einsum("...i,ij,...j->...", o2 - p, P[i], o2 - p)
        out += float(g.density[i]) * np.sqrt(2 * math.pi / a) * np.exp(-0.5 * c)
    return out


def pixel_centres(view):
    w, h = view["width"], view["height"]
    u = (np.arange(w) + 0.5 - w / 2) * view["hu"] + view["off_u"]
    v = (np.arange(h) + 0.5 - h / 2) * view["hv"] + view["off_v"]
    return u, v


def cone_geometry(theta, src_obj, src_det):
    """Scanner of App. A written from its description: source on a circle of
    radius L_SO about the z axis at angle theta, detector perpendicular to the
    central ray (pointing at the rotation centre) at distance L_SD from the
    source, detector u axis (-sin t, cos t, 0), v axis (0, 0, -1)."""
    c, s = math.cos(theta), math.sin(theta)
    src = src_obj * np.array([c, s, 0.0])
    axis = -np.array([c, s, 0.0])
    u_ax = np.array([-s, c, 0.0])
    v_ax = np.array([0.0, 0.0, -1.0])
    return src, axis, u_ax, v_ax


def cone_rays(view, theta):
    src, axis, u_ax, v_ax = cone_geometry(theta, view["L_SO"], view["L_SD"])
    u, v = pixel_centres(view)
    det = src + view["L_SD"] * axis
    pts = det + v[:, None, None] * v_ax + u[None, :, None] * u_ax
    d = pts - src
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.broadcast_to(src, d.shape).copy(), d


def grid(n, lo=-1.0, hi=1.0):
    h = (hi - lo) / n
    return Grid(n, n, n, (lo, lo, lo), (h, h, h))
