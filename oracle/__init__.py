"""FP64 CPU oracle for R^2-Gaussian's X-ray rasterizer, voxelizer and losses.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this package.  It shares
no code with the HIP path (``paper_2405_20693_amd``) and imports nothing from it.

Split of the work:
  * per-Gaussian quantities are written here in float64 PyTorch, in the
    paper's notation and order (Sec. 3.1, Sec. 3.2.1, Eq. 3, Eq. 6, Eq. 7,
    App. A Eq. 10-11); gradients with respect to the Gaussian parameters are
    PyTorch autograd of these plain definitions;
  * the sums over pixels and voxels (Eq. 4, Eq. 7) and their derivatives with
    respect to the per-Gaussian quantities run in ``oracle.c`` (FP64, OpenMP
    over views or z-slabs, fixed loop order per output element);
  * the loss terms (Eq. 8) are float64 PyTorch with autograd.

Readings of points the paper leaves open (quaternion convention, third row of
the local affine Jacobian, pixel sampling, cutoff, TV and D-SSIM forms) are the
ones listed with the design notes; each function below names the reading it
takes.  The interface carries FP32 inputs and FP32 geometry; the oracle widens
exactly those FP32 values to FP64.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

BEAM_PARALLEL = 0
BEAM_CONE = 1
AMB_REL = 1e-3   # ambiguity band |q - kappa^2| <= AMB_REL * kappa^2 (same as oracle.c)


def build(force=True):
    """Compile oracle.c with gcc (FP64, -O2, OpenMP, no fast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src,
                    "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _LIB_PATH)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.orc_splat2d.argtypes = [i64, i64, P, i32, i32, P, f64, i32, P, P, P, P]
        lib.orc_splat2d_bwd.argtypes = [i64, i64, P, i32, i32, P, f64, i32, P, P, P, P, P]
        lib.orc_splat3d.argtypes = [i64, P, i32, i32, i32, P, f64, i32, P, P, P, P]
        lib.orc_splat3d_bwd.argtypes = [i64, P, i32, i32, i32, P, f64, i32, P, P, P, P, P]
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_max_threads.restype = i32
        _lib = lib
    return _lib


def set_threads(n):
    """Threads of the oracle's C sums and of its float64 torch parts; returns
    the previous (C threads, torch threads).  Results do not depend on it."""
    lib = _load()
    prev = (int(lib.orc_max_threads()), torch.get_num_threads())
    lib.orc_set_threads(int(n))
    torch.set_num_threads(int(n))
    return prev


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32to64(x):
    return float(np.float32(x))


# ---------------------------------------------------------------------------
# Scanner geometry (App. A)
# ---------------------------------------------------------------------------

def cone_view(theta, src_obj, src_det, width, height, pitch, off_u=0.0, off_v=0.0):
    """World -> scanner rotation of App. A, Eq. 10: rows (-sin t, cos t, 0),
    (0, 0, -1), (-cos t, -sin t, 0); translation (0, 0, L_SO).  The source is
    the scanner origin; the detector plane sits at depth L_SD.  The rotation is
    evaluated in float64 and rounded to FP32, as the interface carries it."""
    s, c = math.sin(theta), math.cos(theta)
    W = np.array([[-s, c, 0.0], [0.0, 0.0, -1.0], [-c, -s, 0.0]])
    return {"beam": BEAM_CONE, "W": W.astype(np.float32).astype(np.float64),
            "L_SO": _f32to64(src_obj), "L_SD": _f32to64(src_det),
            "width": int(width), "height": int(height),
            "hu": _f32to64(pitch), "hv": _f32to64(pitch),
            "off_u": _f32to64(off_u), "off_v": _f32to64(off_v)}


def parallel_view(rot, width, height, pitch, off_u=0.0, off_v=0.0):
    """Parallel beam (the L_SO -> infinity limit): rows of `rot` are the
    detector u axis, v axis and the ray direction."""
    W = np.asarray(rot, np.float64).astype(np.float32).astype(np.float64)
    return {"beam": BEAM_PARALLEL, "W": W, "L_SO": 0.0, "L_SD": 0.0,
            "width": int(width), "height": int(height),
            "hu": _f32to64(pitch), "hv": _f32to64(pitch),
            "off_u": _f32to64(off_u), "off_v": _f32to64(off_v)}


def views_from_scan(scan):
    """Oracle views for a workloads.ConeScan / ParallelScan."""
    if hasattr(scan, "thetas"):
        return [cone_view(t, scan.src_obj, scan.src_det, scan.width, scan.height, scan.pitch)
                for t in scan.thetas]
    return [parallel_view(r, scan.width, scan.height, scan.pitch) for r in scan.rots]


# ---------------------------------------------------------------------------
# Per-Gaussian quantities (float64 torch, differentiable)
# ---------------------------------------------------------------------------

def _params(g, requires_grad=False):
    t = [torch.tensor(np.asarray(a, np.float32), dtype=torch.float64, requires_grad=requires_grad)
         for a in (g.mean, g.scale, g.quat, g.density)]
    return t


def _valid_gaussian(mean, scale, quat, density):
    fin = (torch.isfinite(mean).all(1) & torch.isfinite(scale).all(1) &
           torch.isfinite(quat).all(1) & torch.isfinite(density))
    return fin & (scale > 0).all(1) & (quat.abs().sum(1) > 0)


def _safe(mean, scale, quat, density, ok):
    """Replace skipped Gaussians' parameters by benign values so that no NaN
    reaches autograd; their outputs are masked to zero afterwards."""
    k = ok[:, None]
    one = torch.ones_like(scale)
    e0 = torch.zeros_like(quat)
    e0[:, 0] = 1.0
    return (torch.where(k, mean, torch.zeros_like(mean)), torch.where(k, scale, one),
            torch.where(k, quat, e0), torch.where(ok, density, torch.zeros_like(density)))


def rotation(quat):
    """R from a quaternion (w, x, y, z), Hamilton convention, normalised first
    (the paper factorises Sigma = R S S^T R^T following 3DGS, Sec. 3.1)."""
    q = quat / quat.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def covariance(scale, quat):
    """Sigma = R S S^T R^T (Sec. 3.1)."""
    R = rotation(quat)
    return R @ torch.diag_embed(scale * scale) @ R.transpose(1, 2)


def precision(scale, quat):
    """Sigma^{-1} = R S^{-2} R^T."""
    R = rotation(quat)
    return R @ torch.diag_embed(1.0 / (scale * scale)) @ R.transpose(1, 2)


def project_gaussians(mean, scale, quat, density, view):
    """Transformation and projection modules for one view (Eq. 6, Eq. 7,
    App. A Eq. 10-11).

    Cone beam: t = W p + (0, 0, L_SO); the projective map is
    phi(t) = (L_SD t0/t2, L_SD t1/t2, |t|) (detector coordinates for the first
    two axes; the third axis is the distance along the ray, so that J, its
    Jacobian at t, is the local affine map of EWA splatting); Sigma_tilde =
    J W Sigma W^T J^T.  Parallel beam: t = W p, Sigma_tilde = W Sigma W^T.
    The 2D Gaussian keeps the first two rows/columns; the rectified density is
    rho_hat = sqrt(2 pi |Sigma_tilde| / |Sigma_hat|) rho (Eq. 7).

    Returns dict of per-Gaussian tensors and a validity mask (pairs with
    t2 <= 1e-3 L_SO are culled for cone beam).
    """
    ok = _valid_gaussian(mean, scale, quat, density)
    mean, scale, quat, density = _safe(mean, scale, quat, density, ok)
    W = torch.tensor(view["W"], dtype=torch.float64)
    Sigma = covariance(scale, quat)
    t = mean @ W.T
    if view["beam"] == BEAM_CONE:
        L_SO, L = view["L_SO"], view["L_SD"]
        t = t + torch.tensor([0.0, 0.0, L_SO], dtype=torch.float64)
        front = t[:, 2] > 1e-3 * L_SO
        ok = ok & front
        t2 = torch.where(front, t[:, 2], torch.ones_like(t[:, 2]))
        t0, t1 = t[:, 0], t[:, 1]
        l = torch.sqrt(t0 * t0 + t1 * t1 + t2 * t2)
        zero = torch.zeros_like(t0)
        J = torch.stack([
            torch.stack([L / t2, zero, -L * t0 / (t2 * t2)], 1),
            torch.stack([zero, L / t2, -L * t1 / (t2 * t2)], 1),
            torch.stack([t0 / l, t1 / l, t2 / l], 1),
        ], 1)
        JW = J @ W
        p_hat = torch.stack([L * t0 / t2, L * t1 / t2], 1)
    else:
        JW = W.expand(mean.shape[0], 3, 3)
        p_hat = t[:, :2]
    Sig_t = JW @ Sigma @ JW.transpose(1, 2)
    Sig_h = Sig_t[:, :2, :2]
    det_t = torch.linalg.det(Sig_t)
    det_h = Sig_h[:, 0, 0] * Sig_h[:, 1, 1] - Sig_h[:, 0, 1] * Sig_h[:, 1, 0]
    mu = torch.sqrt(2.0 * math.pi * det_t / det_h)
    rho_hat = mu * density
    A00 = Sig_h[:, 1, 1] / det_h
    A01 = -Sig_h[:, 0, 1] / det_h
    A11 = Sig_h[:, 0, 0] / det_h
    fin = torch.isfinite(rho_hat) & torch.isfinite(A00) & torch.isfinite(A11) & (det_h > 0)
    ok = ok & fin
    return {"p_hat": p_hat, "A": (A00, A01, A11), "rho_hat": rho_hat, "mu": mu,
            "Sigma_hat": Sig_h, "Sigma_tilde": Sig_t, "t": t, "ok": ok}


def _unrectify(pr, density):
    """The unrectified (3DGS-style) reading of Sec. 3.2.1 "Integration bias":
    the 2D Gaussian keeps the 3D central density, rho_hat = rho."""
    pr = dict(pr)
    pr["rho_hat"] = density * torch.ones_like(pr["rho_hat"])
    return pr


def _rec2d_array(pr, kappa):
    ok = pr["ok"].detach().numpy()
    A00, A01, A11 = (a.detach().numpy() for a in pr["A"])
    Sh = pr["Sigma_hat"].detach().numpy()
    rec = np.zeros((ok.shape[0], 9))
    rec[:, 0:2] = pr["p_hat"].detach().numpy()
    rec[:, 2], rec[:, 3], rec[:, 4] = A00, A01, A11
    rec[:, 5] = pr["rho_hat"].detach().numpy()
    with np.errstate(invalid="ignore"):
        rec[:, 6] = kappa * np.sqrt(np.maximum(Sh[:, 0, 0], 0.0))
        rec[:, 7] = kappa * np.sqrt(np.maximum(Sh[:, 1, 1], 0.0))
    rec[:, 8] = ok.astype(np.float64)
    rec[~ok, :8] = 0.0
    return rec


def _pix(views):
    return np.array([[v["hu"], v["hv"], v["off_u"], v["off_v"]] for v in views], np.float64)


def _check_views(views):
    w, h = views[0]["width"], views[0]["height"]
    assert all(v["width"] == w and v["height"] == h for v in views)
    return w, h


# ---------------------------------------------------------------------------
# Projection (X-ray rasterization)
# ---------------------------------------------------------------------------

def project(g, views, cutoff=3.0, brute=False, rectify=True):
    """Rendered projections I_r[v][b][a] (Eq. 7): sum over Gaussians of
    rho_hat exp(-q/2), q the Mahalanobis distance of the pixel centre under the
    projected covariance, terms with q <= cutoff^2 only (cutoff = inf keeps all).

    Returns dict: image, S (sum |terms|), amb (ambiguity mass), npairs [V].
    """
    lib = _load()
    width, height = _check_views(views)
    params = _params(g)
    nv, n = len(views), g.n
    rec = np.zeros((nv, n, 9))
    with torch.no_grad():
        for v, view in enumerate(views):
            pr = project_gaussians(*params, view)
            if not rectify:
                pr = _unrectify(pr, params[3])
            rec[v] = _rec2d_array(pr, cutoff)
    img = np.zeros((nv, height, width))
    S = np.zeros_like(img)
    amb = np.zeros_like(img)
    npairs = np.zeros(nv, np.int64)
    lib.orc_splat2d(nv, n, _ptr(rec), width, height, _ptr(_pix(views)), float(cutoff),
                    int(brute), _ptr(img), _ptr(S), _ptr(amb), _ptr(npairs))
    return {"image": img, "S": S, "amb": amb, "npairs": npairs}


_REC2D_KEYS = ("pu", "pv", "A00", "A01", "A11", "rho_hat")


def _rec2d_tensors(pr):
    A00, A01, A11 = pr["A"]
    m = pr["ok"].to(torch.float64)
    return [pr["p_hat"][:, 0] * m, pr["p_hat"][:, 1] * m, A00 * m, A01 * m, A11 * m,
            pr["rho_hat"] * m]


def project_grad(g, views, grad_image, cutoff=3.0, brute=False, select=None, with_scale=False,
                 rectify=True):
    """Gradient of L = sum G * I_r with respect to mean, scale, quat
    (unnormalised), density.  The cutoff indicator is treated as locally
    constant (its derivative is zero almost everywhere).

    select: optional index array; only those Gaussians' gradients are computed
    (the others are returned as zero).
    with_scale: also return, per parameter, S_abs = sum over pixels and views of
    |per-pixel contribution| (for tolerances) and amb = the same restricted to
    pixels within the ambiguity band of the cutoff.
    """
    lib = _load()
    width, height = _check_views(views)
    nv, n = len(views), g.n
    G = np.ascontiguousarray(np.asarray(grad_image, np.float64))
    sel = None
    if select is not None:
        sel = np.zeros(n, np.uint8)
        sel[np.asarray(select)] = 1
    params = _params(g, requires_grad=True)
    out = {k: torch.zeros_like(p) for k, p in zip(("mean", "scale", "quat", "density"), params)}
    sabs = {k: torch.zeros_like(p) for k, p in zip(("mean", "scale", "quat", "density"), params)}
    samb = {k: torch.zeros_like(p) for k, p in zip(("mean", "scale", "quat", "density"), params)}
    pix = _pix(views)
    for v, view in enumerate(views):
        pr = project_gaussians(*params, view)
        if not rectify:
            pr = _unrectify(pr, params[3])
        rec = _rec2d_array(pr, cutoff)
        d = np.zeros((n, 6))
        da = np.zeros((n, 6)) if with_scale else None
        dm = np.zeros((n, 6)) if with_scale else None
        lib.orc_splat2d_bwd(1, n, _ptr(rec), width, height, _ptr(pix[v:v + 1]), float(cutoff),
                            int(brute), _ptr(G[v]), _ptr(sel), _ptr(d), _ptr(da), _ptr(dm))
        comps = _rec2d_tensors(pr)
        loss = sum((c * torch.from_numpy(d[:, k])).sum() for k, c in enumerate(comps))
        grads = torch.autograd.grad(loss, params, retain_graph=with_scale, allow_unused=True)
        for k, gr in zip(out, grads):
            if gr is not None:
                out[k] += gr
        if with_scale:
            for k, c in enumerate(comps):
                jac = torch.autograd.grad(c.sum(), params, retain_graph=True, allow_unused=True)
                for key, jr in zip(out, jac):
                    if jr is None:
                        continue
                    w_abs = torch.from_numpy(da[:, k]).reshape(-1, *([1] * (jr.dim() - 1)))
                    w_amb = torch.from_numpy(dm[:, k]).reshape(-1, *([1] * (jr.dim() - 1)))
                    sabs[key] += jr.abs() * w_abs
                    samb[key] += jr.abs() * w_amb
    res = {k: t.detach().numpy() for k, t in out.items()}
    if with_scale:
        res["S_abs"] = {k: t.detach().numpy() for k, t in sabs.items()}
        res["amb"] = {k: t.detach().numpy() for k, t in samb.items()}
    return res


def grad2d(g, views, grad_image, cutoff=3.0, rectify=True):
    """Per (view, Gaussian): the gradient of L = sum G * I_r with respect to
    the projected centre p_hat (detector units, [V][n][2]) and whether the
    Gaussian is visible in the view.  Visible reading (the screen-space
    statistic of the adaptive control that Sec. 3.3 takes from 3DGS): some
    pixel centre lies inside the axis-aligned bounding box of the cutoff
    ellipse, |u - u_hat| <= kappa sqrt(Sigma_hat_uu) and |v - v_hat| <=
    kappa sqrt(Sigma_hat_vv).  ambiguous marks views where moving the box
    edges by 2e-3 pixel changes that answer."""
    lib = _load()
    width, height = _check_views(views)
    nv, n = len(views), g.n
    G = np.ascontiguousarray(np.asarray(grad_image, np.float64))
    params = _params(g)
    pix = _pix(views)
    gp = np.zeros((nv, n, 2))
    vis = np.zeros((nv, n), bool)
    amb = np.zeros((nv, n), bool)
    with torch.no_grad():
        for v, view in enumerate(views):
            pr = project_gaussians(*params, view)
            if not rectify:
                pr = _unrectify(pr, params[3])
            rec = _rec2d_array(pr, cutoff)
            d = np.zeros((n, 6))
            lib.orc_splat2d_bwd(1, n, _ptr(rec), width, height, _ptr(pix[v:v + 1]), float(cutoff),
                                0, _ptr(G[v]), None, _ptr(d), None, None)
            gp[v] = d[:, 0:2]
            hu, hv, ou, ov = pix[v]
            u = (np.arange(width) + 0.5 - width / 2) * hu + ou
            vv = (np.arange(height) + 0.5 - height / 2) * hv + ov
            ok = rec[:, 8] > 0

            def inside(margin):
                du = np.abs(u[None, :] - rec[:, 0:1]) <= rec[:, 6:7] + margin * hu
                dv = np.abs(vv[None, :] - rec[:, 1:2]) <= rec[:, 7:8] + margin * hv
                return ok & du.any(1) & dv.any(1)

            vis[v] = inside(0.0)
            amb[v] = inside(2e-3) != inside(-2e-3)
    return {"grad": gp, "visible": vis, "ambiguous": amb}


def mean_mu(g, views):
    """Mean over the views of each Gaussian's rectification factor
    mu = sqrt(2 pi |Sigma_tilde| / |Sigma_hat|) (views where it is culled are
    left out; 0 if culled in all); the X-3DGS correction divides the densities
    of an unrectified model by it before voxelization (Sec. 4.3)."""
    params = _params(g)
    tot = np.zeros(g.n)
    cnt = np.zeros(g.n)
    with torch.no_grad():
        for view in views:
            pr = project_gaussians(*params, view)
            ok = pr["ok"].numpy()
            tot[ok] += pr["mu"].numpy()[ok]
            cnt[ok] += 1
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0)


# ---------------------------------------------------------------------------
# Voxelization (Eq. 3, Eq. 4; Sec. 3.2.2)
# ---------------------------------------------------------------------------

def _geo(grid):
    return np.array(list(map(_f32to64, grid.origin)) + list(map(_f32to64, grid.spacing)), np.float64)


def _rec3d(params, kappa):
    mean, scale, quat, density = params
    ok = _valid_gaussian(mean, scale, quat, density)
    mean, scale, quat, density = _safe(mean, scale, quat, density, ok)
    P = precision(scale, quat)
    Sig = covariance(scale, quat)
    m = ok.to(torch.float64)
    comps = [mean[:, 0] * m, mean[:, 1] * m, mean[:, 2] * m,
             P[:, 0, 0] * m, P[:, 0, 1] * m, P[:, 0, 2] * m, P[:, 1, 1] * m, P[:, 1, 2] * m,
             P[:, 2, 2] * m, density * m]
    rec = np.zeros((mean.shape[0], 14))
    for k, c in enumerate(comps):
        rec[:, k] = c.detach().numpy()
    d = torch.diagonal(Sig, dim1=1, dim2=2).detach().numpy()
    rec[:, 10:13] = kappa * np.sqrt(np.maximum(d, 0.0))
    rec[:, 13] = ok.numpy().astype(np.float64)
    rec[~ok.numpy(), :13] = 0.0
    return rec, comps


def voxelize(g, grid, cutoff=3.0, brute=False):
    """Density volume V[k][j][i] = sigma(voxel centre) = sum_i rho_i
    exp(-q/2) over terms with q <= cutoff^2 (Eq. 4 with the per-voxel cutoff
    reading of the paper's 99%-confidence tile culling).  Returns dict:
    volume, S, amb, npairs."""
    lib = _load()
    params = _params(g)
    with torch.no_grad():
        rec, _ = _rec3d(params, cutoff)
    shape = (grid.nz, grid.ny, grid.nx)
    vol, S, amb = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    npairs = np.zeros(1, np.int64)
    lib.orc_splat3d(g.n, _ptr(rec), grid.nx, grid.ny, grid.nz, _ptr(_geo(grid)), float(cutoff),
                    int(brute), _ptr(vol), _ptr(S), _ptr(amb), _ptr(npairs))
    return {"volume": vol, "S": S, "amb": amb, "npairs": int(npairs[0])}


def voxelize_grad(g, grid, grad_volume, cutoff=3.0, brute=False, select=None, with_scale=False):
    """Gradient of L = sum H * V with respect to mean, scale, quat, density."""
    lib = _load()
    H = np.ascontiguousarray(np.asarray(grad_volume, np.float64))
    n = g.n
    sel = None
    if select is not None:
        sel = np.zeros(n, np.uint8)
        sel[np.asarray(select)] = 1
    params = _params(g, requires_grad=True)
    rec, comps = _rec3d(params, cutoff)
    d = np.zeros((n, 10))
    da = np.zeros((n, 10)) if with_scale else None
    dm = np.zeros((n, 10)) if with_scale else None
    lib.orc_splat3d_bwd(n, _ptr(rec), grid.nx, grid.ny, grid.nz, _ptr(_geo(grid)), float(cutoff),
                        int(brute), _ptr(H), _ptr(sel), _ptr(d), _ptr(da), _ptr(dm))
    loss = sum((c * torch.from_numpy(d[:, k])).sum() for k, c in enumerate(comps))
    keys = ("mean", "scale", "quat", "density")
    grads = torch.autograd.grad(loss, params, retain_graph=with_scale, allow_unused=True)
    res = {k: (gr.detach().numpy() if gr is not None else np.zeros(p.shape))
           for k, gr, p in zip(keys, grads, params)}
    if with_scale:
        sabs = {k: np.zeros(p.shape) for k, p in zip(keys, params)}
        samb = {k: np.zeros(p.shape) for k, p in zip(keys, params)}
        for k, c in enumerate(comps):
            jac = torch.autograd.grad(c.sum(), params, retain_graph=True, allow_unused=True)
            for key, jr in zip(keys, jac):
                if jr is None:
                    continue
                shp = (-1,) + (1,) * (jr.dim() - 1)
                sabs[key] += jr.abs().numpy() * da[:, k].reshape(shp)
                samb[key] += jr.abs().numpy() * dm[:, k].reshape(shp)
        res["S_abs"], res["amb"] = sabs, samb
    return res


# ---------------------------------------------------------------------------
# Losses (Eq. 8)
# ---------------------------------------------------------------------------

SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size=11, sigma=1.5):
    """Normalised 11x11 Gaussian window with sigma 1.5 (the SSIM paper's
    choice, which the D-SSIM term of Eq. 8 cites)."""
    x = torch.arange(size, dtype=torch.float64) - (size - 1) / 2
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    g = g / g.sum()
    return torch.outer(g, g)


def ssim(x, y):
    """Mean SSIM over pixels and images; local statistics from the 11x11
    window with zero padding ("same" size); data range 1."""
    w = ssim_window()[None, None]
    x = x[:, None]
    y = y[:, None]
    conv = lambda a: torch.nn.functional.conv2d(a, w, padding=5)
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    m = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / \
        ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))
    return m.mean()


def image_loss(render, measured, lambda_ssim=0.25):
    """L1 + lambda_ssim * (1 - SSIM) over a stack of projections (Eq. 8), with
    L1 the mean absolute difference.  Returns (total, l1, ssim, d total / d render)."""
    r = torch.tensor(np.asarray(render, np.float32), dtype=torch.float64, requires_grad=True)
    m = torch.tensor(np.asarray(measured, np.float32), dtype=torch.float64)
    l1 = (r - m).abs().mean()
    s = ssim(r, m)
    total = l1 + lambda_ssim * (1.0 - s)
    (gr,) = torch.autograd.grad(total, r)
    return float(total.detach()), float(l1.detach()), float(s.detach()), gr.numpy()


def image_loss_grad_scale(render, measured, lambda_ssim=0.25):
    """Per-pixel magnitudes that bound the FP32 rounding of d total / d render
    (for tolerances).  With the blurred statistics of the SSIM window at each
    pixel q and S(q) the SSIM map, the D-SSIM part of the gradient at pixel p is
      -lambda/N sum_q w(p - q) [D1(q) + 2 x(p) D2(q) + y(p) D3(q)],
    D2 = dS/dsxx, D3 = dS/dsxy, D1 = dS/dmx - 2 mx D2 - my D3 (chain rule of
    sxx = blur(x^2) - mx^2, sxy = blur(xy) - mx my).  Returns (ssim_abs, l1_abs):
    ssim_abs(p) = lambda/N sum_q w(p - q) [A1(q) + 2|x(p)| |D2(q)| + |y(p)| |D3(q)|]
    with A1 the sum of the absolute values of the terms of D1 (dS/dmx split in
    its two terms), and l1_abs(p) = |sign(x(p) - y(p))| / N."""
    x = torch.tensor(np.asarray(render, np.float32), dtype=torch.float64)
    y = torch.tensor(np.asarray(measured, np.float32), dtype=torch.float64)
    n_pix = x.numel()
    w = ssim_window()[None, None]
    conv = lambda a: torch.nn.functional.conv2d(a[:, None], w, padding=5)[:, 0]
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    A1, A2 = 2 * mx * my + SSIM_C1, 2 * sxy + SSIM_C2
    B1, B2 = mx * mx + my * my + SSIM_C1, sxx + syy + SSIM_C2
    S = A1 * A2 / (B1 * B2)
    dmx_a, dmx_b = 2 * my * A2 / (B1 * B2), 2 * mx * S / B1
    D2 = -S / B2
    D3 = 2 * A1 / (B1 * B2)
    a1 = dmx_a.abs() + dmx_b.abs() + 2 * mx.abs() * D2.abs() + my.abs() * D3.abs()
    blur_abs = lambda a: conv(a)  # the window is non-negative
    ssim_abs = lambda_ssim / n_pix * (blur_abs(a1) + 2 * x.abs() * blur_abs(D2.abs()) +
                                      y.abs() * blur_abs(D3.abs()))
    l1_abs = (x - y).sign().abs() / n_pix
    return ssim_abs.numpy(), l1_abs.numpy()


def tv(vol):
    """Anisotropic 3D total variation: for each axis, the mean absolute
    forward difference over the block; summed over the three axes."""
    v = vol
    return ((v[1:] - v[:-1]).abs().mean() + (v[:, 1:] - v[:, :-1]).abs().mean() +
            (v[:, :, 1:] - v[:, :, :-1]).abs().mean())


def tv_loss(volume, weight=1.0):
    """Returns (tv value, d (weight * tv) / d volume)."""
    v = torch.tensor(np.asarray(volume, np.float32), dtype=torch.float64, requires_grad=True)
    t = tv(v)
    (gv,) = torch.autograd.grad(weight * t, v)
    return float(t.detach()), gv.numpy()
