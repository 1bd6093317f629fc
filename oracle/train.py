"""FP64 CPU oracle for the training loop around the rasterizer: parameter
activations, Adam with the exponential learning-rate schedule, adaptive
density control, and the 3D evaluation metrics (Sec. 3.3, Sec. 4.1).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.
It shares no code with the HIP path.

Readings of points the paper leaves open (it defers to 3DGS for them):
  * activations: mean as is; scale s = exp(s_raw); quaternion as is (the
    operators normalise it); density rho = softplus(rho_raw) = log(1 + e^x);
  * Adam (Kingma & Ba, Algorithm 1) with beta1 = 0.9, beta2 = 0.999,
    eps = 1e-15, one step counter shared by all Gaussians; the gradient is
    taken with respect to the raw parameters (chain rule through the
    activations);
  * learning rate of 0-based iteration k out of T: lr0 * r^(k/T), r = 0.1;
  * adaptive control: the statistic is the mean over the views in which a
    Gaussian is visible of |dL/dp_hat| in normalised device coordinates
    (detector half-width = 1); Gaussians whose mean reaches the threshold are
    cloned when their largest scale is at most clone_max_scale and split
    otherwise.  A clone keeps the Gaussian and adds a copy; a split replaces
    it by two children at p + R (s * z_k), z_k ~ N(0, I) (draws passed in),
    with scales s / 1.6.  Both resulting Gaussians get half the density
    (Sec. 3.3).  A resulting Gaussian whose density is below min_density is
    removed ("empty"); large Gaussians are never removed (Sec. 3.3).  New
    Gaussians start with zero Adam moments; a clone's original keeps its own.
    Outputs keep source order, each source emitting its 0, 1 or 2 results in
    place (the composition is an order-free sum, so order only matters for
    comparing arrays).  The density decisions compare the FP32 raw density
    with FP32 thresholds softplus^-1(min) and softplus^-1(2 min), and the
    scale decision compares the FP32 raw log-scale with FP32 log(clone_max),
    so that both implementations decide identically on identical inputs;
  * metrics: PSNR = 10 log10(R^2 / MSE) over the volume with R = max(gt);
    SSIM = the mean over the three axes of the mean SSIM of the slices
    normal to that axis (the D-SSIM window, data range R).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ssim as _ssim

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15
SPLIT_SCALE_DIV = 1.6
KEYS = ("mean", "scale", "quat", "density")


def softplus(x):
    x = np.asarray(x, np.float64)
    return np.where(x > 30.0, x, np.log1p(np.exp(np.minimum(x, 30.0))))


def softplus_inv(y):
    y = np.asarray(y, np.float64)
    return np.where(y > 30.0, y, np.log(np.expm1(np.minimum(y, 30.0))))


def activate(raw):
    """Post-activation parameters (what the rasterizer consumes) from the raw
    trainable ones: {"mean", "scale", "quat", "density"} -> same keys."""
    return {"mean": np.asarray(raw["mean"], np.float64),
            "scale": np.exp(np.asarray(raw["scale"], np.float64)),
            "quat": np.asarray(raw["quat"], np.float64),
            "density": softplus(raw["density"])}


def activation_slope(raw):
    """d post / d raw, elementwise."""
    rd = np.asarray(raw["density"], np.float64)
    return {"mean": np.ones_like(np.asarray(raw["mean"], np.float64)),
            "scale": np.exp(np.asarray(raw["scale"], np.float64)),
            "quat": np.ones_like(np.asarray(raw["quat"], np.float64)),
            "density": 1.0 / (1.0 + np.exp(-rd))}


def learning_rate(lr0, k, total, final_ratio=0.1):
    """Exponential decay from lr0 at k = 0 to final_ratio * lr0 at k = total
    (Sec. 4.1)."""
    return lr0 * final_ratio ** (k / total)


def adam_step(raw, m, v, grad_post, step, lrs):
    """One Adam update (Kingma & Ba, Algorithm 1) of the raw parameters.
    grad_post: gradient with respect to the post-activation parameters;
    step: 1-based step count; lrs: {key: learning rate}.  Returns new
    (raw, m, v) dicts in float64."""
    slope = activation_slope(raw)
    out_raw, out_m, out_v = {}, {}, {}
    for k in KEYS:
        g = np.asarray(grad_post[k], np.float64) * slope[k]
        mk = BETA1 * np.asarray(m[k], np.float64) + (1 - BETA1) * g
        vk = BETA2 * np.asarray(v[k], np.float64) + (1 - BETA2) * g * g
        mhat = mk / (1 - BETA1 ** step)
        vhat = vk / (1 - BETA2 ** step)
        out_raw[k] = np.asarray(raw[k], np.float64) - lrs[k] * mhat / (np.sqrt(vhat) + EPS)
        out_m[k], out_v[k] = mk, vk
    return out_raw, out_m, out_v


def ndc_gradient_norm(grad2d, views):
    """|dL/dp_hat| in normalised device coordinates per (view, Gaussian) from
    the detector-unit gradient [V][n][2]: NDC u = 2 (pixel u) / width - 1."""
    out = np.zeros(grad2d.shape[:2])
    for v, view in enumerate(views):
        su = view["hu"] * view["width"] / 2
        sv = view["hv"] * view["height"] / 2
        out[v] = np.hypot(grad2d[v, :, 0] * su, grad2d[v, :, 1] * sv)
    return out


def _quat_rotation(q):
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def densify(raw, m, v, grad_sum, visible, normals, grad_threshold, clone_max_scale,
            min_density, densify_on=True):
    """Adaptive control (Sec. 3.3) on FP32 raw parameters (dict of arrays),
    Adam moments m, v (same layout), accumulated statistics grad_sum [n] (FP32)
    and visible [n] (int), and normals [n][2][3] (the split draws).
    Returns (raw, m, v, action) with action[i] in {0 prune, 1 keep, 2 clone,
    3 split} per source Gaussian."""
    f32 = np.float32
    rd = np.asarray(raw["density"], f32)
    ls = np.asarray(raw["scale"], f32)
    t_keep = f32(softplus_inv(min_density))
    t_half = f32(softplus_inv(2.0 * min_density))
    t_scale = f32(math.log(clone_max_scale))
    thr = f32(grad_threshold)
    gsum = np.asarray(grad_sum, f32)
    cnt = np.asarray(visible, np.int64)
    n = rd.shape[0]
    outs = {k: [] for k in KEYS}
    om = {k: [] for k in KEYS}
    ov = {k: [] for k in KEYS}
    action = np.zeros(n, np.int32)
    for i in range(n):
        avg = gsum[i] / f32(cnt[i]) if cnt[i] > 0 else f32(0.0)
        grow = densify_on and cnt[i] > 0 and avg >= thr
        if not grow:
            if rd[i] < t_keep:
                action[i] = 0
                continue
            action[i] = 1
            for k in KEYS:
                outs[k].append(np.asarray(raw[k][i], np.float64))
                om[k].append(np.asarray(m[k][i], np.float64))
                ov[k].append(np.asarray(v[k][i], np.float64))
            continue
        if rd[i] < t_half:       # both halves would be empty
            action[i] = 0
            continue
        half = softplus_inv(softplus(float(rd[i])) / 2.0)
        zero = {k: np.zeros_like(np.asarray(m[k][i], np.float64)) for k in KEYS}
        if ls[i].max() <= t_scale:
            action[i] = 2
            for copy in range(2):
                for k in KEYS:
                    val = np.asarray(raw[k][i], np.float64).copy()
                    if k == "density":
                        val = np.float64(half)
                    outs[k].append(val)
                    om[k].append(np.asarray(m[k][i], np.float64) if copy == 0 else zero[k])
                    ov[k].append(np.asarray(v[k][i], np.float64) if copy == 0 else zero[k])
        else:
            action[i] = 3
            p = np.asarray(raw["mean"][i], np.float64)
            s = np.exp(np.asarray(raw["scale"][i], np.float64))
            R = _quat_rotation(np.asarray(raw["quat"][i], np.float64))
            for c in range(2):
                z = np.asarray(normals[i][c], np.float64)
                child = {"mean": p + R @ (s * z),
                         "scale": np.asarray(raw["scale"][i], np.float64) - math.log(SPLIT_SCALE_DIV),
                         "quat": np.asarray(raw["quat"][i], np.float64).copy(),
                         "density": np.float64(half)}
                for k in KEYS:
                    outs[k].append(child[k])
                    om[k].append(zero[k])
                    ov[k].append(zero[k])
    shapes = {"mean": (3,), "scale": (3,), "quat": (4,), "density": ()}
    stack = lambda lst, k: (np.stack(lst).reshape((-1,) + shapes[k]) if lst
                            else np.zeros((0,) + shapes[k]))
    return ({k: stack(outs[k], k) for k in KEYS}, {k: stack(om[k], k) for k in KEYS},
            {k: stack(ov[k], k) for k in KEYS}, action)


def volume_psnr(vol, gt):
    """PSNR of a reconstructed volume against the ground truth (Sec. 4.1),
    data range max(gt)."""
    vol = np.asarray(vol, np.float64)
    gt = np.asarray(gt, np.float64)
    mse = np.mean((vol - gt) ** 2)
    return 10.0 * math.log10(gt.max() ** 2 / mse)


def volume_ssim(vol, gt):
    """Mean over the three axes of the mean 2D SSIM of the slices normal to
    each axis (Sec. 4.1), data range max(gt)."""
    r = float(np.max(gt))
    x = torch.tensor(np.asarray(vol, np.float64) / r)
    y = torch.tensor(np.asarray(gt, np.float64) / r)
    vals = []
    for axis in range(3):
        xs = x.movedim(axis, 0).contiguous()
        ys = y.movedim(axis, 0).contiguous()
        vals.append(float(_ssim(xs, ys)))
    return float(np.mean(vals))


# ---------------------------------------------------------------------------
# Split draws: a counter-based generator, so that both implementations draw
# the same normals without passing them around
# ---------------------------------------------------------------------------

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
    numbers: as easy as 1, 2, 3", SC 2011): each round multiplies words 0 and
    2 by the two constants, exchanges and xors the 32-bit halves with the
    other words and the key; the key advances by the Weyl constants between
    rounds.  ctr: 4 ints, key: 2 ints; returns 4 ints."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in ctr)
    k0, k1 = (int(x) & MASK32 for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W[0]) & MASK32
            k1 = (k1 + PHILOX_W[1]) & MASK32
        p0 = PHILOX_M[0] * c0
        p1 = PHILOX_M[1] * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK32, p1 & MASK32, \
                         ((p0 >> 32) ^ c3 ^ k1) & MASK32, p0 & MASK32
    return c0, c1, c2, c3


def random_normals(seed, counter, n):
    """n standard normal draws: block b gives four words
    philox4x32_10((b, counter_lo, counter_hi, 0), (seed_lo, seed_hi)); each
    word x becomes u = (x + 1/2) / 2^32 in (0, 1), and the pairs (u0, u1),
    (u2, u3) become sqrt(-2 ln u) cos 2 pi v, sqrt(-2 ln u) sin 2 pi v
    (Box & Muller 1958).  Element 4b + k is the k-th normal of block b."""
    out = np.zeros(((n + 3) // 4) * 4)
    key = (seed & MASK32, (seed >> 32) & MASK32)
    for b in range((n + 3) // 4):
        x = philox4x32_10((b, counter & MASK32, (counter >> 32) & MASK32, 0), key)
        u = [(xi + 0.5) / 2.0 ** 32 for xi in x]
        for j in (0, 2):
            r = math.sqrt(-2.0 * math.log(u[j]))
            out[4 * b + j] = r * math.cos(2 * math.pi * u[j + 1])
            out[4 * b + j + 1] = r * math.sin(2 * math.pi * u[j + 1])
    return out[:n]
