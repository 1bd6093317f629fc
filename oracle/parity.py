"""Tolerance rules for comparing a GPU result with the oracle.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU baseline).

Forward, per output element:
    |gpu - oracle| <= rel * S + amb + floor * max(S)
  S = sum of |terms| of that element, amb = the terms whose Mahalanobis
  distance lies within 1e-3 kappa^2 of the cutoff (FP32 and FP64 may decide
  those differently), rel = 1e-4 (forward tolerance of the method's FP32
  port), floor = 1e-7 (terms far below FP32 resolution of the image).
Gradients, per parameter:
    |gpu - oracle| <= rel * S_abs + amb
  S_abs = sum over (view, pixel) of |per-pixel contribution| through the
  chain rule, rel = 1e-3; plus, per block (mean, scale, quat, density),
  ||gpu - oracle||_2 <= rel * ||oracle||_2.  There is no absolute floor: S_abs
  bounds the FP32 rounding of every term that enters a parameter's gradient.
Image-loss gradient (Eq. 8, L1 + lambda D-SSIM), per pixel:
    |gpu - oracle| <= rel * ssim_abs + 4 eps (l1_abs + ssim_abs)
  ssim_abs = the D-SSIM part's sum of |terms| (oracle.image_loss_grad_scale),
  rel = 1e-3 as for gradients; the L1 part sign(x - y)/N is the same decision
  on both sides (the same FP32 inputs), so it only carries the rounding of
  the final expression, a few units of eps = 2^-24 of its terms.
"""
from __future__ import annotations

import numpy as np


def forward_violation(gpu, ref, rel=1e-4, floor=1e-7):
    """Largest |err| / tolerance over all elements (<= 1 passes)."""
    gpu = np.asarray(gpu, np.float64)
    img = ref.get("image", ref.get("volume"))
    S, amb = ref["S"], ref["amb"]
    tol = rel * S + amb + floor * max(float(S.max()), 1e-30) + 1e-30
    err = np.abs(gpu - img)
    return float((err / tol).max()), err


def grad_violation(gpu, ref, rel=1e-3, keys=("mean", "scale", "quat", "density")):
    """Returns (worst elementwise ratio, worst norm ratio, per-key detail)."""
    worst_el, worst_norm, detail = 0.0, 0.0, {}
    for k in keys:
        g = np.asarray(gpu[k], np.float64)
        o = ref[k]
        sa = ref["S_abs"][k]
        am = ref["amb"][k]
        tol = rel * sa + am + 1e-30
        el = float((np.abs(g - o) / tol).max()) if g.size else 0.0
        nr = float(np.linalg.norm(g - o) / (rel * np.linalg.norm(o) + 1e-30))
        worst_el = max(worst_el, el)
        worst_norm = max(worst_norm, nr)
        detail[k] = (el, nr)
    return worst_el, worst_norm, detail


def loss_grad_violation(gpu, ref, scale, rel=1e-3, eps=2.0 ** -24):
    """Largest |err| / tolerance of an image-loss gradient (<= 1 passes);
    scale = oracle.image_loss_grad_scale(...)."""
    ssim_abs, l1_abs = scale
    tol = rel * ssim_abs + 4 * eps * (l1_abs + ssim_abs) + 1e-300
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    return float((err / tol).max())
