"""Pins of the training-loop oracle (oracle/train.py) against independent
implementations, closed forms and hand-built cases (CPU only)."""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

import oracle
from oracle import train as ot
from tests import scenes
import workloads

KEYS = ot.KEYS


def _raw(seed, n):
    rng = np.random.default_rng(seed)
    return {"mean": rng.uniform(-0.5, 0.5, (n, 3)), "scale": np.log(rng.uniform(0.02, 0.1, (n, 3))),
            "quat": rng.standard_normal((n, 4)), "density": rng.uniform(-4, 1, n)}


def test_adam_matches_torch_adam():
    """Three steps of oracle Adam against torch.optim.Adam driving the raw
    parameters of L = sum(g_post * act(raw)), whose raw gradient is g_post times
    the activation slope."""
    raw = _raw(1, 7)
    lrs = {"mean": 2e-4, "scale": 5e-3, "quat": 1e-3, "density": 1e-2}
    tp = {k: torch.tensor(raw[k], requires_grad=True) for k in KEYS}
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": lrs[k]} for k in KEYS],
                           betas=(ot.BETA1, ot.BETA2), eps=ot.EPS)
    m = {k: np.zeros_like(raw[k]) for k in KEYS}
    v = {k: np.zeros_like(raw[k]) for k in KEYS}
    rng = np.random.default_rng(2)
    for step in range(1, 4):
        gpost = {k: rng.standard_normal(raw[k].shape) for k in KEYS}
        act = {"mean": tp["mean"], "scale": torch.exp(tp["scale"]), "quat": tp["quat"],
               "density": torch.nn.functional.softplus(tp["density"])}
        loss = sum((act[k] * torch.tensor(gpost[k])).sum() for k in KEYS)
        opt.zero_grad()
        loss.backward()
        opt.step()
        raw, m, v = ot.adam_step(raw, m, v, gpost, step, lrs)
        for k in KEYS:
            np.testing.assert_allclose(raw[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_activations_and_inverse():
    x = np.array([-30.0, -3.0, 0.0, 0.5, 20.0, 40.0])
    np.testing.assert_allclose(ot.softplus(x), np.log1p(np.exp(x)), rtol=1e-15)
    np.testing.assert_allclose(ot.softplus_inv(ot.softplus(x[1:])), x[1:], rtol=1e-12)
    raw = _raw(3, 4)
    act = ot.activate(raw)
    np.testing.assert_allclose(act["scale"], np.exp(raw["scale"]))
    # slope against central differences
    sl = ot.activation_slope(raw)
    h = 1e-6
    fd = (ot.softplus(raw["density"] + h) - ot.softplus(raw["density"] - h)) / (2 * h)
    np.testing.assert_allclose(sl["density"], fd, rtol=1e-8)


def test_learning_rate_schedule():
    assert ot.learning_rate(0.01, 0, 30000) == 0.01
    assert abs(ot.learning_rate(0.01, 30000, 30000) - 0.001) < 1e-15
    assert abs(ot.learning_rate(2e-4, 15000, 30000) - 2e-4 * math.sqrt(0.1)) < 1e-18


def test_grad2d_parallel_beam_is_projected_mean_gradient():
    """Parallel beam: p_hat = (W0 . p, W1 . p) and nothing else depends on p,
    so dL/dp_hat = (W0 . dL/dp, W1 . dL/dp); dL/dp is pinned by differences."""
    g = scenes.random_scene(71, 40, lo=0.03, hi=0.1, box=0.5)
    rots = Rotation.random(2, random_state=21).as_matrix()
    views = [oracle.parallel_view(r, 48, 40, 0.03, 0.01, -0.02) for r in rots]
    G = workloads.upstream(5, (2, 40, 48))
    res = oracle.grad2d(g, views, G)
    for v, view in enumerate(views):
        gm = oracle.project_grad(g, [view], G[v:v + 1])["mean"]
        # dL/dp = W0 g_u + W1 g_v; the FP32-rounded rows are orthonormal only to
        # ~1e-7, so solve with their Gram matrix
        W2 = view["W"][:2]
        guv = np.linalg.solve(W2 @ W2.T, W2 @ gm.T).T
        np.testing.assert_allclose(res["grad"][v], guv, rtol=1e-9, atol=1e-12)
    ndc = ot.ndc_gradient_norm(res["grad"], views)
    np.testing.assert_allclose(ndc[0], np.hypot(res["grad"][0, :, 0] * 0.03 * 24,
                                                res["grad"][0, :, 1] * 0.03 * 20))


def test_visibility_at_the_detector_edge():
    """Isotropic Gaussians (sigma 0.1) on a parallel view whose pixel centres
    span u in [-0.45, 0.45] (pitch 0.1, 10 pixels): the cutoff box (3 sigma)
    reaches the last centre iff |u_hat| <= 0.75."""
    us = [0.0, 0.74, 0.76, -0.749, -0.7515, 2.0]
    g = scenes.gaussians([[u, 0.0, 0.0] for u in us], [[0.1] * 3] * len(us),
                         [[1, 0, 0, 0]] * len(us), [1.0] * len(us))
    view = oracle.parallel_view(np.eye(3), 10, 10, 0.1)
    res = oracle.grad2d(g, [view], np.zeros((1, 10, 10)))
    assert list(res["visible"][0]) == [True, True, False, True, False, False]
    assert not res["ambiguous"].any()




def test_densify_actions():
    s_small, s_big = math.log(0.01), math.log(0.2)
    raw = {"mean": np.arange(18, dtype=np.float64).reshape(6, 3) * 0.1,
           "scale": np.array([[s_small] * 3, [s_big, s_small, s_small], [s_small] * 3,
                              [s_small] * 3, [s_big] * 3, [s_small] * 3]),
           "quat": Rotation.random(6, random_state=4).as_quat()[:, [3, 0, 1, 2]],
           "density": ot.softplus_inv(np.array([0.5, 0.6, 1e-5, 1.5e-4, 0.2, 0.4]))}
    raw = {k: np.asarray(a, np.float32) for k, a in raw.items()}
    m = {k: np.ones_like(np.asarray(raw[k], np.float64)) for k in KEYS}
    v = {k: 2 * np.ones_like(np.asarray(raw[k], np.float64)) for k in KEYS}
    # statistics: Gaussian 0 and 1 and 3 over the threshold, 4 just below, 5 never visible
    gsum = np.array([3e-4, 2e-4, 9e-4, 1e-4, 1.9e-4, 1.0], np.float32)
    cnt = np.array([2, 2, 2, 1, 4, 0])
    z = np.zeros((6, 2, 3))
    z[1, 0] = [1.0, 0.0, 0.0]
    z[1, 1] = [0.0, -1.0, 0.0]
    new, nm, nv, act = ot.densify(raw, m, v, gsum, cnt, z, 5e-5, 0.02, 1e-4)
    # 0 clone, 1 split, 2 prune (empty), 3 over threshold but halves empty: pruned,
    # 4 keep (big, below threshold: never pruned for size), 5 keep
    assert list(act) == [2, 3, 0, 0, 1, 1]
    assert new["mean"].shape == (6, 3)
    half0 = ot.softplus(new["density"][:2])
    np.testing.assert_allclose(half0, [0.25, 0.25], rtol=1e-6)
    np.testing.assert_allclose(new["mean"][0], raw["mean"][0])
    np.testing.assert_allclose(new["mean"][1], raw["mean"][0])
    assert (nm["mean"][0] == 1).all() and (nm["mean"][1] == 0).all()
    assert (nv["density"][0] == 2) and (nv["density"][1] == 0)
    # split children: p + R (s * z)
    R = Rotation.from_quat(np.asarray(raw["quat"][1], np.float64)[[1, 2, 3, 0]]).as_matrix()
    s = np.exp(np.asarray(raw["scale"][1], np.float64))
    np.testing.assert_allclose(new["mean"][2], raw["mean"][1] + s[0] * R[:, 0], rtol=1e-12)
    np.testing.assert_allclose(new["mean"][3], raw["mean"][1] - s[1] * R[:, 1], rtol=1e-12)
    np.testing.assert_allclose(np.exp(new["scale"][2]), s / 1.6, rtol=1e-12)
    np.testing.assert_allclose(ot.softplus(new["density"][2:4]), [0.3, 0.3], rtol=1e-6)
    assert (nm["quat"][2:4] == 0).all()
    # untouched Gaussians keep everything
    np.testing.assert_array_equal(new["scale"][4], raw["scale"][4])
    np.testing.assert_array_equal(new["density"][5], raw["density"][5])
    assert (nm["mean"][4:] == 1).all() and (nv["mean"][4:] == 2).all()


def test_clone_preserves_the_density_field():
    """Cloning puts two half-density copies where one Gaussian was: the
    voxelized field is unchanged (Sec. 3.3's halving keeps the images too)."""
    g = scenes.random_scene(72, 30, lo=0.02, hi=0.05, box=0.5)
    raw = {"mean": g.mean, "scale": np.log(g.scale.astype(np.float64)).astype(np.float32),
           "quat": g.quat, "density": ot.softplus_inv(g.density.astype(np.float64)).astype(np.float32)}
    m = {k: np.zeros_like(np.asarray(raw[k], np.float64)) for k in KEYS}
    new, _, _, act = ot.densify(raw, m, m, np.ones(30, np.float32), np.ones(30), np.zeros((30, 2, 3)),
                                5e-5, 1.0, 1e-6)
    assert (act == 2).all()
    post = ot.activate(new)
    g2 = scenes.gaussians(post["mean"], post["scale"], post["quat"], post["density"])
    grid = workloads.Grid(24, 24, 24, (-0.6, -0.6, -0.6), (0.05, 0.05, 0.05))
    np.testing.assert_allclose(oracle.voxelize(g2, grid)["volume"], oracle.voxelize(g, grid)["volume"],
                               rtol=2e-6, atol=1e-9)


def test_volume_metrics():
    rng = np.random.default_rng(9)
    gt = rng.uniform(0, 0.8, (12, 14, 16))
    assert abs(ot.volume_psnr(gt + 0.01, gt) - 20 * math.log10(gt.max() / 0.01)) < 1e-9
    assert abs(ot.volume_ssim(gt, gt) - 1.0) < 1e-14
    # against per-slice SSIM with scipy's Gaussian filter, one axis at a time
    from scipy.ndimage import gaussian_filter
    vol = gt + rng.normal(0, 0.05, gt.shape)
    r = gt.max()

    def ssim2(a, b):
        f = lambda t: gaussian_filter(t, 1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
        mx, my = f(a), f(b)
        sxx, syy, sxy = f(a * a) - mx * mx, f(b * b) - my * my, f(a * b) - mx * my
        c1, c2 = 0.01 ** 2, 0.03 ** 2
        return np.mean(((2 * mx * my + c1) * (2 * sxy + c2)) /
                       ((mx * mx + my * my + c1) * (sxx + syy + c2)))

    per_axis = []
    for ax in range(3):
        a, b = np.moveaxis(vol / r, ax, 0), np.moveaxis(gt / r, ax, 0)
        per_axis.append(np.mean([ssim2(a[i], b[i]) for i in range(a.shape[0])]))
    assert abs(ot.volume_ssim(vol, gt) - np.mean(per_axis)) < 1e-12


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator."""
    assert ot.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    f = 0xFFFFFFFF
    assert ot.philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert ot.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344),
                            (0xA4093822, 0x299F31D0)) == (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_random_normals_statistics():
    z = ot.random_normals(seed=12345, counter=7, n=40000)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.03
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # other counters and seeds give other draws; a prefix is stable
    assert not np.allclose(z[:8], ot.random_normals(12345, 8, 8))
    assert not np.allclose(z[:8], ot.random_normals(12346, 7, 8))
    np.testing.assert_array_equal(z[:10], ot.random_normals(12345, 7, 10))
