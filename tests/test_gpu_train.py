"""GPU tests of the optimisation-loop kernels (include/gs_train.h) against the
oracle: densification statistics, Adam, adaptive density control, volume
metrics, and the trainer's first iteration against the oracle's composition;
then properties of whole reconstructions on a synthetic phantom."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import train as ot
from tests import scenes
import workloads
from workloads import Grid, upstream

pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "quat", "density")


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20693_amd import ops as _ops
    return _ops


@pytest.fixture(scope="module")
def tr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20693_amd import train as _tr
    return _tr


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _gdev(g):
    return [_dev(a) for a in (g.mean, g.scale, g.quat, g.density)]


def _cone(ops, thetas, w, h, pitch):
    views = ops.Views.cone(thetas, 13.64, 20.46, w, h, pitch)
    oviews = [oracle.cone_view(t, 13.64, 20.46, w, h, pitch) for t in thetas]
    return views, oviews


# ------------------------------------------------------- statistics ------

def test_grad_stats_match_oracle(ops, tr):
    g = scenes.random_scene(81, 1500, lo=0.02, hi=0.1, box=0.9)
    views, ov = _cone(ops, [0.3, 1.2, 2.8, 4.0, 5.5], 72, 60, 0.035)
    G = upstream(11, (views.n, views.height, views.width))
    t = _gdev(g)
    plan = ops.Plan()
    ops.project_forward(*t, views, 3.0, plan)
    gsum = torch.full((g.n,), 0.5, device="cuda")
    vis = torch.full((g.n,), 2, device="cuda", dtype=torch.int32)
    tr.project_backward_stats(*t, views, _dev(G), plan, gsum, vis, stat_scale=3.0)
    torch.cuda.synchronize()
    ref = oracle.grad2d(g, ov, G)
    ndc = ot.ndc_gradient_norm(ref["grad"], ov)
    amb = ref["ambiguous"].any(0)
    exp_vis = ref["visible"].sum(0) + 2
    got_vis = vis.cpu().numpy()
    assert (got_vis[~amb] == exp_vis[~amb]).all()
    assert (np.abs(got_vis[amb] - exp_vis[amb]) <= ref["ambiguous"].sum(0)[amb]).all()
    exp = 0.5 + 3.0 * (ndc * ref["visible"]).sum(0)
    got = gsum.cpu().numpy()
    ok = ~amb
    err = np.abs(got[ok] - exp[ok])
    tol = 1e-3 * np.abs(exp[ok] - 0.5) + 2e-6 * np.abs(exp[ok]) + 1e-6 * (exp.max() - 0.5)
    print("stats worst ratio", float((err / tol).max()), "ambiguous", int(amb.sum()), flush=True)
    assert (err <= tol).all()


# ------------------------------------------------------------- Adam ------

def _random_state(seed, n):
    rng = np.random.default_rng(seed)
    raw = {"mean": rng.uniform(-0.5, 0.5, (n, 3)), "scale": np.log(rng.uniform(0.01, 0.1, (n, 3))),
           "quat": rng.standard_normal((n, 4)), "density": rng.uniform(-6, 2, n)}
    m = {k: rng.standard_normal(a.shape) * 1e-3 for k, a in raw.items()}
    v = {k: rng.uniform(0, 1e-5, a.shape) for k, a in raw.items()}
    f32 = lambda d: {k: a.astype(np.float32) for k, a in d.items()}
    return f32(raw), f32(m), f32(v)


def _state_to_gpu(tr, raw, m, v, cap=None):
    n = raw["density"].shape[0]
    st = tr.ParamState(cap or n)
    names = {"mean": "mean", "scale": "log_scale", "quat": "quat", "density": "density_raw"}
    for k in KEYS:
        st.t[names[k]][:n] = _dev(raw[k])
        st.t["m_" + k][:n] = _dev(m[k])
        st.t["v_" + k][:n] = _dev(v[k])
    return st


def test_adam_step_matches_oracle(tr):
    n = 3001
    raw, m, v = _random_state(12, n)
    rng = np.random.default_rng(13)
    gpost = {k: (rng.standard_normal(a.shape) * 10.0 ** rng.uniform(-6, 0, a.shape)).astype(np.float32)
             for k, a in raw.items()}
    lrs = {"mean": 2e-4, "scale": 5e-3, "quat": 1e-3, "density": 1e-2}
    st = _state_to_gpu(tr, raw, m, v)
    tr.adam_step(st, n, tuple(_dev(gpost[k]) for k in KEYS), lrs, step=7)
    torch.cuda.synchronize()
    lr32 = {k: float(np.float32(x)) for k, x in lrs.items()}
    r2, m2, v2 = ot.adam_step(raw, m, v, gpost, 7, lr32)
    names = {"mean": "mean", "scale": "log_scale", "quat": "quat", "density": "density_raw"}
    for k in KEYS:
        got = st.t[names[k]].cpu().numpy().astype(np.float64)
        # update error ~1e-5 of lr, plus the FP32 rounding of the parameter
        tol = 1e-5 * lr32[k] + 2.0 ** -23 * np.abs(r2[k]) * 2
        assert (np.abs(got - r2[k]) <= tol).all(), k
        # moments: FP32 rounding of beta m + (1 - beta) g with g the raw-space
        # gradient (the two terms can cancel, so the bound is on their sizes).
        # The kernel's g carries the activation slope's error (exp, divide:
        # ~3 ulp) and its product (~1 ulp); g^2 doubles that; the multiply-add
        # adds ~2 ulp.
        graw = gpost[k].astype(np.float64) * ot.activation_slope(raw)[k]
        u = 2.0 ** -24
        tol_m = 8 * u * (ot.BETA1 * np.abs(m[k]) + (1 - ot.BETA1) * np.abs(graw)) + 1e-30
        tol_v = 14 * u * (ot.BETA2 * np.abs(v[k]) + (1 - ot.BETA2) * graw * graw) + 1e-38
        assert (np.abs(st.t["m_" + k].cpu().numpy() - m2[k]) <= tol_m).all(), k
        assert (np.abs(st.t["v_" + k].cpu().numpy() - v2[k]) <= tol_v).all(), k
    act = ot.activate(r2)
    np.testing.assert_allclose(st.t["scale"].cpu().numpy(), act["scale"], rtol=2e-6)
    np.testing.assert_allclose(st.t["density"].cpu().numpy(), act["density"], rtol=3e-6, atol=1e-30)


def test_activation_round_trip(tr):
    g = scenes.random_scene(14, 500, lo=1e-3, hi=0.5, rho=(1e-6, 30.0))
    st = tr.ParamState.from_activated(*_gdev(g))
    torch.cuda.synchronize()
    np.testing.assert_allclose(st.t["log_scale"].cpu().numpy(), np.log(g.scale.astype(np.float64)),
                               rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(st.t["density_raw"].cpu().numpy(),
                               ot.softplus_inv(g.density.astype(np.float64)), rtol=2e-5, atol=2e-5)


# ---------------------------------------------------------- densify ------

def test_densify_matches_oracle(tr):
    n = 20000
    raw, m, v = _random_state(15, n)
    rng = np.random.default_rng(16)
    raw["density"] = rng.uniform(-9, 2, n).astype(np.float32)  # some below min_density
    vis = rng.integers(0, 5, n).astype(np.int32)
    gsum = (vis * 10.0 ** rng.uniform(-6, -3, n)).astype(np.float32)
    normals = rng.standard_normal((n, 2, 3)).astype(np.float32)
    cfg = dict(grad_threshold=5e-5, clone_max_scale=0.04, min_density=1e-3)
    st = _state_to_gpu(tr, raw, m, v)
    dst, n_out, action = tr.densify(st, n, _dev(gsum), _dev(vis, torch.int32), _dev(normals), **cfg)
    torch.cuda.synchronize()
    f = lambda x: float(np.float32(x))
    new, nm, nv, act = ot.densify(raw, m, v, gsum, vis, normals, f(cfg["grad_threshold"]),
                                  f(cfg["clone_max_scale"]), f(cfg["min_density"]))
    assert np.array_equal(action.cpu().numpy(), act), "decisions differ"
    assert n_out == new["density"].shape[0]
    counts = np.bincount(act, minlength=4)
    print("densify actions (removed, kept, cloned, split):", counts.tolist(), flush=True)
    assert (counts > 100).all()
    names = {"mean": "mean", "scale": "log_scale", "quat": "quat", "density": "density_raw"}
    for k in KEYS:
        got = dst.t[names[k]][:n_out].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, new[k], rtol=3e-6, atol=3e-6, err_msg=k)
        np.testing.assert_array_equal(dst.t["m_" + k][:n_out].cpu().numpy(), nm[k].astype(np.float32))
        np.testing.assert_array_equal(dst.t["v_" + k][:n_out].cpu().numpy(), nv[k].astype(np.float32))
    post = ot.activate(new)
    np.testing.assert_allclose(dst.t["scale"][:n_out].cpu().numpy(), post["scale"], rtol=5e-6)
    np.testing.assert_allclose(dst.t["density"][:n_out].cpu().numpy(), post["density"], rtol=5e-5,
                               atol=1e-30)


def test_densify_overflow_and_prune_only(tr):
    n = 1000
    raw, m, v = _random_state(17, n)
    vis = np.ones(n, np.int32)
    gsum = np.full(n, 1.0, np.float32)  # everything over the threshold
    st = _state_to_gpu(tr, raw, m, v)
    from paper_2405_20693_amd import _native as N
    with pytest.raises(N.GsError) as e:
        tr.densify(st, n, _dev(gsum), _dev(vis, torch.int32), _dev(np.zeros((n, 2, 3), np.float32)),
                   5e-5, 0.04, 1e-3, dst_capacity=n)
    assert "GS_EOVERFLOW" in str(e.value)
    dst, n_out, action = tr.densify(st, n, _dev(gsum), _dev(vis, torch.int32), None, 5e-5, 0.04, 1e-3,
                                    densify=False)
    torch.cuda.synchronize()
    keep = ot.softplus(raw["density"]) >= 1e-3
    a = action.cpu().numpy()
    assert set(np.unique(a)) <= {0, 1}
    assert n_out == int((a == 1).sum())
    assert abs(int(keep.sum()) - n_out) <= 2  # decisions at the FP32 threshold


# ---------------------------------------------------------- metrics ------

def test_volume_metrics_match_oracle(tr):
    rng = np.random.default_rng(18)
    gt = rng.uniform(0, 0.7, (30, 36, 41)).astype(np.float32)
    vol = (gt + rng.normal(0, 0.03, gt.shape)).astype(np.float32)
    ps, ss = tr.volume_metrics(_dev(vol), _dev(gt))
    assert abs(ps - ot.volume_psnr(vol, gt)) < 1e-5
    assert abs(ss - ot.volume_ssim(vol, gt)) < 2e-5
    ps2, ss2 = tr.volume_metrics(_dev(gt), _dev(gt))
    assert math.isinf(ps2) and abs(ss2 - 1.0) < 1e-6


# ---------------------------------------------------------- trainer ------

def _small_problem(seed=19, m=800, n_views=6, det=48):
    wl = workloads.c2_cone(m=m, n_views=n_views, det=det, pitch_mm=1.5 * 256 / det, seed=seed)
    return wl


@pytest.mark.parametrize("vidx,lambda_tv", [([4, 1], 0.05), ([0, 5, 2], 0.0), ([3], 0.05)])
def test_trainer_first_iteration_matches_oracle(ops, tr, vidx, lambda_tv):
    """One trainer iteration (explicit views and TV block) against the
    oracle's composition: image loss on the views, TV of the block, their
    gradients through the projection and voxelizer, then one Adam step.  Covers
    one view, a batch of views (measured images gathered) and no TV term."""
    wl = _small_problem()
    g = wl.gaussians
    views = ops.Views.from_scan(wl.scan)
    ov = oracle.views_from_scan(wl.scan)
    measured = workloads.measured_projections(wl)
    grid = Grid(40, 40, 40, (-1.0, -1.0, -1.0), (0.05, 0.05, 0.05))
    D = 12
    cfg = dict(iterations=100, densify_from=10 ** 6, tv_size=D, views_per_iter=len(vidx),
               lambda_tv=lambda_tv)
    trainer = tr.Trainer(*_gdev(g), _dev(measured), views, grid, **cfg)
    off = (7, 20, 3)
    loss = trainer.step(vidx, off)
    assert trainer.iteration() == 1
    mean, scale, quat, dens = (t.cpu().numpy().astype(np.float64) for t in trainer.model())
    trainer.close()
    # oracle composition
    oviews = [ov[i] for i in vidx]
    img = oracle.project(g, oviews)["image"]
    total, l1, s, gimg = oracle.image_loss(img.astype(np.float32), measured[vidx], 0.25)
    gp = oracle.project_grad(g, oviews, gimg)
    if lambda_tv > 0:
        block = Grid(D, D, D, tuple(grid.origin[k] + off[k] * grid.spacing[k] for k in range(3)),
                     grid.spacing)
        vol = oracle.voxelize(g, block)["volume"]
        tv, gvol = oracle.tv_loss(vol.astype(np.float32), lambda_tv)
        gv = oracle.voxelize_grad(g, block, gvol)
    else:
        tv, gv = 0.0, {k: 0.0 for k in KEYS}
    assert abs(loss - (total + lambda_tv * tv)) <= 1e-4 * abs(total + lambda_tv * tv)
    grad = {k: gp[k] + gv[k] for k in KEYS}
    raw = {"mean": g.mean.astype(np.float64), "scale": np.log(g.scale.astype(np.float64)),
           "quat": g.quat.astype(np.float64), "density": ot.softplus_inv(g.density.astype(np.float64))}
    zero = {k: np.zeros_like(a) for k, a in raw.items()}
    lrs = {"mean": 2e-4, "scale": 5e-3, "quat": 1e-3, "density": 1e-2}
    r2, _, _ = ot.adam_step(raw, zero, zero, grad, 1, lrs)
    got = {"mean": mean, "scale": np.log(scale), "quat": quat, "density": ot.softplus_inv(dens)}
    # first Adam step: lr * g / (|g| + eps) per element; where the gradient is
    # within its own FP32 error of zero, any step in [-lr, lr] is right
    for k in KEYS:
        d_got, d_ref = got[k] - raw[k], r2[k] - raw[k]
        small = np.abs(grad[k]) <= 1e-3 * np.abs(grad[k]).max()
        tol = 2e-3 * lrs[k] + 4 * 2.0 ** -23 * np.abs(raw[k])
        bad = (np.abs(d_got - d_ref) > tol) & ~small
        print(k, "elements off", int(bad.sum()), "of", bad.size, flush=True)
        assert not bad.any(), k
        assert (np.abs(d_got) <= lrs[k] * 1.001 + 4 * 2.0 ** -23 * np.abs(raw[k])).all()


def test_trainer_explicit_densify_step(ops, tr):
    """A step that is due to densify needs the split draws; with them the
    model changes size as the adaptive control decides, and stays finite."""
    wl = _small_problem(m=1500)
    views = ops.Views.from_scan(wl.scan)
    measured = _dev(workloads.measured_projections(wl))
    grid = Grid(40, 40, 40, (-1.0, -1.0, -1.0), (0.05, 0.05, 0.05))
    trainer = tr.Trainer(*_gdev(wl.gaussians), measured, views, grid, iterations=100, tv_size=8,
                         densify_from=1, densify_interval=2, grad_threshold=1e-6,
                         min_density=1e-3)
    trainer.step([0], (0, 0, 0))                       # iteration 1: no densification
    n = trainer.count()
    from paper_2405_20693_amd import _native as N
    with pytest.raises(N.GsError):
        trainer.step([1], (0, 0, 0))                   # iteration 2 densifies: draws missing
    trainer.close()
    trainer = tr.Trainer(*_gdev(wl.gaussians), measured, views, grid, iterations=100, tv_size=8,
                         densify_from=1, densify_interval=2, grad_threshold=1e-6,
                         min_density=1e-3)
    trainer.step([0], (0, 0, 0))
    normals = _dev(np.random.default_rng(3).standard_normal((n, 2, 3)).astype(np.float32))
    trainer.step([1], (5, 5, 5), normals)
    n2 = trainer.count()
    mean, scale, quat, dens = trainer.model()
    print(f"densify step: {n} -> {n2} Gaussians", flush=True)
    assert n2 > n                                      # tiny threshold: most Gaussians grow
    for t in (mean, scale, quat, dens):
        assert torch.isfinite(t).all()
    assert (scale > 0).all() and (dens > 0).all()
    vol, none = trainer.evaluate(grid)
    assert none is None and torch.isfinite(vol).all()
    trainer.close()


def test_trainer_reservation_overflow_skips_updates_and_recovers(ops, tr):
    """The trainer sizes its reserved tile lists from its first iteration.
    Scaling every Gaussian up 6x afterwards needs several times the entries: the
    iterations that overflow change no parameter (their Adam steps are
    guarded on the plans' overflow record), the run reports GS_EOVERFLOW, and
    the grown reservation lets the next run train."""
    import ctypes
    from paper_2405_20693_amd import _native as N
    wl = _small_problem(m=1500)
    views = ops.Views.from_scan(wl.scan)
    measured = _dev(workloads.measured_projections(wl))
    grid = Grid(40, 40, 40, (-1.0, -1.0, -1.0), (0.05, 0.05, 0.05))
    trainer = tr.Trainer(*_gdev(wl.gaussians), measured, views, grid, iterations=100, tv_size=8,
                         densify_from=10 ** 6)
    trainer.step([0], (0, 0, 0))  # sizes the reservation
    mean, scale, quat, dens = trainer.model()
    big = (6.0 * scale).contiguous()
    P, n = N.GsParams(), ctypes.c_int64()
    N.call("gs_trainer_state", trainer._h, ctypes.byref(P), ctypes.byref(n), None)
    tmp = N.GsParams(*[getattr(P, f) for f in N.PARAM_FIELDS])
    tmp.scale, tmp.density = big.data_ptr(), dens.data_ptr()
    torch.cuda.synchronize()
    N.call("gs_params_from_activated", ctypes.byref(tmp), n.value, None)  # raw from the new scales
    N.call("gs_params_activate", ctypes.byref(P), n.value, None)          # the trainer's copies
    torch.cuda.synchronize()
    before = trainer.model()
    assert torch.allclose(before[1], big, rtol=1e-5)
    with pytest.raises(N.GsError) as e:
        trainer.run(3)
    assert "GS_EOVERFLOW" in str(e.value)
    after = trainer.model()
    for a, b in zip(after, before):
        assert torch.equal(a, b)  # no update from an overflowing iteration
    losses = trainer.run(2)
    assert np.isfinite(losses).all()
    moved = trainer.model()
    assert not torch.equal(moved[0], before[0])
    trainer.close()


def _phantom_problem(n_views=24, det=96, m=6000, seed=21):
    """Reconstruction of the C3 head phantom from its exact projections: the
    initial Gaussians follow the paper's initialisation statistics (Sec. 3.3),
    with the phantom's density standing in for the FDK volume."""
    wl = workloads.c3_iteration(m=m, n_views=n_views, det=det, pitch_mm=0.75 * 512 / det, seed=seed)
    return wl


def test_trainer_reconstruction_improves_and_rectification_wins(ops, tr):
    """Rectified training and the X-3DGS variant from the same initial images
    (the unrectified model starts from rho * mean mu, which renders like the
    rectified initial model): both fit the projections, and the rectified model
    reconstructs the volume better (Sec. 4.3).  The densification threshold is
    scaled for the 96^2 detector: the per-pixel gradient of the mean loss in
    normalised device coordinates is about 5x the 512^2 value."""
    wl = _phantom_problem()
    views = ops.Views.from_scan(wl.scan)
    measured = _dev(workloads.measured_projections(wl))
    grid = Grid(64, 64, 64, (-1.0, -1.0, -1.0), (2 / 64, 2 / 64, 2 / 64))
    gt = _dev(workloads.phantom_volume(wl, grid))
    g0 = _gdev(wl.gaussians)
    mu, _ = ops.mean_mu(*g0, views)
    results = {}
    for rect in (1, 0):
        init = g0 if rect else g0[:3] + [(g0[3] * mu).contiguous()]
        trainer = tr.Trainer(*init, measured, views, grid, iterations=1500, tv_size=16,
                             densify_from=250, densify_until=1200, densify_interval=100,
                             grad_threshold=2.5e-4, rectify=rect, seed=5)
        _, (p0, s0) = trainer.evaluate(grid, gt)
        losses = trainer.run(1500)
        _, (p1, s1) = trainer.evaluate(grid, gt)
        n1 = trainer.count()
        trainer.close()
        print(f"rectify={rect}: loss {losses[:50].mean():.4g} -> {losses[-50:].mean():.4g}, "
              f"PSNR {p0:.2f} -> {p1:.2f}, SSIM {s0:.3f} -> {s1:.3f}, Gaussians "
              f"{wl.gaussians.n} -> {n1}", flush=True)
        assert np.isfinite(losses).all()
        assert losses[-50:].mean() < 0.7 * losses[:50].mean()
        assert p1 > p0 and s1 > s0
        results[rect] = (p1, s1, n1)
    # the integration bias costs 3D accuracy: the test checks the direction of
    # the paper's comparison (Sec. 4.3), rectified PSNR and SSIM above X-3DGS,
    # not the size of the gap, which the paper measures after 30k iterations
    # on its CT data and this 1500-iteration synthetic run cannot reproduce
    print(f"rectified minus X-3DGS: {results[1][0] - results[0][0]:+.2f} dB, "
          f"SSIM {results[1][1] - results[0][1]:+.4f}", flush=True)
    assert results[1][0] > results[0][0]
    assert results[1][1] > results[0][1]
    assert results[1][2] != wl.gaussians.n      # adaptive control ran


def test_random_normals_match_oracle(tr):
    """The device generator reproduces the oracle's Philox4x32-10 +
    Box-Muller draws (bit-exact words; the transform in double, rounded)."""
    for seed, counter, n in ((0, 0, 37), (12345, 7, 4001), (2 ** 40 + 3, 2 ** 33 + 5, 64)):
        got = tr.random_normals(seed, counter, n).cpu().numpy()
        ref = ot.random_normals(seed, counter, n)
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
