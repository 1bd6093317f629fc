"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (oracle/parity.py): forward |gpu - oracle| <= 1e-4 S + amb +
1e-7 max S per element; gradients <= 1e-3 S_abs + amb per parameter and
1e-3 in norm per block.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import parity
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


def _dev(g):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.mean, g.scale, g.quat, g.density)]


def _np(grads):
    return {k: t.cpu().numpy() for k, t in zip(KEYS, grads)}


def _proj_fwd(ops, g, views, cutoff=3.0):
    plan = ops.Plan()
    img = ops.project_forward(*_dev(g), views, cutoff, plan)
    torch.cuda.synchronize()
    return img.cpu().numpy(), plan


def _report(name, v):
    print(f"{name}: worst tolerance ratio {v:.3g}", flush=True)


# ---------------------------------------------------------------- forward --

def test_c1_parallel_forward(ops):
    wl = workloads.c1_forward()
    views = ops.Views.from_scan(wl.scan)
    img, plan = _proj_fwd(ops, wl.gaussians, views)
    ref = oracle.project(wl.gaussians, oracle.views_from_scan(wl.scan))
    v, _ = parity.forward_violation(img, ref)
    _report("c1 projection", v)
    assert v <= 1.0
    st = plan.status()
    assert st["skipped"] == 0 and st["tile_entries"] > 0


def test_c1_voxel_forward(ops):
    wl = workloads.c1_forward()
    vol = ops.voxelize_forward(*_dev(wl.gaussians), ops.grid_from(wl.grid), 3.0, ops.Plan())
    torch.cuda.synchronize()
    ref = oracle.voxelize(wl.gaussians, wl.grid)
    v, _ = parity.forward_violation(vol.cpu().numpy(), ref)
    _report("c1 voxelize", v)
    assert v <= 1.0


@pytest.mark.parametrize("det", [(100, 75), (256, 256), (33, 17)])
def test_cone_forward_ragged(ops, det):
    """Cone beam on detectors that are not multiples of the 16-pixel tile,
    several views and a Gaussian count spanning several binning chunks."""
    w, h = det
    wl = workloads.c2_cone(m=9000, n_views=5, det=max(w, h), pitch_mm=1.5 * 256 / max(w, h))
    thetas = wl.scan.thetas
    views = ops.Views.cone(thetas, wl.scan.src_obj, wl.scan.src_det, w, h, wl.scan.pitch)
    oviews = [oracle.cone_view(t, wl.scan.src_obj, wl.scan.src_det, w, h, wl.scan.pitch) for t in thetas]
    img, _ = _proj_fwd(ops, wl.gaussians, views)
    ref = oracle.project(wl.gaussians, oviews)
    v, _ = parity.forward_violation(img, ref)
    _report(f"cone {det}", v)
    assert v <= 1.0


def test_parallel_offsets_and_rotations(ops):
    g = scenes.random_scene(31, 400, lo=0.02, hi=0.1, box=0.8)
    from scipy.spatial.transform import Rotation
    rots = Rotation.random(3, random_state=5).as_matrix()
    views = ops.Views.parallel(rots, 90, 70, 0.025, off_u=0.037, off_v=-0.051)
    ov = [oracle.parallel_view(r, 90, 70, 0.025, 0.037, -0.051) for r in rots]
    img, _ = _proj_fwd(ops, g, views)
    v, _ = parity.forward_violation(img, oracle.project(g, ov))
    _report("parallel offsets", v)
    assert v <= 1.0


def test_no_cutoff_matches_brute_force(ops):
    g = scenes.random_scene(32, 60, lo=0.03, hi=0.15)
    views = ops.Views.cone([0.2, 2.9], 13.64, 20.46, 40, 36, 0.05)
    ov = [oracle.cone_view(t, 13.64, 20.46, 40, 36, 0.05) for t in (0.2, 2.9)]
    img, _ = _proj_fwd(ops, g, views, cutoff=math.inf)
    v, _ = parity.forward_violation(img, oracle.project(g, ov, cutoff=math.inf, brute=True))
    _report("no cutoff", v)
    assert v <= 1.0


def test_voxel_ragged_grid_and_groups(ops):
    """A grid whose tile planes force several z groups, with ragged edges."""
    g = scenes.random_scene(33, 3000, lo=0.01, hi=0.05, box=0.9)
    grid = Grid(300, 230, 45, (-1.0, -0.95, -0.3), (2.0 / 300, 1.9 / 230, 0.6 / 45))
    vol = ops.voxelize_forward(*_dev(g), ops.grid_from(grid), 3.0, ops.Plan())
    torch.cuda.synchronize()
    v, _ = parity.forward_violation(vol.cpu().numpy(), oracle.voxelize(g, grid))
    _report("voxel ragged", v)
    assert v <= 1.0


# -------------------------------------------------------------- gradients --

def _check_proj_grad(ops, g, views, oviews, seed, cutoff=3.0):
    G = upstream(seed, (views.n, views.height, views.width))
    t = _dev(g)
    plan = ops.Plan()
    ops.project_forward(*t, views, cutoff, plan)
    grads = ops.project_backward(*t, views, torch.from_numpy(G).cuda(), plan, cutoff)
    torch.cuda.synchronize()
    ref = oracle.project_grad(g, oviews, G, cutoff, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), ref)
    print("grad detail", det, flush=True)
    return el, nr


@pytest.mark.parametrize("cutoff", [3.0, math.inf])
def test_cone_gradients(ops, cutoff):
    g = scenes.random_scene(41, 250, lo=0.03, hi=0.12, box=0.5)
    th = [0.4, 1.7, 3.3, 5.0]
    views = ops.Views.cone(th, 13.64, 20.46, 64, 52, 0.045)
    ov = [oracle.cone_view(t, 13.64, 20.46, 64, 52, 0.045) for t in th]
    el, nr = _check_proj_grad(ops, g, views, ov, 3, cutoff)
    _report(f"cone grads cutoff={cutoff}", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_cone_gradients_thin_and_wide(ops):
    """Projected widths from a third of a pixel to several pixels: the
    backward walks of the wide ones step exp2 by multiplication, those of the
    thin ones (form beyond the multiplicative range over an 8x8 sub-tile)
    evaluate exp2 per pixel; both against the oracle."""
    g = scenes.random_scene(43, 300, lo=0.006, hi=0.1, box=0.5)
    th = [0.2, 2.1, 4.4]
    views = ops.Views.cone(th, 13.64, 20.46, 80, 72, 0.045)
    ov = [oracle.cone_view(t, 13.64, 20.46, 80, 72, 0.045) for t in th]
    params = [torch.from_numpy(np.asarray(a, np.float64)) for a in (g.mean, g.scale, g.quat, g.density)]
    with torch.no_grad():
        pr = oracle.project_gaussians(*params, ov[0])
    A = torch.stack([torch.stack([pr["A"][0], pr["A"][1]], -1), torch.stack([pr["A"][1], pr["A"][2]], -1)], -2)
    sig_px = 1.0 / torch.sqrt(torch.linalg.eigvalsh(A)[:, 1]).numpy() / 0.045
    assert (sig_px < 0.6).mean() > 0.1 and (sig_px > 1.5).mean() > 0.3
    el, nr = _check_proj_grad(ops, g, views, ov, 6)
    _report("cone grads thin and wide", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_signed_densities(ops):
    """Densities of both signs (the projection is linear in them), thin and
    wide Gaussians: the forward's multiplicative columns carry the sign on
    exp2, its per-pixel path multiplies by it; image and gradients against
    the oracle."""
    g = scenes.random_scene(45, 300, lo=0.006, hi=0.1, box=0.5, rho=(-1.0, 1.0))
    assert (g.density < 0).mean() > 0.3 and (g.density > 0).mean() > 0.3
    th = [0.7, 2.6]
    views = ops.Views.cone(th, 13.64, 20.46, 80, 72, 0.045)
    ov = [oracle.cone_view(t, 13.64, 20.46, 80, 72, 0.045) for t in th]
    img, _ = _proj_fwd(ops, g, views)
    v, _ = parity.forward_violation(img, oracle.project(g, ov))
    _report("signed densities forward", v)
    assert v <= 1.0
    el, nr = _check_proj_grad(ops, g, views, ov, 8)
    _report("signed densities grads", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_small_density_scale(ops):
    """Densities near 1e-20 (log2|rho_hat| about -66): the forward's
    multiplicative columns then need the form below about 34 over a
    sub-tile, and their cutoff is compared on e = |rho_hat| exp2(...) itself;
    image and gradients against the oracle, whose tolerances scale with the
    image."""
    g = scenes.random_scene(46, 300, lo=0.006, hi=0.1, box=0.5, rho=(-2e-20, 2e-20))
    th = [1.1, 3.9]
    views = ops.Views.cone(th, 13.64, 20.46, 80, 72, 0.045)
    ov = [oracle.cone_view(t, 13.64, 20.46, 80, 72, 0.045) for t in th]
    img, _ = _proj_fwd(ops, g, views)
    v, _ = parity.forward_violation(img, oracle.project(g, ov))
    _report("small densities forward", v)
    assert v <= 1.0
    el, nr = _check_proj_grad(ops, g, views, ov, 9)
    _report("small densities grads", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_parallel_gradients(ops):
    from scipy.spatial.transform import Rotation
    g = scenes.random_scene(42, 200, lo=0.03, hi=0.12, box=0.6)
    rots = Rotation.random(2, random_state=9).as_matrix()
    views = ops.Views.parallel(rots, 50, 47, 0.03)
    ov = [oracle.parallel_view(r, 50, 47, 0.03) for r in rots]
    el, nr = _check_proj_grad(ops, g, views, ov, 4)
    _report("parallel grads", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_voxel_gradients(ops):
    g = scenes.random_scene(43, 200, lo=0.03, hi=0.1, box=0.45)
    grid = Grid(37, 29, 33, (-0.5, -0.48, -0.52), (1 / 36, 1 / 28, 1 / 32))
    H = upstream(5, (grid.nz, grid.ny, grid.nx))
    t = _dev(g)
    plan = ops.Plan()
    ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, plan)
    grads = ops.voxelize_backward(*t, ops.grid_from(grid), torch.from_numpy(H).cuda(), plan, 3.0)
    torch.cuda.synchronize()
    ref = oracle.voxelize_grad(g, grid, H, 3.0, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), ref)
    print(det)
    _report("voxel grads", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_voxel_gradients_thin_and_wide(ops):
    """Widths from a tenth of a voxel to two voxels: the backward walks of the
    wide Gaussians step exp2 by multiplication, those whose form leaves the
    multiplicative range over a 4^3 sub-cube evaluate exp2 per voxel."""
    g = scenes.random_scene(44, 260, lo=0.004, hi=0.06, box=0.45)
    grid = Grid(37, 29, 33, (-0.5, -0.48, -0.52), (1 / 36, 1 / 28, 1 / 32))
    smin = np.asarray(g.scale, np.float64).min(axis=1) / (1 / 28)
    assert (smin < 0.3).mean() > 0.1 and (smin > 0.6).mean() > 0.3
    H = upstream(7, (grid.nz, grid.ny, grid.nx))
    t = _dev(g)
    plan = ops.Plan()
    ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, plan)
    grads = ops.voxelize_backward(*t, ops.grid_from(grid), torch.from_numpy(H).cuda(), plan, 3.0)
    torch.cuda.synchronize()
    ref = oracle.voxelize_grad(g, grid, H, 3.0, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), ref)
    print(det)
    _report("voxel grads thin and wide", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_backward_without_forward_and_accumulate(ops):
    """Backward on a fresh plan recomputes the binning; accumulate adds."""
    g = scenes.random_scene(44, 150)
    views = ops.Views.cone([0.9], 13.64, 20.46, 40, 40, 0.05)
    G = torch.from_numpy(upstream(6, (1, 40, 40))).cuda()
    t = _dev(g)
    a = ops.project_backward(*t, views, G, ops.Plan(), 3.0)
    plan = ops.Plan()
    ops.project_forward(*t, views, 3.0, plan)
    b = ops.project_backward(*t, views, G, plan, 3.0)
    c = tuple(x.clone() for x in b)
    ops.project_backward(*t, views, G, plan, 3.0, grads=c, accumulate=True)
    torch.cuda.synchronize()
    # the backward is deterministic (each entry's moments depend on that entry
    # alone and every sum runs in a fixed order), and y + y = 2y is exact
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y)
        assert torch.equal(z, 2 * y)


def test_binning_and_results_are_bitwise_reproducible(ops):
    """The tile lists are a stable counting sort (Gaussian order within every
    tile), so repeated calls, on the same plan or on new plans, give bitwise
    equal images, volumes and gradients.  Several binning chunks, two views,
    ragged detector and grid."""
    g = scenes.random_scene(45, 9000, lo=0.01, hi=0.09, box=0.9)
    views = ops.Views.cone([0.4, 2.2], 13.64, 20.46, 75, 53, 0.04)
    grid = Grid(35, 29, 41, (-0.9, -0.8, -0.95), (0.05, 0.055, 0.045))
    G = torch.from_numpy(upstream(8, (2, 53, 75))).cuda()
    H = torch.from_numpy(upstream(9, (grid.nz, grid.ny, grid.nx))).cuda()
    t = _dev(g)
    runs = []
    keep = ops.Plan(), ops.Plan()
    for k in range(3):
        pp, pv = keep if k < 2 else (ops.Plan(), ops.Plan())
        img = ops.project_forward(*t, views, 3.0, pp)
        gp = ops.project_backward(*t, views, G, pp, 3.0)
        vol = ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, pv)
        gv = ops.voxelize_backward(*t, ops.grid_from(grid), H, pv, 3.0)
        torch.cuda.synchronize()
        runs.append((img.clone(), vol.clone()) + tuple(x.clone() for x in gp + gv))
    for later in runs[1:]:
        for x, y in zip(runs[0], later):
            assert torch.equal(x, y)


@pytest.mark.parametrize("width,height,pitch", [(1040, 800, 0.017), (2048, 1100, 0.0015)])
def test_wide_detector_binning(ops, width, height, pitch):
    """Detectors of more than 2048 tiles, where the scatter places entries
    with 32-bit tile masks: 1040 x 800 (3250 tiles, one window of tiles in
    LDS) and 2048 x 1100 (8832 tiles, three windows of 4096; the scene covers
    all three).  Two calls give bitwise equal images and gradients, and both
    match the oracle."""
    g = scenes.random_scene(46, 2000, lo=0.005, hi=0.05, box=0.9)
    views = ops.Views.cone([0.7], 13.64, 20.46, width, height, pitch)
    ov = [oracle.cone_view(0.7, 13.64, 20.46, width, height, pitch)]
    G = upstream(12, (1, height, width))
    t = _dev(g)
    runs = []
    for _ in range(2):
        plan = ops.Plan()
        img = ops.project_forward(*t, views, 3.0, plan)
        gp = ops.project_backward(*t, views, torch.from_numpy(G).cuda(), plan, 3.0)
        torch.cuda.synchronize()
        runs.append((img.clone(),) + tuple(x.clone() for x in gp))
    for x, y in zip(runs[0], runs[1]):
        assert torch.equal(x, y)
    v, _ = parity.forward_violation(runs[0][0].cpu().numpy(), oracle.project(g, ov))
    _report(f"wide detector {width}x{height} forward", v)
    assert v <= 1.0
    el, nr, det = parity.grad_violation(_np(runs[0][1:]), oracle.project_grad(g, ov, G, 3.0, with_scale=True))
    _report(f"wide detector {width}x{height} gradients", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


# ----------------------------------------------------------------- losses --

def test_image_loss(ops):
    x = workloads.random_images(11, 3, 70, 45)
    y = workloads.random_images(12, 3, 70, 45)
    loss, grad = ops.image_loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), ops.Plan(), 0.25)
    torch.cuda.synchronize()
    total, l1, s, gref = oracle.image_loss(x, y, 0.25)
    lv = loss.cpu().numpy()
    assert abs(lv[1] - l1) <= 1e-5 * l1 + 1e-7
    assert abs(lv[2] - s) <= 2e-5
    assert abs(lv[0] - total) <= 1e-5 * abs(total) + 1e-6
    gg = grad.cpu().numpy()
    ratio = parity.loss_grad_violation(gg, gref, oracle.image_loss_grad_scale(x, y, 0.25))
    _report("image loss gradient (per pixel)", ratio)
    assert ratio <= 1.0
    assert np.abs(gg - gref).max() <= 1e-3 * np.abs(gref).max()


def test_image_loss_marching_kernel(ops):
    """A stack just large enough for the marching loss kernel (512 images of
    65 rows by 55 columns: two 64-row segments by two 54-column strips each,
    2048 wavefronts, every last segment and strip one pixel wide) against the
    oracle; on this stack and on a small one (the 32 x 32 tile kernel) the
    loss without the gradient is bitwise the loss with it."""
    x = workloads.random_images(13, 512, 65, 55)
    y = workloads.random_images(14, 512, 65, 55)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    loss, grad = ops.image_loss(xt, yt, ops.Plan(), 0.25)
    loss0, _ = ops.image_loss(xt, yt, ops.Plan(), 0.25, grad=False)
    torch.cuda.synchronize()
    assert torch.equal(loss, loss0)
    total, l1, s_, gref = oracle.image_loss(x, y, 0.25)
    lv = loss.cpu().numpy()
    assert abs(lv[1] - l1) <= 1e-5 * l1 + 1e-7
    assert abs(lv[2] - s_) <= 2e-5
    assert abs(lv[0] - total) <= 1e-5 * abs(total) + 1e-6
    ratio = parity.loss_grad_violation(grad.cpu().numpy(), gref, oracle.image_loss_grad_scale(x, y, 0.25))
    _report("image loss gradient, marching kernel (per pixel)", ratio)
    assert ratio <= 1.0
    xs, ys = xt[:3, :45, :70].contiguous(), yt[:3, :45, :70].contiguous()
    a, _ = ops.image_loss(xs, ys, ops.Plan(), 0.25)
    b, _ = ops.image_loss(xs, ys, ops.Plan(), 0.25, grad=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_tv_loss(ops):
    rng = np.random.default_rng(3)
    v = rng.standard_normal((13, 17, 19)).astype(np.float32)
    vt = torch.from_numpy(v).cuda()
    loss, grad = ops.tv_loss(vt, ops.Plan(), weight=0.05)
    torch.cuda.synchronize()
    t, gref = oracle.tv_loss(v, 0.05)
    assert abs(float(loss.cpu()[0]) - t) <= 1e-5 * t
    np.testing.assert_allclose(grad.cpu().numpy(), gref, rtol=1e-5, atol=1e-9)


# ------------------------------------------------------------ edge cases --

def test_empty_and_degenerate_inputs(ops):
    views = ops.Views.cone([0.5], 13.64, 20.46, 20, 20, 0.1)
    z = [torch.zeros((0, k), device="cuda") for k in (3, 3, 4)] + [torch.zeros(0, device="cuda")]
    img = ops.project_forward(*z, views, 3.0, ops.Plan())
    assert torch.count_nonzero(img) == 0
    # NaN centre, zero scale, zero quaternion, a centre behind the source: all skipped
    bad = scenes.gaussians([[np.nan, 0, 0], [0, 0, 0], [0.1, 0, 0], [30.0, 0.0, 0.0], [0.05, 0.02, 0.0]],
                           [[0.1] * 3, [0.0, 0.1, 0.1], [0.1] * 3, [0.1] * 3, [0.1] * 3],
                           [[1, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]],
                           [1, 1, 1, 1, 1])
    ov = [oracle.cone_view(0.0, 13.64, 20.46, 20, 20, 0.1)]
    views0 = ops.Views.cone([0.0], 13.64, 20.46, 20, 20, 0.1)
    img, plan = _proj_fwd(ops, bad, views0)
    assert np.all(np.isfinite(img))
    v, _ = parity.forward_violation(img, oracle.project(bad, ov))
    assert v <= 1.0
    assert plan.status()["skipped"] == 4
    G = torch.ones((1, 20, 20), device="cuda")
    grads = ops.project_backward(*_dev(bad), views0, G, plan, 3.0)
    torch.cuda.synchronize()
    for t in grads:
        t = t.cpu().numpy()
        assert np.all(np.isfinite(t))
        assert np.all(t[:4] == 0)


def test_tiny_detector_and_grid(ops):
    g = scenes.random_scene(51, 30, lo=0.1, hi=0.3, box=0.2)
    views = ops.Views.cone([1.0], 13.64, 20.46, 1, 1, 0.3)
    img, _ = _proj_fwd(ops, g, views)
    ref = oracle.project(g, [oracle.cone_view(1.0, 13.64, 20.46, 1, 1, 0.3)])
    assert parity.forward_violation(img, ref)[0] <= 1.0
    grid = Grid(1, 1, 1, (-0.05, -0.05, -0.05), (0.1, 0.1, 0.1))
    vol = ops.voxelize_forward(*_dev(g), ops.grid_from(grid), 3.0, ops.Plan())
    torch.cuda.synchronize()
    assert parity.forward_violation(vol.cpu().numpy(), oracle.voxelize(g, grid))[0] <= 1.0


def test_invalid_arguments_raise(ops):
    from paper_2405_20693_amd._native import GsError
    g = scenes.random_scene(52, 10)
    t = _dev(g)
    views = ops.Views.cone([0.0], 13.64, 20.46, 16, 16, 0.1)
    with pytest.raises(GsError, match="GS_EINVAL"):
        ops.project_forward(*t, views, 0.0, ops.Plan())
    bad = ops.Views.cone([0.0], 13.64, 20.46, 16, 16, 0.1)
    bad.arr[0].src_det = 5.0
    with pytest.raises(GsError, match="GS_EINVAL"):
        ops.project_forward(*t, bad, 3.0, ops.Plan())


# -------------------------------------------------------------- autograd --

def test_autograd_functions_match_direct_calls(ops):
    g = scenes.random_scene(61, 120)
    views = ops.Views.cone([0.3, 2.0], 13.64, 20.46, 32, 32, 0.06)
    t = [x.clone().requires_grad_(True) for x in _dev(g)]
    img = ops.project(*t, views, 3.0)
    G = torch.from_numpy(upstream(7, tuple(img.shape))).cuda()
    (img * G).sum().backward()
    plan = ops.Plan()
    d = _dev(g)
    ops.project_forward(*d, views, 3.0, plan)
    ref = ops.project_backward(*d, views, G, plan, 3.0)
    for a, b in zip(t, ref):
        assert torch.allclose(a.grad, b, rtol=1e-5, atol=1e-6 * float(b.abs().max()))


# ----------------------------------------------------- full-size configs --

def test_c2_full_size(ops):
    """C2 (50k Gaussians, 75 cone views of 256^2) in one launch: every pixel
    of the 75 views and the gradients of all 50k Gaussians for an upstream
    gradient on every pixel, per element and norm-wise."""
    wl = workloads.c2_cone()
    views = ops.Views.from_scan(wl.scan)
    t = _dev(wl.gaussians)
    plan = ops.Plan()
    img = ops.project_forward(*t, views, 3.0, plan)
    G = upstream(1, (75, 256, 256))
    grads = ops.project_backward(*t, views, torch.from_numpy(G).cuda(), plan, 3.0)
    torch.cuda.synchronize()
    ov = oracle.views_from_scan(wl.scan)
    ref = oracle.project(wl.gaussians, ov)
    v, _ = parity.forward_violation(img.cpu().numpy(), ref)
    _report("c2 forward (75 views)", v)
    assert v <= 1.0
    rg = oracle.project_grad(wl.gaussians, ov, G, 3.0, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), rg)
    print(det)
    _report("c2 grads (50k Gaussians)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_c2_tv_voxelization_full_size(ops):
    """C2's TV term at full size: the 50k Gaussians voxelized on the 128^3
    grid over [-1, 1]^3 in one launch, the TV loss and its gradient, and the
    voxelizer backward of that gradient, all checked whole against the
    oracle (every voxel; every Gaussian's gradient, per element and
    norm-wise)."""
    wl = workloads.c2_cone()
    grid = wl.grid
    assert (grid.nx, grid.ny, grid.nz) == (128, 128, 128)
    t = _dev(wl.gaussians)
    plan = ops.Plan()
    vol = ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, plan)
    lt, gvol = ops.tv_loss(vol, ops.Plan(), weight=0.05)
    grads = ops.voxelize_backward(*t, ops.grid_from(grid), gvol, plan, 3.0)
    torch.cuda.synchronize()
    v = vol.cpu().numpy()
    vv, _ = parity.forward_violation(v, oracle.voxelize(wl.gaussians, grid))
    _report("c2 128^3 volume (every voxel)", vv)
    assert vv <= 1.0
    tv_ref, gref = oracle.tv_loss(v, 0.05)
    assert abs(float(lt.cpu()[0]) - tv_ref) <= 1e-5 * tv_ref
    H = gvol.cpu().numpy()
    np.testing.assert_allclose(H, gref, rtol=1e-5, atol=1e-12)
    rg = oracle.voxelize_grad(wl.gaussians, grid, H, 3.0, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), rg)
    print(det)
    _report("c2 128^3 TV gradients (50k Gaussians)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_training_iteration_matches_oracle_composition(ops):
    """The fused iteration's gradients equal the oracle's projection gradient
    of the image-loss gradient plus the voxelization gradient of the weighted
    TV gradient (small scene)."""
    from paper_2405_20693_amd.iteration import TrainingIteration
    g = scenes.random_scene(71, 300, lo=0.03, hi=0.1, box=0.5)
    th = [0.1, 2.2, 4.1]
    views = ops.Views.cone(th, 13.64, 20.46, 48, 40, 0.05)
    ov = [oracle.cone_view(t, 13.64, 20.46, 48, 40, 0.05) for t in th]
    meas = workloads.random_images(8, 3, 40, 48) * np.float32(0.5)
    grid = Grid(24, 24, 24, (-0.4, -0.4, -0.4), (1 / 30, 1 / 30, 1 / 30))
    it = TrainingIteration(*_dev(g), views, torch.from_numpy(meas).cuda(), (24, 24, 24))
    grads = it.step(ops.grid_from(grid))
    torch.cuda.synchronize()
    img = oracle.project(g, ov)["image"]
    total, l1, s, Gimg = oracle.image_loss(img.astype(np.float32), meas, 0.25)
    vol = oracle.voxelize(g, grid)["volume"]
    tv, Hvol = oracle.tv_loss(vol.astype(np.float32), 0.05)
    lv = it.loss_img.cpu().numpy()
    assert abs(lv[0] - total) <= 1e-4 * total
    assert abs(float(it.loss_tv.cpu()[0]) - tv) <= 1e-4 * tv
    # each stage on its own inputs: the loss gradients of the GPU's own image
    # and volume, then the operators' backward of the GPU's own loss gradients
    gimg = it.grad_image.cpu().numpy()
    rimg = it.image.cpu().numpy()
    _, _, _, Gown = oracle.image_loss(rimg, meas, 0.25)
    ratio = parity.loss_grad_violation(gimg, Gown, oracle.image_loss_grad_scale(rimg, meas, 0.25))
    _report("iteration image-loss gradient", ratio)
    assert ratio <= 1.0
    _, Hown = oracle.tv_loss(it.volume.cpu().numpy(), 0.05)
    hvol = it.grad_volume.cpu().numpy()
    np.testing.assert_allclose(hvol, Hown, rtol=1e-5, atol=1e-12)
    rp = oracle.project_grad(g, ov, gimg, 3.0, with_scale=True)
    rv = oracle.voxelize_grad(g, grid, hvol, 3.0, with_scale=True)
    comb = {k: rp[k] + rv[k] for k in KEYS}
    comb["S_abs"] = {k: rp["S_abs"][k] + rv["S_abs"][k] for k in KEYS}
    comb["amb"] = {k: rp["amb"][k] + rv["amb"][k] for k in KEYS}
    el, nr, det = parity.grad_violation(_np(grads), comb)
    print(det)
    _report("iteration gradients (projection + voxelizer)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def _grad_subset(gpu, ref, sel):
    sub_gpu = {k: gpu[k][sel] for k in KEYS}
    sub_ref = {k: ref[k][sel] for k in KEYS}
    sub_ref["S_abs"] = {k: ref["S_abs"][k][sel] for k in KEYS}
    sub_ref["amb"] = {k: ref["amb"][k][sel] for k in KEYS}
    return parity.grad_violation(sub_gpu, sub_ref)


def test_c3_training_workload_full_size(ops):
    """The measured workload at full size, in the launch configuration the
    benchmark times (200k Gaussians, 75 views of 512^2 in one launch, a 64^3
    TV block of the 256^3 grid): projection forward on three sampled views,
    projection gradients of 32 sampled Gaussians with an upstream gradient on
    those views, the full TV block forward and backward, and the loss terms on
    the full 75-image stack."""
    from paper_2405_20693_amd.iteration import TrainingIteration
    wl = workloads.c3_iteration()
    views = ops.Views.from_scan(wl.scan)
    t = _dev(wl.gaussians)
    plan = ops.Plan()
    img = ops.project_forward(*t, views, 3.0, plan)
    sel_v = [5, 40, 71]
    G = np.zeros((75, 512, 512), np.float32)
    G[sel_v] = upstream(2, (3, 512, 512))
    grads = ops.project_backward(*t, views, torch.from_numpy(G).cuda(), plan, 3.0)
    torch.cuda.synchronize()
    ov = oracle.views_from_scan(wl.scan)
    sub = [ov[i] for i in sel_v]
    ref = oracle.project(wl.gaussians, sub)
    v, _ = parity.forward_violation(img.cpu().numpy()[sel_v], ref)
    _report("c3 forward (3 views)", v)
    assert v <= 1.0
    sel_g = np.random.default_rng(1).choice(wl.gaussians.n, 32, replace=False)
    rg = oracle.project_grad(wl.gaussians, sub, G[sel_v], 3.0, select=sel_g, with_scale=True)
    el, nr, det = _grad_subset(_np(grads), rg, sel_g)
    print(det)
    _report("c3 grads (32 Gaussians)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0
    # TV block of the iteration: voxelization forward + backward in full
    grid = workloads.tv_block_grid(wl, 0)
    vplan = ops.Plan()
    vol = ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, vplan)
    H = upstream(3, (64, 64, 64))
    vg = ops.voxelize_backward(*t, ops.grid_from(grid), torch.from_numpy(H).cuda(), vplan, 3.0)
    torch.cuda.synchronize()
    vref = oracle.voxelize(wl.gaussians, grid)
    vv, _ = parity.forward_violation(vol.cpu().numpy(), vref)
    _report("c3 TV block voxelize", vv)
    assert vv <= 1.0
    touched = np.unique(np.random.default_rng(2).choice(wl.gaussians.n, 20000, replace=False))
    vr = oracle.voxelize_grad(wl.gaussians, grid, H, 3.0, select=touched, with_scale=True)
    nz_sel = touched[np.abs(vr["density"][touched]) > 0][:64]
    if nz_sel.size:
        el, nr, det = _grad_subset(_np(vg), vr, nz_sel)
        _report(f"c3 TV block grads ({nz_sel.size} Gaussians)", max(el, nr))
        assert el <= 1.0 and nr <= 1.0
    # loss terms on the full stack (rendered image vs measured projections)
    meas = workloads.measured_projections(wl)
    rimg = img.cpu().numpy()
    loss, lg = ops.image_loss(img, torch.from_numpy(meas).cuda(), ops.Plan(), 0.25)
    torch.cuda.synchronize()
    total, l1, s, gref = oracle.image_loss(rimg, meas, 0.25)
    lv = loss.cpu().numpy()
    assert abs(lv[1] - l1) <= 1e-5 * l1 and abs(lv[2] - s) <= 2e-5
    gg = lg.cpu().numpy()
    ratio = parity.loss_grad_violation(gg, gref, oracle.image_loss_grad_scale(rimg, meas, 0.25))
    _report("c3 image loss gradient (75 x 512^2, per pixel)", ratio)
    assert ratio <= 1.0
    assert np.abs(gg - gref).max() <= 1e-3 * np.abs(gref).max()


def test_c3_whole_view_stack(ops):
    """The measured workload's projection on its whole view stack, in the
    launch configuration the benchmark times (200k Gaussians, 75 views of
    512^2 in one launch): every pixel of all 75 images, and the gradients of
    all 200k Gaussians for an upstream gradient on every pixel, against the
    oracle at the stated tolerances (per element and norm-wise)."""
    wl = workloads.c3_iteration()
    views = ops.Views.from_scan(wl.scan)
    t = _dev(wl.gaussians)
    plan = ops.Plan()
    img = ops.project_forward(*t, views, 3.0, plan)
    G = upstream(6, (75, 512, 512))
    grads = ops.project_backward(*t, views, torch.from_numpy(G).cuda(), plan, 3.0)
    torch.cuda.synchronize()
    ov = oracle.views_from_scan(wl.scan)
    print("c3 whole stack: oracle forward ...", flush=True)
    ref = oracle.project(wl.gaussians, ov)
    v, _ = parity.forward_violation(img.cpu().numpy(), ref)
    _report("c3 forward (75 views, every pixel)", v)
    assert v <= 1.0
    print("c3 whole stack: oracle gradients ...", flush=True)
    rg = oracle.project_grad(wl.gaussians, ov, G, 3.0, with_scale=True)
    el, nr, det = parity.grad_violation(_np(grads), rg)
    print(det, flush=True)
    _report("c3 grads (200k Gaussians)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0


def test_c5_large_sampled(ops):
    """1M anisotropic Gaussians, 150 cone views of 1024^2 in one launch and a
    512^3 voxelization: every pixel of 15 views spread over the orbit, the
    gradients of all 1M Gaussians for an upstream gradient on those views
    (per element and norm-wise), and the volume on two sampled 24^3
    sub-blocks."""
    wl = workloads.c5_large()
    views = ops.Views.from_scan(wl.scan)
    t = _dev(wl.gaussians)
    plan = ops.Plan()
    img = ops.project_forward(*t, views, 3.0, plan)
    sel_v = list(range(3, 150, 10))
    G = torch.zeros((150, 1024, 1024), device="cuda")
    Gs = upstream(4, (len(sel_v), 1024, 1024))
    G[sel_v] = torch.from_numpy(Gs).cuda()
    grads = ops.project_backward(*t, views, G, plan, 3.0)
    torch.cuda.synchronize()
    st = plan.status()
    print("c5 tile entries", st["tile_entries"], flush=True)
    img_s = img[sel_v].cpu().numpy()
    del img, G
    ov = oracle.views_from_scan(wl.scan)
    sub = [ov[i] for i in sel_v]
    print("c5: oracle forward ...", flush=True)
    ref = oracle.project(wl.gaussians, sub)
    v, _ = parity.forward_violation(img_s, ref)
    _report(f"c5 forward ({len(sel_v)} views)", v)
    assert v <= 1.0
    print("c5: oracle gradients ...", flush=True)
    rg = oracle.project_grad(wl.gaussians, sub, Gs, 3.0, with_scale=True)
    gg = _np(grads)
    el, nr, det = parity.grad_violation(gg, rg)
    print(det)
    for k in KEYS:  # the worst elements, for the record
        g64 = np.asarray(gg[k], np.float64)
        ratio = np.abs(g64 - rg[k]) / (1e-3 * rg["S_abs"][k] + rg["amb"][k] + 1e-30)
        flat = np.argsort(ratio.ravel())[-3:][::-1]
        for f in flat:
            gi = np.unravel_index(f, ratio.shape)[0]
            print(f"c5 worst {k}{np.unravel_index(f, ratio.shape)}: ratio {ratio.ravel()[f]:.3g} gpu "
                  f"{g64.ravel()[f]:.6g} oracle {rg[k].ravel()[f]:.6g} S_abs "
                  f"{rg['S_abs'][k].ravel()[f]:.3g} amb {rg['amb'][k].ravel()[f]:.3g}; scale "
                  f"{wl.gaussians.scale[gi]} quat {wl.gaussians.quat[gi]} mean {wl.gaussians.mean[gi]}",
                  flush=True)
    _report("c5 grads (1M Gaussians)", max(el, nr))
    assert el <= 1.0 and nr <= 1.0
    vol = ops.voxelize_forward(*t, ops.grid_from(wl.grid), 3.0, ops.Plan())
    torch.cuda.synchronize()
    for (i0, j0, k0) in [(240, 250, 244), (100, 300, 380)]:
        sg = workloads.sub_grid(wl.grid, i0, j0, k0, 24, 24, 24)
        vr = oracle.voxelize(wl.gaussians, sg)
        part = vol[k0:k0 + 24, j0:j0 + 24, i0:i0 + 24].cpu().numpy()
        vv, _ = parity.forward_violation(part, vr)
        _report(f"c5 volume block {(i0, j0, k0)}", vv)
        assert vv <= 1.0
