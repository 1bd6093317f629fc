"""GPU tests of reserved plans (gs_plan_reserve / gs_plan_check): the same
results as allocating plans without host synchronization, overflow reported
and harmless, calls larger than the reservation refused, and projection
forward/backward captured in a HIP graph and replayed."""
import numpy as np
import pytest
import torch

from tests import scenes
import workloads
from workloads import Grid, upstream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20693_amd import ops as _ops
    return _ops


def _dev(g):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.mean, g.scale, g.quat, g.density)]


def _problem(ops, m=4000, seed=51):
    g = scenes.random_scene(seed, m, lo=0.02, hi=0.08, box=0.8)
    th = [0.3, 1.4, 2.9, 4.1]
    views = ops.Views.cone(th, 13.64, 20.46, 72, 60, 0.035)
    grid = Grid(40, 36, 30, (-0.9, -0.8, -0.7), (0.045, 0.045, 0.045))
    return g, views, grid


def _run(ops, t, views, grid, G, H, plan_p, plan_v, plan_l):
    img = ops.project_forward(*t, views, 3.0, plan_p)
    gp = ops.project_backward(*t, views, G, plan_p, 3.0)
    vol = ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, plan_v)
    gv = ops.voxelize_backward(*t, ops.grid_from(grid), H, plan_v, 3.0)
    loss, gimg = ops.image_loss(img, G.abs(), plan_l)
    return img, gp, vol, gv, loss, gimg


def test_reserved_plan_matches_allocating_plan(ops):
    g, views, grid = _problem(ops)
    t = _dev(g)
    G = torch.from_numpy(upstream(3, (views.n, views.height, views.width))).cuda()
    H = torch.from_numpy(upstream(4, (grid.nz, grid.ny, grid.nx))).cuda()
    ref = _run(ops, t, views, grid, G, H, ops.Plan(), ops.Plan(), ops.Plan())
    torch.cuda.synchronize()
    pp, pv, pl = ops.Plan(), ops.Plan(), ops.Plan()
    pp.reserve(g.n, views.n, views.width, views.height, max_proj_entries=400_000)
    pv.reserve(g.n, grid=(grid.nx, grid.ny, grid.nz), max_vox_entries=400_000)
    pl.reserve(0, views.n, views.width, views.height)
    for _ in range(3):  # queued back to back: no host synchronization in between
        got = _run(ops, t, views, grid, G, H, pp, pv, pl)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):  # the binning and every sum are deterministic
        for x, y in zip(a if isinstance(a, tuple) else (a,), b if isinstance(b, tuple) else (b,)):
            assert torch.equal(x, y)
    pe, _ = pp.check()
    _, ve = pv.check()
    plan = ops.Plan()
    ops.project_forward(*t, views, 3.0, plan)
    assert pe == plan.status()["tile_entries"]
    plan = ops.Plan()
    ops.voxelize_forward(*t, ops.grid_from(grid), 3.0, plan)
    assert ve == plan.status()["tile_entries"]
    assert pp.status()["tile_entries"] == pe  # a reserved plan reports what its last call needed


def test_reservation_overflow_is_reported(ops):
    """A call that needs more tile entries than reserved: its backward writes
    no gradient; once the device has recorded the overflow, the next operator
    call and gs_plan_status return GS_EOVERFLOW before any launch; gs_plan_check
    reports it with the entries needed and clears it, after which a call on a
    plan reserved for that need gives the allocating plan's results."""
    from paper_2405_20693_amd import _native as N
    g, views, grid = _problem(ops)
    t = _dev(g)
    plan = ops.Plan()
    ref = ops.project_forward(*t, views, 3.0, plan)
    G = torch.ones_like(ref)
    ref_g = ops.project_backward(*t, views, G, plan, 3.0)
    entries = plan.status()["tile_entries"]
    assert entries > 20_000
    small = ops.Plan()
    small.reserve(g.n, views.n, views.width, views.height, max_proj_entries=10_000)
    sentinel = tuple(torch.full_like(x, 7.0) for x in t)
    ops.project_forward(*t, views, 3.0, small)
    try:  # queued behind the overflowing forward, or refused if the host saw it first
        ops.project_backward(*t, views, G, small, 3.0, grads=sentinel)
    except N.GsError as e:
        assert "GS_EOVERFLOW" in str(e)
    torch.cuda.synchronize()
    for x in sentinel:
        assert (x == 7.0).all()  # no gradient written from incomplete slots
    with pytest.raises(N.GsError) as e:
        ops.project_forward(*t, views, 3.0, small)
    assert "GS_EOVERFLOW" in str(e.value)
    with pytest.raises(N.GsError) as e:
        small.status()
    assert "GS_EOVERFLOW" in str(e.value)
    need, _, over = small.check(raise_overflow=False)
    assert over and need == entries
    assert small.check() == (0, 0)  # cleared
    small.reserve(g.n, views.n, views.width, views.height, max_proj_entries=need)
    img = ops.project_forward(*t, views, 3.0, small)
    gr = ops.project_backward(*t, views, G, small, 3.0)
    torch.cuda.synchronize()
    assert small.check() == (need, 0)
    assert torch.equal(img, ref)
    for a, b in zip(gr, ref_g):
        assert torch.equal(a, b)


def test_tile_entries_beyond_32_bits_are_refused(ops):
    """A projection whose binning needs 2^32 - 1 or more tile entries (no
    cutoff, so every one of 70,000 Gaussians covers all 1,024 tiles of each of
    64 views of 512^2: 4.59e9 entries) is refused with GS_EOVERFLOW before its
    scatter runs: the entry totals are summed in 64 bits with saturated block
    sums, so they cannot wrap to a small count.  The same plan then serves an
    ordinary call exactly as a fresh plan does."""
    from paper_2405_20693_amd import _native as N
    g = scenes.random_scene(61, 70_000, lo=0.02, hi=0.08, box=0.8)
    t = _dev(g)
    views = ops.Views.cone(np.linspace(0.0, 2.0 * np.pi, 64, endpoint=False), 13.64, 20.46,
                           512, 512, 0.035)
    plan = ops.Plan()
    with pytest.raises(N.GsError) as e:
        ops.project_forward(*t, views, float("inf"), plan)
    assert "GS_EOVERFLOW" in str(e.value)
    img = ops.project_forward(*t, views, 3.0, plan)
    ref = ops.project_forward(*t, views, 3.0, ops.Plan())
    torch.cuda.synchronize()
    assert torch.equal(img, ref)


def test_reserved_plan_refuses_larger_calls(ops):
    g, views, grid = _problem(ops, m=3000)
    t = _dev(g)
    plan = ops.Plan()
    plan.reserve(1000, views.n, views.width, views.height, max_proj_entries=100_000)
    from paper_2405_20693_amd import _native as N
    with pytest.raises(N.GsError) as e:
        ops.project_forward(*t, views, 3.0, plan)
    assert "GS_EINVAL" in str(e.value)
    plan = ops.Plan()
    plan.reserve(g.n, 2, views.width, views.height, max_proj_entries=100_000)
    with pytest.raises(N.GsError):
        ops.project_forward(*t, views, 3.0, plan)  # four views, two reserved


def test_graph_capture_of_projection(ops):
    """Forward + backward on a reserved plan captured once in a HIP graph and
    replayed after changing the Gaussians in place; every replay matches the
    eager result for the same Gaussians."""
    g, views, grid = _problem(ops, m=3000, seed=52)
    t = _dev(g)
    G = torch.from_numpy(upstream(5, (views.n, views.height, views.width))).cuda()
    plan = ops.Plan()
    plan.reserve(g.n, views.n, views.width, views.height, max_proj_entries=300_000)
    img = torch.empty((views.n, views.height, views.width), device="cuda")
    grads = tuple(torch.empty_like(x) for x in t)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream (views uploaded)
        ops.project_forward(*t, views, 3.0, plan, out=img)
        ops.project_backward(*t, views, G, plan, 3.0, grads=grads)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ops.project_forward(*t, views, 3.0, plan, out=img)
        ops.project_backward(*t, views, G, plan, 3.0, grads=grads)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    for k in range(4):
        with torch.no_grad():
            t[0].add_(torch.from_numpy(rng.normal(0, 0.01, g.mean.shape).astype(np.float32)).cuda())
            t[3].mul_(1.0 + 0.1 * k)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        eager_plan = ops.Plan()
        ref_img = ops.project_forward(*t, views, 3.0, eager_plan)
        ref_g = ops.project_backward(*t, views, G, eager_plan, 3.0)
        torch.cuda.synchronize()
        assert torch.equal(img, ref_img)
        for a, b in zip(grads, ref_g):
            assert torch.equal(a, b)
    assert plan.check()[0] > 0
