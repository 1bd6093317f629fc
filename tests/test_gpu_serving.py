"""Serving loop (include/gs_serve.h): results are the same alone and in a
mixed, batched run; admission refuses work above the memory budget."""
import numpy as np
import pytest
import torch

import oracle
from oracle import parity
from tests import scenes
import workloads
from workloads import Grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20693_amd import ops as _ops
    return _ops


def _dev(g):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.mean, g.scale, g.quat, g.density)]


def _requests(ops, rng, n):
    reqs = []
    for i in range(n):
        model = int(rng.integers(0, 2))
        if i % 4 == 3:
            o = rng.uniform(-0.6, 0.1, 3)
            g = Grid(20, 20, 20, tuple(o), (0.03, 0.03, 0.03))
            reqs.append({"kind": "volume", "model": model, "arrival_s": 0.0, "grid_np": g,
                         "grid": ops.grid_from(g),
                         "out": torch.full((20, 20, 20), float("nan"), device="cuda")})
        else:
            nv = int(rng.integers(1, 5))
            th = rng.uniform(0, 6.28) + np.arange(nv) * 6.28 / nv
            det = 48 if i % 2 else 40
            v = ops.Views.cone(th, 13.64, 20.46, det, det, 0.05)
            reqs.append({"kind": "project", "model": model, "arrival_s": 0.0, "thetas": th,
                         "det": det, "views": v,
                         "out": torch.full((nv, det, det), float("nan"), device="cuda")})
    return reqs


def test_multi_model_projection_matches_single_model_calls(ops):
    """gs_project_fwd_multi: views of three models of different sizes (one of
    them empty) in one launch equal each model's own gs_project_fwd of the
    same views, within the FP32 order of partial sums, and the oracle; a
    view index beyond the models is refused before any launch."""
    models = [scenes.random_scene(86, 2500, lo=0.02, hi=0.1), scenes.random_scene(87, 700, lo=0.03, hi=0.12),
              scenes.random_scene(88, 0)]
    dm = [_dev(m) for m in models]
    th = [0.2, 1.1, 2.5, 3.3, 4.4, 5.9, 0.7]
    vm = [0, 1, 0, 2, 1, 1, 0]
    views = ops.Views.cone(th, 13.64, 20.46, 56, 44, 0.045)
    img = ops.project_forward_multi(dm, vm, views, 3.0)
    torch.cuda.synchronize()
    got = img.cpu().numpy()
    for k in range(3):
        idx = [i for i, m in enumerate(vm) if m == k]
        alone = ops.project_forward(*dm[k], views.subset(idx), 3.0, ops.Plan())
        torch.cuda.synchronize()
        a = alone.cpu().numpy()
        assert np.abs(a - got[idx]).max() <= 1e-5 * max(float(np.abs(a).max()), 1e-30)
        if models[k].n:
            ov = [oracle.cone_view(th[i], 13.64, 20.46, 56, 44, 0.045) for i in idx]
            v, _ = parity.forward_violation(got[idx], oracle.project(models[k], ov))
            print(f"multi-model view set of model {k}: worst tolerance ratio {v:.3g}", flush=True)
            assert v <= 1.0
        else:
            assert not got[idx].any()
    from paper_2405_20693_amd._native import GsError
    with pytest.raises(GsError, match="GS_EINVAL"):
        ops.project_forward_multi(dm, [0, 1, 3, 0, 0, 0, 0], views, 3.0)


@pytest.mark.parametrize("graphs", [False, True])
def test_results_same_alone_and_in_the_mix(ops, graphs):
    """A mixed trace of projections (two detector sizes, two models) and
    volume queries, served with continuous batching (directly launched, or by
    replaying the graph captured for each batch shape): every result equals
    the same request run alone within the FP32 summation-order tolerance, and
    sampled results match the oracle."""
    models = [scenes.random_scene(81, 1500, lo=0.02, hi=0.1), scenes.random_scene(82, 900, lo=0.03, hi=0.12)]
    dm = [_dev(m) for m in models]
    srv = ops.Server(n_workers=3, batching=True, max_batch_views=64, hbm_budget_bytes=1 << 30,
                     graphs=graphs)
    for m in dm:
        srv.add_model(*m)
    reqs = _requests(ops, np.random.default_rng(0), 24)
    res, wall = srv.run(reqs, time_scale=0.0)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in res)
    assert max(r["batch_size"] for r in res) > 1          # merging happened
    for r in reqs:
        m = dm[r["model"]]
        if r["kind"] == "project":
            alone = ops.project_forward(*m, r["views"], 3.0, ops.Plan())
        else:
            alone = ops.voxelize_forward(*m, r["grid"], 3.0, ops.Plan())
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), r["out"].cpu().numpy()
        assert np.all(np.isfinite(b))
        scale = max(float(np.abs(a).max()), 1e-30)
        assert np.abs(a - b).max() <= 1e-5 * scale
    # and the mixed results match the oracle
    r = next(x for x in reqs if x["kind"] == "project")
    ov = [oracle.cone_view(t, 13.64, 20.46, r["det"], r["det"], 0.05) for t in r["thetas"]]
    v, _ = parity.forward_violation(r["out"].cpu().numpy(), oracle.project(models[r["model"]], ov))
    assert v <= 1.0
    r = next(x for x in reqs if x["kind"] == "volume")
    v, _ = parity.forward_violation(r["out"].cpu().numpy(), oracle.voxelize(models[r["model"]], r["grid_np"]))
    assert v <= 1.0


def test_admission_refuses_work_above_the_budget(ops):
    m = _dev(scenes.random_scene(83, 2000))
    srv = ops.Server(n_workers=2, batching=True, max_batch_views=8, hbm_budget_bytes=4 << 20)
    srv.add_model(*m)
    small = {"kind": "project", "model": 0, "arrival_s": 0.0,
             "views": ops.Views.cone([0.1], 13.64, 20.46, 16, 16, 0.1)}
    big = {"kind": "project", "model": 0, "arrival_s": 0.0,
           "views": ops.Views.cone(np.arange(64) * 0.1, 13.64, 20.46, 256, 256, 0.01)}
    from paper_2405_20693_amd._native import GsError
    with pytest.raises(GsError, match="GS_ENOMEM"):
        srv.run([small, big, small], time_scale=0.0)


@pytest.mark.parametrize("graphs", [False, True])
def test_serving_a_c4_sized_model(ops, graphs):
    """A resident model of the serving workload's size class (220k phantom
    Gaussians) next to two small ones: 512^2 and 256^2 cone projections of 1-8
    views and a 128^3 sub-volume of the 256^3 grid, served in one mixed,
    batched run.  Each result equals the same request run alone (within the
    FP32 summation-order tolerance: a batch splits tile lists differently),
    and sampled parts match the oracle: one 512^2 view, and a 24^3 block of
    the sub-volume."""
    big = workloads.phantom_model(1003, 220_000)
    models = [big, scenes.random_scene(84, 1200, lo=0.02, hi=0.1),
              scenes.random_scene(85, 800, lo=0.03, hi=0.12)]
    dm = [_dev(m) for m in models]
    srv = ops.Server(n_workers=3, batching=True, max_batch_views=64, hbm_budget_bytes=8 << 30,
                     graphs=graphs)
    for m in dm:
        srv.add_model(*m)
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(10):
        model = 0 if i % 2 == 0 else int(rng.integers(1, 3))
        if i == 4:
            off = (40, 96, 64)
            h = 2.0 / 256
            g = Grid(128, 128, 128, tuple(-1.0 + o * h for o in off), (h, h, h))
            reqs.append({"kind": "volume", "model": 0, "arrival_s": 0.0, "grid_np": g,
                         "grid": ops.grid_from(g),
                         "out": torch.full((128, 128, 128), float("nan"), device="cuda")})
            continue
        nv = int(rng.integers(1, 9))
        det, pitch = (512, 0.75) if i % 4 == 0 else (256, 1.5)
        scan = workloads.cone_scan(nv, det, det, pitch)
        scan.thetas = rng.uniform(0, 2 * np.pi) + scan.thetas
        reqs.append({"kind": "project", "model": model, "arrival_s": 0.0, "scan": scan,
                     "views": ops.Views.from_scan(scan),
                     "out": torch.full((nv, det, det), float("nan"), device="cuda")})
    res, wall = srv.run(reqs, time_scale=0.0)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in res)
    for r in reqs:
        m = dm[r["model"]]
        if r["kind"] == "project":
            alone = ops.project_forward(*m, r["views"], 3.0, ops.Plan())
        else:
            alone = ops.voxelize_forward(*m, r["grid"], 3.0, ops.Plan())
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), r["out"].cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.abs(a - b).max() <= 1e-5 * max(float(np.abs(a).max()), 1e-30)
    r = next(x for x in reqs if x["kind"] == "project" and x["model"] == 0 and x["scan"].width == 512)
    ov = oracle.views_from_scan(r["scan"])[:1]
    v, _ = parity.forward_violation(r["out"].cpu().numpy()[:1], oracle.project(big, ov))
    print(f"c4-sized model, 512^2 view: worst tolerance ratio {v:.3g}", flush=True)
    assert v <= 1.0
    r = next(x for x in reqs if x["kind"] == "volume")
    sg = workloads.sub_grid(r["grid_np"], 50, 60, 70, 24, 24, 24)
    part = r["out"].cpu().numpy()[70:94, 60:84, 50:74]
    v, _ = parity.forward_violation(part, oracle.voxelize(big, sg))
    print(f"c4-sized model, 24^3 of the 128^3 query: worst tolerance ratio {v:.3g}", flush=True)
    assert v <= 1.0


@pytest.mark.parametrize("graphs", [False, True])
def test_continuous_workspace_stays_within_the_budget(ops, graphs):
    """Continuous batching reserves each worker's workspace from its share of
    the HBM budget when a run starts: the reservation is at most the budget,
    the device memory the run takes is that reservation, and requests of
    several models share launches."""
    models = [scenes.random_scene(90 + k, 600 + 400 * k, lo=0.02, hi=0.1) for k in range(4)]
    dm = [_dev(m) for m in models]
    budget = 96 << 20
    srv = ops.Server(n_workers=2, batching=True, max_batch_views=32, hbm_budget_bytes=budget,
                     graphs=graphs)
    for m in dm:
        srv.add_model(*m)
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(40):
        nv = int(rng.integers(1, 6))
        th = rng.uniform(0, 6.28) + np.arange(nv) * 6.28 / nv
        reqs.append({"kind": "project", "model": int(rng.integers(0, 4)), "arrival_s": 0.0,
                     "views": ops.Views.cone(th, 13.64, 20.46, 64, 64, 0.04),
                     "out": torch.empty((nv, 64, 64), device="cuda")})
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    res, wall = srv.run(reqs, time_scale=0.0)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    used = srv.reserved_bytes()
    print(f"budget {budget}, reserved {used}, device memory taken {free0 - free1}", flush=True)
    assert 0 < used <= budget
    assert free0 - free1 <= budget + (64 << 20)  # allocation granularity
    assert all(r["status"] == 0 for r in res)
    batched = [i for i, r in enumerate(res) if r["batch_size"] > 1]
    assert batched
    assert any(len({reqs[j]["model"] for j in range(len(reqs))
                    if res[j]["start_s"] == res[i]["start_s"]}) > 1 for i in batched)
    for r in reqs[:8]:
        alone = ops.project_forward(*dm[r["model"]], r["views"], 3.0, ops.Plan())
        torch.cuda.synchronize()
        a = alone.cpu().numpy()
        assert np.abs(a - r["out"].cpu().numpy()).max() <= 1e-5 * max(float(np.abs(a).max()), 1e-30)


def test_graph_replays_across_runs_and_batches(ops):
    """Graph replay over two runs of one server (the second trace smaller, with
    the models' densities changed in place in between): the graphs of each run
    are replayed for many batches of different request state, and every result
    equals the same request run alone on the current Gaussians."""
    models = [scenes.random_scene(95, 1300, lo=0.02, hi=0.1), scenes.random_scene(96, 500, lo=0.03, hi=0.12),
              scenes.random_scene(97, 9000, lo=0.01, hi=0.05)]
    dm = [_dev(m) for m in models]
    srv = ops.Server(n_workers=2, batching=True, max_batch_views=16, hbm_budget_bytes=1 << 30,
                     graphs=True)
    for m in dm:
        srv.add_model(*m)
    rng = np.random.default_rng(21)
    for n_req, scale in ((48, 1.0), (20, 1.7)):
        with torch.no_grad():
            for m in dm:
                m[3].mul_(scale)
        reqs = []
        for i in range(n_req):
            nv = int(rng.integers(1, 7))
            th = rng.uniform(0, 6.28) + np.arange(nv) * 6.28 / nv
            det = (32, 48)[i % 2]
            reqs.append({"kind": "project", "model": int(rng.integers(0, 3)), "arrival_s": 0.0,
                         "views": ops.Views.cone(th, 13.64, 20.46, det, det, 0.05),
                         "out": torch.full((nv, det, det), float("nan"), device="cuda")})
        res, wall = srv.run(reqs, time_scale=0.0)
        torch.cuda.synchronize()
        assert all(r["status"] == 0 for r in res)
        assert max(r["batch_size"] for r in res) > 1
        for r in reqs:
            alone = ops.project_forward(*dm[r["model"]], r["views"], 3.0, ops.Plan())
            torch.cuda.synchronize()
            a, b = alone.cpu().numpy(), r["out"].cpu().numpy()
            assert np.all(np.isfinite(b))
            assert np.abs(a - b).max() <= 1e-5 * max(float(np.abs(a).max()), 1e-30)


@pytest.mark.parametrize("graphs", [False, True])
def test_overflowing_batches_are_served_again_alone(ops, graphs):
    """Aligned prolate Gaussians bin into 2.7 times more tile entries seen
    side-on (theta = pi/2: 1308) than end-on (theta = 0: 487; counts of the
    oracle's projection).  The server sizes its reservation from the first
    request of the model, end-on, with a 1.25 margin per view, so batches of
    side-on views overflow their tile lists.  Such a batch is detected from
    the entries the device needed and its requests are served again one by
    one (each fits alone): every request succeeds and equals the same request
    run alone, with direct launches and with graph replay."""
    rng = np.random.default_rng(5)
    m = 400
    needles = scenes.gaussians(rng.uniform(-0.4, 0.4, (m, 3)),
                               np.tile([0.25, 0.012, 0.012], (m, 1)),
                               np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)), rng.uniform(0.5, 1.0, m))
    dm = _dev(needles)
    srv = ops.Server(n_workers=1, batching=True, max_batch_views=16, hbm_budget_bytes=1 << 30,
                     graphs=graphs)
    srv.add_model(*dm)
    reqs = []
    for i in range(33):
        th = [0.0] if i == 0 else [np.pi / 2 + 0.01 * i]
        reqs.append({"kind": "project", "model": 0, "arrival_s": 0.0,
                     "views": ops.Views.cone(th, 13.64, 20.46, 48, 48, 0.05),
                     "out": torch.full((1, 48, 48), float("nan"), device="cuda")})
    res, wall = srv.run(reqs, time_scale=0.0)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in res)
    assert sum(1 for r in res[1:] if r["batch_size"] == 1) > 0  # served again alone
    for r in reqs:
        alone = ops.project_forward(*dm, r["views"], 3.0, ops.Plan())
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), r["out"].cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.abs(a - b).max() <= 1e-5 * max(float(np.abs(a).max()), 1e-30)
