"""Serving loop (include/gs_serve.h): results are the same alone and in a
mixed, batched run; admission refuses work above the memory budget."""
import numpy as np
import pytest
import torch

import oracle
from oracle import parity
from tests import scenes
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


def test_results_same_alone_and_in_the_mix(ops):
    models = [scenes.random_scene(81, 1500, lo=0.02, hi=0.1), scenes.random_scene(82, 900, lo=0.03, hi=0.12)]
    dm = [_dev(m) for m in models]
    srv = ops.Server(n_workers=3, batching=True, max_batch_views=64, hbm_budget_bytes=1 << 30)
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
