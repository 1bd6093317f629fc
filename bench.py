#!/usr/bin/env python3
"""Training-iteration throughput of the R^2-Gaussian hot path on one MI355X.

Workload (synthetic, seeded): 200,000 Gaussians on a 12-ellipsoid phantom,
75 cone-beam views of 512x512 rendered in one launch, loss L1 + 0.25 D-SSIM
against measured projections (exact line integrals of the phantom), plus
0.05 TV on a random 64^3 block of a 256^3 voxelization; forward and backward of
both operators and of the losses.  A step is one such iteration; all of it runs
in libgs.so.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit (the scope table's counts): VALU lane-slots per
# in-cutoff term of the render and voxel kernels (an FMA is one slot, exp2 a
# quarter-rate transcendental counted as 4), and compulsory HBM bytes of the
# memory-bound stages.
SLOTS_PER_PAIR = {"fwd": 10, "bwd": 25}
PEAK_SLOTS_PER_S = 256 * 128 * 2.4e9       # CUs x FP32 lanes per clock x clock (157.3 TFLOP/s / 2)
HBM_PEAK_BYTES_PER_S = 8.0e12


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "c3_iteration_hbm_traffic.json")


def measured_traffic():
    """HBM bytes per launch of each kernel from the committed rocprofv3
    counter profile (FETCH_SIZE + WRITE_SIZE, calibrated), or {} if there is
    none or a kernel source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            prof = json.load(f)
        for rel, digest in prof["sources_sha256"].items():
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return {}
        return prof["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return {}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_iteration(wl, measured, k, with_tv):
    """Seconds the FP64 oracle takes for k views of the iteration (projection
    forward, L1 + D-SSIM, projection backward) and, optionally, the TV block
    (voxelize forward, TV, voxelize backward)."""
    import numpy as np
    import oracle
    import workloads
    views = oracle.views_from_scan(wl.scan)[:k]
    t0 = time.perf_counter()
    img = oracle.project(wl.gaussians, views, wl.cutoff)["image"]
    _, _, _, G = oracle.image_loss(img.astype(np.float32), measured[:k], 0.25)
    oracle.project_grad(wl.gaussians, views, G, wl.cutoff)
    t_views = time.perf_counter() - t0
    t_vox = 0.0
    if with_tv:
        grid = workloads.tv_block_grid(wl, 0)
        t1 = time.perf_counter()
        vol = oracle.voxelize(wl.gaussians, grid, wl.cutoff)["volume"]
        _, H = oracle.tv_loss(vol.astype(np.float32), 0.05)
        oracle.voxelize_grad(wl.gaussians, grid, H, wl.cutoff)
        t_vox = time.perf_counter() - t1
    return t_views, t_vox


def cpu_baseline(wl, measured):
    """The FP64 oracle on bounded samples of the same iteration, extrapolated
    to one iteration: on all host threads (all 75 views, the full TV block)
    and on one thread (2 views and the full TV block)."""
    import oracle
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                         os.cpu_count() or 1))
    nv = len(wl.scan.thetas)
    prev = oracle.set_threads(threads)
    t_views, t_vox = _oracle_iteration(wl, measured, nv, True)
    oracle.set_threads(1)
    k1 = 2
    t1_views, t1_vox = _oracle_iteration(wl, measured, k1, True)
    oracle.set_threads(prev[0])
    t_all = t_views + t_vox
    t_one = t1_views * nv / k1 + t1_vox
    return {"value": round(1.0 / t_all, 5), "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{nv} of {nv} views (projection fwd, L1+D-SSIM, projection bwd) + the "
                      f"full 64^3 TV block (voxelize fwd, TV, voxelize bwd) on {threads} threads: "
                      f"{t_all:.1f} s",
            "one_thread": {"value": round(1.0 / t_one, 6), "unit": "iters/s", "cores": 1,
                           "sample": f"{k1} of {nv} views scaled x{nv / k1:.1f} + the full TV "
                                     f"block on 1 thread: measured {t1_views + t1_vox:.1f} s, "
                                     f"{t_one:.0f} s per iteration"},
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}


def stage_model(stages_ms, M, V, H, W, entries, pairs, vox_pairs, block):
    """Per stage: its binding resource and algorithmic work, the floor that
    work sets on the stage's time, and the measured fraction of it."""
    pix = V * H * W
    work = {
        # projection + rectification + tile histograms: read the parameters
        # once, write one 32-B record per (view, Gaussian)
        "proj_bin": ("hbm", 44 * M + 32 * V * M),
        # scatter: read the records, write 8-B entries and 4-B slot offsets
        "proj_scatter": ("hbm", 32 * V * M + 8 * entries + 4 * V * M),
        "render_fwd": ("alu", SLOTS_PER_PAIR["fwd"] * pairs),
        "render_bwd": ("alu", SLOTS_PER_PAIR["bwd"] * pairs),
        # chain rule: parameters once and the 24-B 2D gradient per (Gaussian, view)
        "proj_chain": ("hbm", 44 * M + 24 * V * M + 44 * M),
        "vox_bin": ("hbm", 44 * M + 64 * M),
        "vox_scatter": ("hbm", 64 * M),
        "vox_fwd": ("alu", SLOTS_PER_PAIR["fwd"] * vox_pairs),
        "vox_bwd": ("alu", SLOTS_PER_PAIR["bwd"] * vox_pairs),
        "vox_chain": ("hbm", 44 * M + 44 * M),
        # fused L1 + D-SSIM: read rendered and measured, write the gradient
        "loss_image": ("hbm", 12 * pix),
        "loss_tv": ("hbm", 8 * block ** 3),
    }
    # HBM bytes the ALU-bound stages move at least: their inputs and outputs
    # (records, tile lists, images, per-(view, Gaussian) 2D gradients; voxel
    # records, the block)
    nvox = block ** 3
    io = {"render_fwd": 32 * V * M + 8 * entries + 4 * pix,
          "render_bwd": 32 * V * M + 8 * entries + 4 * pix + 24 * V * M,
          "vox_fwd": 64 * M + 4 * nvox,
          "vox_bwd": 64 * M + 4 * nvox + 40 * M}
    out, t_floor = {}, 0.0
    hbm_bytes = 0
    for k, ms in stages_ms.items():
        if k not in work:
            continue
        bound, w = work[k]
        hbm_bytes += w if bound == "hbm" else io[k]
        peak = PEAK_SLOTS_PER_S if bound == "alu" else HBM_PEAK_BYTES_PER_S
        floor_s = w / peak
        t_floor += floor_s
        out[k] = {"ms": round(ms, 4), "bound": bound,
                  ("slots" if bound == "alu" else "bytes"): int(w),
                  "achieved": round(w / (ms * 1e-3) / (1e12 if bound == "alu" else 1e9), 3),
                  "achieved_unit": "T slots/s" if bound == "alu" else "GB/s",
                  "frac": round(floor_s / (ms * 1e-3), 4)}
    return out, t_floor * 1e3, hbm_bytes


def serving_measure(n_requests, fracs, models=None):
    """Served renders/s and latencies for 16 resident models (20k-500k
    Gaussians) under Poisson arrivals, for the continuous-batching server
    against the plain per-request path (one request per launch, one at a
    time).  Each path is loaded at fractions of its own saturation rate;
    projection and volume-query latencies are reported apart."""
    import numpy as np
    import torch
    import workloads
    from paper_2405_20693_amd import ops
    dev = torch.device("cuda:0")
    if models is None:
        log("generating 16 serving models ...")
        models = [[torch.from_numpy(a).to(dev) for a in (m.mean, m.scale, m.quat, m.density)]
                  for m in workloads.c4_models()]
    servers = {"continuous": ops.Server(n_workers=4, batching=True, max_batch_views=64),
               "continuous_graphs": ops.Server(n_workers=4, batching=True, max_batch_views=64,
                                               graphs=True),
               "per_request": ops.Server(n_workers=1, batching=False)}
    for srv in servers.values():
        for m in models:
            srv.add_model(*m)

    def trace(seed, n, rate):
        reqs = []
        for r in workloads.c4_requests(seed, n, rate):
            d = {"kind": r["kind"], "model": r["model"], "arrival_s": r["arrival_s"]}
            if r["kind"] == "project":
                d["views"] = ops.Views.from_scan(r["scan"])
            else:
                d["grid"] = ops.grid_from(r["grid"])
            reqs.append(d)
        return reqs

    def pct(x, q):
        return round(float(np.percentile(x, q)), 2) if len(x) else None

    def summarize(reqs, res, wall):
        lat_p = np.array([x["latency_s"] for r, x in zip(reqs, res) if r["kind"] == "project"]) * 1e3
        lat_v = np.array([x["latency_s"] for r, x in zip(reqs, res) if r["kind"] == "volume"]) * 1e3
        views = sum(r["views"].n for r in reqs if r["kind"] == "project")
        vols = sum(1 for r in reqs if r["kind"] == "volume")
        return {"renders_per_s": round(views / wall, 1), "volumes_per_s": round(vols / wall, 2),
                "requests_per_s": round(len(reqs) / wall, 2),
                "render_p50_ms": pct(lat_p, 50), "render_p99_ms": pct(lat_p, 99),
                "volume_p50_ms": pct(lat_v, 50), "volume_p99_ms": pct(lat_v, 99),
                "mean_batch": round(float(np.mean([x["batch_size"] for x in res])), 2)}

    warm = trace(7, 48, 0.0)
    for srv in servers.values():
        srv.run(warm, time_scale=0.0)
    torch.cuda.synchronize()
    sat, loads = {}, {}
    for name, srv in servers.items():
        reqs = trace(3, n_requests, 0.0)
        res, wall = srv.run(reqs, time_scale=0.0)
        sat[name] = summarize(reqs, res, wall)
        log(f"saturation {name}: {sat[name]}")
    for frac in fracs:
        row = {}
        for name, srv in servers.items():
            rate = frac * sat[name]["requests_per_s"]
            reqs = trace(11, n_requests, rate)
            res, wall = srv.run(reqs, time_scale=1.0)
            row[name] = dict(summarize(reqs, res, wall), rate_req_per_s=round(rate, 2))
        loads[f"{frac:.1f}x_own_saturation"] = row
        log(f"load {frac:.1f}x: {row}")
    return {"saturation": sat, "loads": loads, "requests_per_point": n_requests,
            "mix": "80% projections (1-64 views, 256^2@1.5mm or 512^2@0.75mm), "
                   "20% 128^3 sub-volumes of a 256^3 grid",
            "continuous": "4 workers (streams), 2 batches in flight each, projections of one model "
                          "size class merged across models up to 64 views per launch",
            "continuous_graphs": "the same batches, each replaying the HIP graph captured for its "
                                 "shape (views padded to a multiple of 8 above 8, detector, size class) "
                                 "with its views and Gaussian sets copied to device memory first",
            "per_request": "1 worker, one request per launch"}


def serving(args):
    import torch
    torch.cuda.set_device(0)
    m = serving_measure(args.serving_requests, (0.1, 0.3, 0.6, 0.9))
    out = {"metric": "served renders/s + p99 (16 resident models 20k-500k, Poisson arrivals)",
           "value": m["saturation"]["continuous"]["renders_per_s"], "unit": "renders/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "c4_serving_16_models_20k-500k"}, **m}
    print(json.dumps(out), flush=True)


def reconstruct(args):
    """Wall-clock of a whole reconstruction with the paper's training settings
    (Sec. 4.1): 30k iterations of one 512^2 cone view each out of 75, 50k
    initial Gaussians (phantom density standing in for the FDK volume, scaled
    by 0.15, nearest-neighbour scales), L1 + 0.25 D-SSIM + 0.05 TV on a random
    32^3 block of the 256^3 grid, Adam with the exponential decay, adaptive
    control from 500 to 15k iterations every 100.  Then the 3D PSNR / SSIM of
    the voxelized model against the phantom on the 256^3 grid."""
    import numpy as np
    import torch
    import workloads
    from paper_2405_20693_amd import ops
    from paper_2405_20693_amd import train as tr
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating phantom, 75 measured projections of 512^2 and the 256^3 ground truth ...")
    wl = workloads.c3_iteration(m=50_000)
    views = ops.Views.from_scan(wl.scan)
    measured = torch.from_numpy(workloads.measured_projections(wl)).to(dev)
    grid = workloads.Grid(256, 256, 256, (-1.0, -1.0, -1.0), (2 / 256,) * 3)
    gt = torch.from_numpy(workloads.phantom_volume(wl, grid)).to(dev)
    g0 = [torch.from_numpy(a).to(dev) for a in (wl.gaussians.mean, wl.gaussians.scale,
                                                 wl.gaussians.quat, wl.gaussians.density)]
    iters = args.iterations
    warm = tr.Trainer(*g0, measured, views, grid, iterations=iters, seed=1)
    warm.run(min(200, iters))
    warm.close()
    trainer = tr.Trainer(*g0, measured, views, grid, iterations=iters, seed=0)
    _, (p0, s0) = trainer.evaluate(grid, gt)
    torch.cuda.synchronize()
    log(f"start: PSNR {p0:.2f} dB, SSIM {s0:.4f}, {wl.gaussians.n} Gaussians")
    chunk = 1000
    done, losses = 0, []
    t0 = time.perf_counter()
    while done < iters:
        k = min(chunk, iters - done)
        losses.append(trainer.run(k))
        done += k
        log(f"  {done} iterations, {time.perf_counter() - t0:.1f} s, {trainer.count()} Gaussians, "
            f"loss {float(losses[-1][-100:].mean()):.5f}")
    wall = time.perf_counter() - t0
    _, (p1, s1) = trainer.evaluate(grid, gt)
    n1 = trainer.count()
    trainer.close()
    out = {"metric": "reconstruction wall-clock (30k iterations, 75 views of 512^2, 50k initial "
                     "Gaussians, D=32)",
           "value": round(wall, 3), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "iterations": iters, "ms_per_iteration": round(1e3 * wall / iters, 4),
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "reconstruct_c3_phantom_75x512_m50k", "views": 75,
                      "detector": [512, 512], "initial_gaussians": wl.gaussians.n,
                      "views_per_iteration": 1, "tv_block": 32, "grid": 256},
           "result": {"psnr_db": round(p1, 3), "ssim": round(s1, 4), "psnr_init_db": round(p0, 3),
                      "ssim_init": round(s0, 4), "final_gaussians": n1,
                      "final_loss": round(float(np.concatenate(losses)[-100:].mean()), 6)},
           "context": "the paper reports 8m21s for 30k iterations at 75 views on an RTX 3090 "
                      "(Table 1); other hardware and data, not a target"}
    print(json.dumps(out), flush=True)


def large(args):
    """The large configuration on one GPU at its real shape: 1,000,000
    anisotropic Gaussians (up to 20:1), 150 cone views of 1024^2 in one
    launch, L1 + D-SSIM against exact line integrals of the phantom, and TV
    over the full 512^3 voxelization, forward and backward."""
    import concurrent.futures
    import dataclasses
    import numpy as np
    import torch
    import workloads
    from paper_2405_20693_amd import ops
    from paper_2405_20693_amd.iteration import TrainingIteration
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating 1M Gaussians and 150 measured projections of 1024^2 ...")
    wl = workloads.c5_large()
    th = wl.scan.thetas
    parts = [th[i::8] for i in range(8)]

    def measure(sub):
        return workloads.measured_projections(
            dataclasses.replace(wl, scan=dataclasses.replace(wl.scan, thetas=sub)))

    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        chunks = list(ex.map(measure, parts))
    measured = np.empty((len(th), wl.scan.height, wl.scan.width), np.float32)
    for i, c in enumerate(chunks):
        measured[i::8] = c
    views = ops.Views.from_scan(wl.scan)
    params = [torch.from_numpy(a).to(dev) for a in (wl.gaussians.mean, wl.gaussians.scale,
                                                     wl.gaussians.quat, wl.gaussians.density)]
    g = wl.grid
    it = TrainingIteration(*params, views, torch.from_numpy(measured).to(dev), (g.nz, g.ny, g.nx))
    del measured
    grid = ops.grid_from(g)
    for p in (it.plan_proj, it.plan_vox, it.plan_loss):
        p.set_timing(True)
    log("warmup ...")
    for _ in range(args.warmup):
        it.step(grid)
    torch.cuda.synchronize()
    for p in (it.plan_proj, it.plan_vox, it.plan_loss):
        p.stage_times()
    log("timed region ...")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        it.step(grid)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = {}
    for p in (it.plan_proj, it.plan_vox, it.plan_loss):
        for k, (ms, n) in p.stage_times().items():
            if n:
                stages[k] = round(ms / n, 3)
    st = it.plan_proj.status()
    ms = 1e3 * (t1 - t0) / args.steps
    out = {"metric": "training iters/sec at 1M Gaussians (150 views of 1024^2, 512^3 TV)",
           "value": round(1e3 / ms, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl.name, "gaussians": wl.gaussians.n, "views": len(th),
                      "detector": [wl.scan.width, wl.scan.height], "tv_grid": g.nx,
                      "anisotropy": "up to 20:1"},
           "roofline": None, "tile_entries": st["tile_entries"], "stage_ms": stages,
           "final_loss": float(it.total_loss().cpu())}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--trials", type=int, default=5,
                    help="timed trials of --steps steps each; the median is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the short serving leg of the default run")
    ap.add_argument("--serving-requests-short", type=int, default=300)
    ap.add_argument("--serving", action="store_true",
                    help="measure the serving loop instead of the training iteration")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--reconstruct", action="store_true",
                    help="time a whole reconstruction (trainer) instead of the iteration")
    ap.add_argument("--iterations", type=int, default=30000)
    ap.add_argument("--workload", choices=("c3", "c5"), default="c3",
                    help="c5: the 1M-Gaussian, 150 x 1024^2 configuration instead of the "
                         "75 x 512^2 iteration")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a reference kernel of known "
                         "traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(views would be sharded across GPUs with one all-reduce of the parameter "
              "gradients; not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_2405_20693_amd import ops
    from paper_2405_20693_amd._native import call, lib
    from paper_2405_20693_amd.iteration import TrainingIteration

    lib()  # fails loudly if the HIP library is not built
    if args.serving:
        serving(args)
        return
    if args.reconstruct:
        reconstruct(args)
        return
    if args.workload == "c5":
        large(args)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, device=dev)          # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
    log("generating workload ...")
    wl = workloads.c3_iteration()
    measured = workloads.measured_projections(wl)
    g = wl.gaussians
    params = [torch.from_numpy(a).to(dev) for a in (g.mean, g.scale, g.quat, g.density)]
    views = ops.Views.from_scan(wl.scan)
    meas_d = torch.from_numpy(measured).to(dev)
    block = wl.extra["block"]
    it = TrainingIteration(*params, views, meas_d, (block, block, block), cutoff=wl.cutoff)
    n_iter = args.warmup + args.trials * args.steps + args.steps
    grids = [ops.grid_from(workloads.tv_block_grid(wl, i)) for i in range(n_iter)]
    log("warmup ...")
    for i in range(args.warmup):
        it.step(grids[i])
    torch.cuda.synchronize()
    # timed trials: K steps each between events on the stream the library
    # launches on (torch's current stream), no per-stage events; the median
    # trial is reported
    log(f"timed region: {args.trials} trials of {args.steps} steps ...")
    stream = torch.cuda.current_stream()
    trial_ms = []
    nxt = args.warmup
    for _ in range(args.trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(args.steps):
            it.step(grids[nxt + i])
        e1.record(stream)
        torch.cuda.synchronize()
        nxt += args.steps
        trial_ms.append(e0.elapsed_time(e1))
    ms_total = float(np.median(trial_ms))
    ms_per_step = ms_total / args.steps
    loss = float(it.total_loss().cpu())
    # per-stage launch times: one more pass with HIP events around each stage
    # on the plans' stream (outside the timed trials)
    for p in (it.plan_proj, it.plan_vox, it.plan_loss):
        p.stage_times()
        p.set_timing(True)
    stage_blocks = list(range(nxt, nxt + args.steps))
    for i in stage_blocks:
        it.step(grids[i])
    torch.cuda.synchronize()
    stages = {}
    for p in (it.plan_proj, it.plan_vox, it.plan_loss):
        for k, (ms, n) in p.stage_times().items():
            stages[k] = (stages.get(k, (0.0, 0))[0] + ms, stages.get(k, (0.0, 0))[1] + n)
        p.set_timing(False)
    avg = {k: ms / n for k, (ms, n) in stages.items()}
    log("stage ms/launch: " + ", ".join(f"{k}={v:.3f}" for k, v in sorted(avg.items(), key=lambda x: -x[1])))
    entries = it.plan_proj.status()["tile_entries"]

    # the work units: exact in-cutoff term counts from the oracle (stored)
    gold = os.path.join(ROOT, "tests", "golden", "c3_pairs.json")
    pairs, vox_pairs = None, None
    if os.path.exists(gold):
        with open(gold) as f:
            gd = json.load(f)
        if gd.get("workload") == wl.name:
            pairs = gd["proj_pairs"]
            tvp = gd.get("tv_block_pairs", [])
            have = [tvp[i] for i in stage_blocks if i < len(tvp)]
            vox_pairs = float(np.mean(have)) if have else (float(np.mean(tvp)) if tvp else 0.0)
    roofline, stage_frac, floor = None, None, None
    probe = None
    try:
        fma, ex2 = ctypes.c_double(), ctypes.c_double()
        call("gs_probe_alu", ctypes.byref(fma), ctypes.byref(ex2), ctypes.c_void_p(stream.cuda_stream))
        probe = {"fma_per_s": round(fma.value / 1e12, 2), "exp2_per_s": round(ex2.value / 1e12, 2),
                 "unit": "T/s", "kernel": "independent v_fmac_f32 / v_exp_f32 chains, 8 waves per SIMD"}
        log(f"ALU probe: {probe}")
    except Exception as e:  # the probe is context, the line stands without it
        log(f"ALU probe failed: {e}")
    if pairs is not None:
        stage_frac, t_floor_ms, hbm_bytes = stage_model(avg, g.n, views.n, views.height,
                                                        views.width, entries, pairs, vox_pairs,
                                                        block)
        floor = {"t_floor_ms": round(t_floor_ms, 4), "t_measured_ms": round(ms_per_step, 4),
                 "frac": round(t_floor_ms / ms_per_step, 4),
                 "rule": "sum over stages of max(algorithmic bytes / 8 TB/s, VALU slots / peak)",
                 "hbm": {"bytes": int(hbm_bytes),
                         "achieved_gbs": round(hbm_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                         "frac": round(hbm_bytes / (ms_per_step * 1e-3) / HBM_PEAK_BYTES_PER_S, 4),
                         "rule": "sum over stages of their algorithmic HBM bytes (ALU-bound stages: "
                                 "their inputs and outputs) / (ms_per_step x 8 TB/s)"}}
        dom = "render_bwd"
        traffic = measured_traffic()
        ops_per_launch = pairs * SLOTS_PER_PAIR["bwd"]
        achieved = ops_per_launch / (avg[dom] * 1e-3) / 1e12
        peak = PEAK_SLOTS_PER_S / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                    "peak": round(peak, 2), "unit": "T slots/s", "frac": round(achieved / peak, 4),
                    "traffic": traffic.get(dom), "pairs_per_launch": pairs,
                    "slots_per_pair": SLOTS_PER_PAIR["bwd"], "avg_launch_ms": round(avg[dom], 4),
                    "peak_rule": "256 CUs x 128 FP32 lanes x 2.4 GHz (157.3 TFLOP/s counted as FMAs)"}
        if traffic:
            roofline["traffic_per_kernel"] = traffic

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(wl, measured)

    serving_leg = None
    if not args.no_serving:
        del it, meas_d
        torch.cuda.synchronize()
        serving_leg = serving_measure(args.serving_requests_short, (0.5, 0.9))

    out = {"metric": "training iters/sec (fwd+bwd proj+voxelize) at 200k Gaussians",
           "value": round(1000.0 / ms_per_step, 3), "unit": "iters/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "trials": args.trials,
           "ms_per_step": round(ms_per_step, 4),
           "trial_ms_per_step": [round(t / args.steps, 4) for t in trial_ms],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": wl.name, "gaussians": g.n, "views": views.n,
                      "detector": [views.height, views.width], "tv_block": block,
                      "tv_grid": wl.extra["full"], "cutoff": wl.cutoff, "loss": "L1+0.25 D-SSIM+0.05 TV"},
           "roofline": roofline, "cpu_baseline": cpu, "tile_entries": entries,
           "stages": stage_frac, "iteration_floor": floor, "alu_probe": probe,
           "stage_ms": {k: round(v, 4) for k, v in avg.items()}, "final_loss": loss,
           "serving": serving_leg}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
