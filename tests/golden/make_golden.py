"""Writes tests/golden/*.json from the oracle only (FP64 CPU).

c3_pairs.json: the exact number of in-cutoff (view, pixel, Gaussian) terms of
the 200k-Gaussian, 75-view, 512^2 cone-beam training workload (the algorithmic
work unit of the rasterizer's forward and backward), the same count of
(voxel, Gaussian) terms for the 64^3 TV blocks of its first 64 iterations, and
a fingerprint of the generated inputs so that a stale file is detected.

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def fingerprint(wl):
    h = hashlib.sha256()
    g = wl.gaussians
    for a in (g.mean, g.scale, g.quat, g.density):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.asarray(wl.scan.thetas, np.float64).tobytes())
    h.update(repr((wl.scan.src_obj, wl.scan.src_det, wl.scan.width, wl.scan.height,
                   wl.scan.pitch, wl.cutoff)).encode())
    return h.hexdigest()


def main():
    wl = workloads.c3_iteration()
    views = oracle.views_from_scan(wl.scan)
    per_view = []
    for v0 in range(0, len(views), 15):
        r = oracle.project(wl.gaussians, views[v0:v0 + 15], wl.cutoff)
        per_view += [int(x) for x in r["npairs"]]
        print(v0, sum(per_view), flush=True)
    # in-cutoff (voxel, Gaussian) terms of the 64^3 TV blocks of the first
    # 64 iterations (the block offset is drawn with seed = iteration)
    tv_pairs = []
    for i in range(64):
        tv_pairs.append(int(oracle.voxelize(wl.gaussians, workloads.tv_block_grid(wl, i),
                                            wl.cutoff)["npairs"]))
    print("tv blocks", sum(tv_pairs) / len(tv_pairs), flush=True)
    out = {"workload": wl.name, "fingerprint": fingerprint(wl), "cutoff": wl.cutoff,
           "proj_pairs_per_view": per_view, "proj_pairs": int(sum(per_view)),
           "tv_block_pairs": tv_pairs}
    with open(os.path.join(ROOT, "tests", "golden", "c3_pairs.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["proj_pairs"])


if __name__ == "__main__":
    main()
