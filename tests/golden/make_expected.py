"""Write tests/golden/full_size_expected.json (the fixed workloads),
tests/golden/batch_expected.json (the 256 jobs of the batched workload) and
tests/golden/served_expected.json (requests of the served workload up to 2M
points and 5 axes): the oracle's labels, stored as SHA-256 digests of the
little-endian int32 label arrays plus summary counts.  Calls only the CPU
oracle (its definition part; for the served requests its grid part, which
the pins tie to the definition) and the seeded input generator.

    python tests/golden/make_expected.py [--threads N] [--only fixed|batch|served]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_1912_00323_amd.datagen import make_batch, make_config, make_served  # noqa: E402

OUT = Path(__file__).resolve().parent / "full_size_expected.json"
OUT_BATCH = Path(__file__).resolve().parent / "batch_expected.json"
OUT_SERVED = Path(__file__).resolve().parent / "served_expected.json"
# requests of make_served(seed=5, count=64) spanning the served workload's
# range: 24k and 20k points (2-D, 5-D), 496k (5-D), 1.2M (2-D), 1.9M (3-D),
# 2.0M (5-D)
SERVED_PICK = (4, 57, 24, 31, 59, 9)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).astype("<i4").tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", choices=["fixed", "batch", "served"], default=None)
    args = ap.parse_args()
    if args.only in (None, "served"):
        served(args.threads)
    if args.only == "served":
        return
    if args.only != "fixed":
        batch(args.threads)
    if args.only == "batch":
        return
    out = {"note": "labels of the CPU oracle (DBSCAN definition) on the seeded workloads; "
                   "points_sha256 guards against generator drift",
           "workloads": {}}
    for k in (1, 2, 3):
        w = make_config(k)
        t0 = time.time()
        labels, counts, _ = oracle.dbscan(w.points, w.eps, w.min_pts, threads=args.threads,
                                          details=True)
        dt = time.time() - t0
        core = counts >= w.min_pts
        out["workloads"][w.name] = {
            "config": k, "seed": k, "n": w.n, "d": w.d, "eps": w.eps, "min_pts": w.min_pts,
            "eps2": oracle.exact_eps2(w.eps),
            "points_sha256": digest(w.points.reshape(-1)),
            "labels_sha256": digest(labels),
            "core_sha256": digest(core.astype(np.int32)),
            "n_clusters": int(labels.max() + 1) if len(labels) else 0,
            "n_noise": int((labels < 0).sum()),
            "n_core": int(core.sum()),
            "oracle_seconds": round(dt, 2),
        }
        print(w.name, out["workloads"][w.name], flush=True)
    OUT.write_text(json.dumps(out, indent=1) + "\n")


def served(threads: int):
    reqs = make_served(seed=5, count=64)
    out = {"note": "labels of the CPU oracle (grid part, exact) on requests of the served workload "
                   "(make_served(seed=5, count=64)); points_sha256 guards against generator drift",
           "seed": 5, "count": 64, "requests": []}
    for k in SERVED_PICK:
        w = reqs[k]
        t0 = time.time()
        labels = oracle.hca_grid(w.points, w.eps, w.min_pts, threads=threads)
        out["requests"].append({"index": k, "name": w.name, "n": w.n, "d": w.d, "eps": w.eps,
                                "min_pts": w.min_pts, "points_sha256": digest(w.points.reshape(-1)),
                                "labels_sha256": digest(labels),
                                "n_clusters": int(labels.max() + 1) if len(labels) else 0,
                                "n_noise": int((labels < 0).sum()),
                                "oracle_seconds": round(time.time() - t0, 1)})
        print(out["requests"][-1], flush=True)
    OUT_SERVED.write_text(json.dumps(out, indent=1) + "\n")


def batch(threads: int):
    jobs = make_batch(seed=4, count=256)
    out = {"note": "labels of the CPU oracle (DBSCAN definition) on each job of the batched workload "
                   "(make_batch(seed=4, count=256)); points_sha256 guards against generator drift",
           "seed": 4, "count": len(jobs), "jobs": []}
    t_all = time.time()
    for w in jobs:
        labels = oracle.dbscan(w.points, w.eps, w.min_pts, threads=threads)
        out["jobs"].append({"name": w.name, "n": w.n, "d": w.d, "eps": w.eps, "min_pts": w.min_pts,
                            "points_sha256": digest(w.points.reshape(-1)),
                            "labels_sha256": digest(labels),
                            "n_clusters": int(labels.max() + 1) if len(labels) else 0,
                            "n_noise": int((labels < 0).sum())})
    print(f"batch: {len(jobs)} jobs, {sum(j['n'] for j in out['jobs'])} points, "
          f"{time.time() - t_all:.1f} s", flush=True)
    OUT_BATCH.write_text(json.dumps(out, indent=1) + "\n")


if __name__ == "__main__":
    main()
