"""GPU parity of batch handles (hca_batch_*): a batch planned, tuned and
captured in a HIP graph on its first run, then replayed on new data of the
same shape; every replay must give each data set exactly the labels the
oracle gives it alone."""
from __future__ import annotations

import hashlib
import json
from pathlib import Path

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import make_batch

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no HIP device visible"
    from paper_1912_00323_amd import hca
    c = hca.Context(0)
    yield c
    c.close()


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype("<i4").tobytes()).hexdigest()


def to_device(sets):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(p, np.int32)).cuda() for p in sets]


def handle(ctx, jobs, tune):
    from paper_1912_00323_amd import hca
    return hca.Batch(ctx, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                     [j.min_pts for j in jobs], tune=tune)


def test_batch_graph_full_workload(ctx, tmp_path, monkeypatch):
    """The 256-set workload: the first run (planned on the host and tuned),
    then graph replays with eager work and syncs between them; every run
    matches the oracle's stored digests."""
    import torch
    monkeypatch.setenv("HCA_TUNE_CACHE", str(tmp_path / "tune.json"))
    exp = json.loads((GOLDEN / "batch_expected.json").read_text())
    jobs = make_batch(seed=exp["seed"], count=exp["count"])
    pts = to_device([j.points for j in jobs])
    outs = [torch.empty(j.n, dtype=torch.int32, device="cuda") for j in jobs]
    b = handle(ctx, jobs, tune=2)
    try:
        for run in range(4):
            print(f"[case] batch handle run {run}", flush=True)
            for o in outs:
                o.fill_(-9)
            b.run(pts, outs)
            for j, o, e in zip(jobs, outs, exp["jobs"]):
                assert digest(o.cpu().numpy()) == e["labels_sha256"], (run, j.name)
            # eager work between replays on the same device
            x = torch.from_numpy(jobs[0].points).cuda()
            ctx.cluster(x, jobs[0].eps, jobs[0].min_pts)
            torch.cuda.synchronize()
        st = b.stats()
        assert st["plans"] == 1 and st["graph_replays"] == 3, st
        assert [g["d"] for g in st["groups"]] == [2, 3, 4]
        assert all(g["tuned"] == 1 and g["tuned_ms"] > 0 for g in st["groups"]), st
        cache = json.loads((tmp_path / "tune.json").read_text())
        assert len(cache["entries"]) == 3
    finally:
        b.close()
    # a new handle of the same shape takes the knobs from the cache
    b2 = handle(ctx, jobs, tune=1)
    try:
        for o in outs:
            o.fill_(-9)
        b2.run(pts, outs)
        for j, o, e in zip(jobs, outs, exp["jobs"]):
            assert digest(o.cpu().numpy()) == e["labels_sha256"], j.name
        assert all(g["tuned"] == 2 for g in b2.stats()["groups"])
    finally:
        b2.close()


def test_batch_graph_new_data(ctx):
    """Replays on other data of the same shape: every data set translated by
    its own vector and its rows permuted (the device finds the new origins),
    then data sets spread too wide for the captured key layout (the run is
    planned and captured again); labels equal the oracle's each time."""
    import torch
    jobs = make_batch(seed=14, count=24, n_range=(500, 12000), dims=(1, 2, 3, 4))
    rng = np.random.default_rng(15)
    b = handle(ctx, jobs, tune=0)
    outs = [torch.empty(j.n, dtype=torch.int32, device="cuda") for j in jobs]
    try:
        variants = [("original", [j.points for j in jobs])]
        moved = []
        for j in jobs:
            shift = rng.integers(-50_000, 50_000, size=j.d).astype(np.int32)
            moved.append(np.ascontiguousarray(j.points[rng.permutation(j.n)] + shift))
        variants.append(("translated and permuted", moved))
        wide = [p.copy() for p in moved]
        for k in range(0, len(jobs), 5):
            wide[k] = np.ascontiguousarray(wide[k] * 8)      # spans 8x: past the captured fields
        variants.append(("spread wider", wide))
        variants.append(("translated again", moved))
        for name, sets in variants:
            print(f"[case] batch handle on {name} data", flush=True)
            b.run(to_device(sets), outs)
            for j, p, o in zip(jobs, sets, outs):
                assert np.array_equal(o.cpu().numpy(), oracle.dbscan(p, j.eps, j.min_pts)), (name, j.name)
        st = b.stats()
        assert st["runs"] == 4 and st["plans"] == 2 and st["graph_replays"] == 2, st
    finally:
        b.close()


def test_batch_graph_errors(ctx):
    import torch
    from paper_1912_00323_amd import hca
    with pytest.raises(hca.HcaError):
        hca.Batch(ctx, [10], [5], [1.0], [3])                    # d > 4
    jobs = make_batch(seed=16, count=3, n_range=(100, 500), dims=(2,))
    b = handle(ctx, jobs, tune=0)
    try:
        big = [np.ascontiguousarray(j.points) for j in jobs]
        big[1] = big[1].astype(np.int64).copy()
        big[1][0, 0] = big[1][1, 0] + (1 << 30)
        big[1] = np.ascontiguousarray(big[1].astype(np.int32))
        with pytest.raises(hca.HcaError) as e:
            b.run(to_device(big), [torch.empty(j.n, dtype=torch.int32, device="cuda") for j in jobs])
        assert e.value.status == hca.HCA_E_RANGE
        outs = [torch.empty(j.n, dtype=torch.int32, device="cuda") for j in jobs]
        b.run(to_device([j.points for j in jobs]), outs)           # usable after the error
        for j, o in zip(jobs, outs):
            assert np.array_equal(o.cpu().numpy(), oracle.dbscan(j.points, j.eps, j.min_pts))
    finally:
        b.close()
