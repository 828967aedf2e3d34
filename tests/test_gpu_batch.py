"""GPU parity of the batched form (hca_cluster_batch) against the CPU oracle:
every data set of a batch must get exactly the labels the oracle gives it
alone (and that hca_cluster gives it alone)."""
from __future__ import annotations

import hashlib
import json
from pathlib import Path

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import Workload, make_batch, quantise, make_blobs

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


def run_batch(ctx, jobs):
    import torch
    flat = np.concatenate([j.points.reshape(-1) for j in jobs]) if jobs else np.zeros(0, np.int32)
    pts = torch.from_numpy(np.ascontiguousarray(flat, np.int32)).cuda()
    labels = ctx.cluster_batch(pts, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                               [j.min_pts for j in jobs]).cpu().numpy()
    out, at = [], 0
    for j in jobs:
        out.append(labels[at:at + j.n])
        at += j.n
    return out


def test_batch_small_jobs(ctx):
    jobs = make_batch(seed=11, count=40, n_range=(50, 5000), dims=(1, 2, 3, 4))
    print(f"[case] batch of {len(jobs)} small jobs", flush=True)
    got = run_batch(ctx, jobs)
    for j, g in zip(jobs, got):
        want = oracle.dbscan(j.points, j.eps, j.min_pts)
        assert np.array_equal(g, want), j.name


def test_batch_equals_single_calls(ctx):
    import torch
    jobs = make_batch(seed=12, count=12, n_range=(2000, 30000))
    print("[case] batch vs single calls", flush=True)
    got = run_batch(ctx, jobs)
    for j, g in zip(jobs, got):
        alone = ctx.cluster(torch.from_numpy(j.points).cuda(), j.eps, j.min_pts).cpu().numpy()
        assert np.array_equal(g, alone), j.name
        assert np.array_equal(g, oracle.dbscan(j.points, j.eps, j.min_pts)), j.name


def test_batch_edge_cases(ctx):
    rng = np.random.default_rng(21)
    jobs = []

    def job(pts, eps, mp):
        pts = np.ascontiguousarray(pts, np.int32)
        return Workload(f"edge{len(jobs)}", pts, eps, mp, 0, {})

    jobs.append(job(np.zeros((0, 2)), 5.0, 3))                           # empty
    jobs.append(job(np.full((50, 2), 7), 0.5, 50))                       # identical, minPts = n
    jobs.append(job(np.full((50, 2), 7), 0.5, 51))                       # identical, all noise
    jobs.append(job(np.array([[3, 4]]), 1.0, 1))                         # single point
    jobs.append(job(np.zeros((0, 3)), 5.0, 3))                           # empty
    line = np.stack([np.arange(3000) * 3, np.zeros(3000)], 1)
    jobs.append(job(line[rng.permutation(3000)], 3.0, 3))                # chain exactly eps apart
    jobs.append(job(quantise(make_blobs(rng, 4000, 4, 5, 0.03, 0.1), 12) - 50_000, 0.05 * 2 ** 12, 5))
    jobs.append(job(quantise(make_blobs(rng, 3000, 3, 4, 0.02, 0.1), 20), 0.04 * 2 ** 20, 4))  # wide
    jobs.append(job(rng.integers(-3000, 3000, size=(2000, 1)), 2.0, 2))  # 1-D
    jobs.append(job(rng.integers(0, 100, size=(2000, 2)), 1e5, 7))       # eps beyond the diameter
    print(f"[case] batch edge cases ({len(jobs)} jobs)", flush=True)
    got = run_batch(ctx, jobs)
    for j, g in zip(jobs, got):
        assert np.array_equal(g, oracle.dbscan(j.points, j.eps, j.min_pts)), j.name


def test_batch_errors(ctx):
    import torch
    from paper_1912_00323_amd import hca
    pts = torch.zeros(5 * 10, dtype=torch.int32, device="cuda")
    with pytest.raises(hca.HcaError) as e:
        ctx.cluster_batch(pts, [10], [5], [1.0], [2])                   # d > 4
    assert e.value.status == hca.HCA_E_INVAL
    with pytest.raises(hca.HcaError) as e:
        ctx.cluster_batch(pts[:20], [10], [2], [float("nan")], [2])
    assert e.value.status == hca.HCA_E_INVAL
    big = torch.tensor([0, 0, 1 << 30, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(hca.HcaError) as e:
        ctx.cluster_batch(big, [2], [2], [1.0], [1])
    assert e.value.status == hca.HCA_E_RANGE
    with pytest.raises(ValueError):
        ctx.cluster_batch(pts, [10, 1], [2], [1.0], [2])
    # the context stays usable
    ok = torch.zeros(8, dtype=torch.int32, device="cuda")
    assert ctx.cluster_batch(ok, [4], [2], [1.0], [1]).cpu().tolist() == [0, 0, 0, 0]


def test_batch_full_workload(ctx):
    exp = json.loads((GOLDEN / "batch_expected.json").read_text())
    jobs = make_batch(seed=exp["seed"], count=exp["count"])
    print(f"[case] full batched workload: {len(jobs)} jobs, {sum(j.n for j in jobs)} points", flush=True)
    for j, e in zip(jobs, exp["jobs"]):
        assert digest(j.points.reshape(-1)) == e["points_sha256"], "input generator drifted"
    got = run_batch(ctx, jobs)
    for j, g, e in zip(jobs, got, exp["jobs"]):
        assert digest(g) == e["labels_sha256"], j.name
    again = run_batch(ctx, jobs)
    assert all(np.array_equal(a, b) for a, b in zip(got, again))


def test_cluster_sets_own_arrays(ctx):
    import torch
    import ctypes
    jobs = make_batch(seed=13, count=10, n_range=(100, 8000), dims=(2, 3, 4))
    pts = [torch.from_numpy(j.points).cuda() for j in jobs]
    outs = [torch.full((j.n,), -7, dtype=torch.int32, device="cuda") for j in jobs]
    lib = ctx._lib
    P = (ctypes.c_void_p * len(jobs))(*[p.data_ptr() for p in pts])
    L = (ctypes.c_void_p * len(jobs))(*[o.data_ptr() for o in outs])
    rows = np.array([j.n for j in jobs], np.int64)
    dims = np.array([j.d for j in jobs], np.int32)
    eps = np.array([j.eps for j in jobs], np.float64)
    mps = np.array([j.min_pts for j in jobs], np.int32)
    st = lib.hca_cluster_sets(ctx._ctx, P, L, len(jobs), rows.ctypes.data_as(ctypes.c_void_p),
                              dims.ctypes.data_as(ctypes.c_void_p), eps.ctypes.data_as(ctypes.c_void_p),
                              mps.ctypes.data_as(ctypes.c_void_p))
    assert st == 0
    for j, o in zip(jobs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.dbscan(j.points, j.eps, j.min_pts)), j.name


def test_server_results_alone_and_in_the_mix():
    """Requests submitted together (batched, overlapping on two workers, a
    5-D request among them) get exactly what each gets alone."""
    import torch
    from paper_1912_00323_amd import hca
    jobs = make_batch(seed=14, count=30, n_range=(500, 40000), dims=(2, 3, 5))
    srv = hca.Server(0, workers=2, budget_bytes=1 << 30, max_batch=8)
    pts = [torch.from_numpy(j.points).cuda() for j in jobs]
    outs = [torch.full((j.n,), -7, dtype=torch.int32, device="cuda") for j in jobs]
    print(f"[case] server mix of {len(jobs)} requests", flush=True)
    for k, (j, p, o) in enumerate(zip(jobs, pts, outs)):
        srv.submit(p, j.eps, j.min_pts, o, tag=k)
    srv.drain()
    done = {}
    while len(done) < len(jobs):
        got = srv.poll()
        assert got, "server drained without reporting every request"
        for t, st, _ in got:
            done[t] = st
    srv.close()
    assert all(st == 0 for st in done.values())
    c = hca.Context(0)
    for j, p, o in zip(jobs, pts, outs):
        alone = c.cluster(p, j.eps, j.min_pts).cpu().numpy()
        assert np.array_equal(o.cpu().numpy(), alone), j.name
        assert np.array_equal(alone, oracle.dbscan(j.points, j.eps, j.min_pts)), j.name
    c.close()


def test_served_full_range(ctx):
    """Requests of the served workload across its whole range (up to 2M points
    and 5 axes), submitted together with smaller ones to the request loop:
    each result matches the oracle's stored digest, in the mix and alone."""
    import torch
    from paper_1912_00323_amd import hca
    from paper_1912_00323_amd.datagen import make_served
    exp = json.loads((GOLDEN / "served_expected.json").read_text())
    reqs = make_served(seed=exp["seed"], count=exp["count"])
    picked = {e["index"]: e for e in exp["requests"]}
    for k, e in picked.items():
        assert digest(reqs[k].points.reshape(-1)) == e["points_sha256"], "input generator drifted"
    mix = sorted(set(picked) | set(range(0, 64, 3)))
    pts = {k: torch.from_numpy(reqs[k].points).cuda() for k in mix}
    outs = {k: torch.full((reqs[k].n,), -7, dtype=torch.int32, device="cuda") for k in mix}
    print(f"[case] served mix of {len(mix)} requests, {sum(reqs[k].n for k in mix)} points", flush=True)
    srv = hca.Server(0, workers=2, budget_bytes=64 << 30, max_batch=16, batch_ms=4.0)
    try:
        for k in mix:
            srv.submit(pts[k], reqs[k].eps, reqs[k].min_pts, outs[k], tag=k)
        srv.drain()
        done = {t: st for t, st, _ in srv.poll(1 << 12)}
    finally:
        srv.close()
    assert sorted(done) == mix and all(st == 0 for st in done.values())
    for k, e in picked.items():
        assert digest(outs[k].cpu().numpy()) == e["labels_sha256"], ("mix", e["name"])
        alone = ctx.cluster(pts[k], reqs[k].eps, reqs[k].min_pts).cpu().numpy()
        assert digest(alone) == e["labels_sha256"], ("alone", e["name"])
    for k in mix:
        if k not in picked:
            alone = ctx.cluster(pts[k], reqs[k].eps, reqs[k].min_pts)
            assert torch.equal(outs[k], alone), reqs[k].name
