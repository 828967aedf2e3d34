"""The entry point that allocates nothing (hca_cluster_noalloc) against
hca_cluster, through the C ABI: the same labels bit for bit on two calls in a
row (the second smaller, so stale contents of the shared area would show), no
device memory taken by the call, and its limits."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import make_blobs, make_config, quantise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hca_mod():
    import torch
    assert torch.cuda.is_available(), "no HIP device visible"
    from paper_1912_00323_amd import hca
    return hca


def run_both(hca, ctx, pts_np, eps, mp):
    import torch
    pts = torch.from_numpy(np.ascontiguousarray(pts_np, np.int32)).cuda()
    want = ctx.cluster(pts, eps, mp).cpu().numpy()
    out = torch.full((len(pts_np),), -7, dtype=torch.int32, device="cuda")
    got = ctx.cluster_noalloc(pts, eps, mp, out).cpu().numpy()
    return got, want


def test_noalloc_matches_hca_cluster(hca_mod):
    hca = hca_mod
    ctx = hca.Context(0)
    try:
        cases = [("2-D 1M", make_config(2)), ("2-D 10k", make_config(1))]
        for tag, w in cases:                    # large, then smaller: the area keeps the first call's data
            print(f"[case] noalloc {tag} n={w.n}", flush=True)
            got, want = run_both(hca, ctx, w.points, w.eps, w.min_pts)
            assert np.array_equal(got, want), tag
        assert np.array_equal(got, oracle.dbscan(cases[1][1].points, cases[1][1].eps, cases[1][1].min_pts))
        # 8-D (search groups, neighbour lists), then 3-D cubes with lists, then 1-D
        w8 = make_config(3, n=100_000)
        rng = np.random.default_rng(161)
        p3 = quantise(make_blobs(rng, 20000, 3, 6, 0.02, 0.1), 12)
        p1 = quantise(make_blobs(rng, 5000, 1, 4, 0.02, 0.1), 12)
        for tag, pts, eps, mp in (("8-D 100k", w8.points, w8.eps, w8.min_pts),
                                  ("3-D 20k", p3, 0.015 * 2 ** 12, 6), ("1-D 5k", p1, 0.004 * 2 ** 12, 4)):
            print(f"[case] noalloc {tag}", flush=True)
            got, want = run_both(hca, ctx, pts, eps, mp)
            assert np.array_equal(got, want), tag
    finally:
        ctx.close()


def test_noalloc_takes_no_device_memory(hca_mod):
    import torch
    hca = hca_mod
    ctx = hca.Context(0)                        # fresh: its own workspace was never grown
    try:
        w = make_config(2)
        pts = torch.from_numpy(w.points).cuda()
        out = torch.empty(w.n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        ctx.cluster_noalloc(pts, w.eps, w.min_pts, out)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        # hca_cluster would grow a workspace of about 150 MB for this call
        assert free0 - free1 < (16 << 20), (free0, free1)
        ref = hca.Context(0)
        try:
            assert torch.equal(out, ref.cluster(pts, w.eps, w.min_pts))
        finally:
            ref.close()
    finally:
        ctx.close()


def test_noalloc_limits(hca_mod):
    import torch
    hca = hca_mod
    ctx = hca.Context(0)
    try:
        # more points than the area holds: HCA_E_RANGE, labels untouched, the context still usable
        w = make_config(2, n=4_000_000)
        pts = torch.from_numpy(w.points).cuda()
        out = torch.full((w.n,), -5, dtype=torch.int32, device="cuda")
        with pytest.raises(hca.HcaError) as e:
            ctx.cluster_noalloc(pts, w.eps, w.min_pts, out)
        print(f"[range] {e.value}", flush=True)
        assert e.value.status == hca.HCA_E_RANGE
        assert bool((out == -5).all())
        # the 8-D 500k workload: equal to hca_cluster when it fits the area
        w8 = make_config(3)
        p8 = torch.from_numpy(w8.points).cuda()
        o8 = torch.empty(w8.n, dtype=torch.int32, device="cuda")
        try:
            ctx.cluster_noalloc(p8, w8.eps, w8.min_pts, o8)
            assert torch.equal(o8, ctx.cluster(p8, w8.eps, w8.min_pts))
            print("[range] 8-D 500k fits", flush=True)
        except hca.HcaError as err:
            assert err.status == hca.HCA_E_RANGE
            print(f"[range] 8-D 500k: {err}", flush=True)
        # more than 8 axes, and rows off their vector alignment: HCA_E_INVAL
        hi = torch.zeros((100, 9), dtype=torch.int32, device="cuda")
        with pytest.raises(hca.HcaError) as e:
            ctx.cluster_noalloc(hi, 1.0, 1, torch.empty(100, dtype=torch.int32, device="cuda"))
        assert e.value.status == hca.HCA_E_INVAL
        flat = torch.zeros(2 * 100 + 1, dtype=torch.int32, device="cuda")
        off = flat[1:].view(100, 2)
        with pytest.raises(hca.HcaError) as e:
            ctx.cluster_noalloc(off, 1.0, 1, torch.empty(100, dtype=torch.int32, device="cuda"))
        assert e.value.status == hca.HCA_E_INVAL
        small = make_config(1)
        sp = torch.from_numpy(small.points).cuda()
        o2 = torch.empty(small.n, dtype=torch.int32, device="cuda")
        ctx.cluster_noalloc(sp, small.eps, small.min_pts, o2)
        assert np.array_equal(o2.cpu().numpy(), oracle.dbscan(small.points, small.eps, small.min_pts))
        # n = 0 is a no-op
        ctx.cluster_noalloc(torch.zeros((0, 2), dtype=torch.int32, device="cuda"), 1.0, 1,
                            torch.empty(0, dtype=torch.int32, device="cuda"))
    finally:
        ctx.close()
