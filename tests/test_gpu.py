"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Labels must be bit-identical: exact DBSCAN with the fixed border rule and
canonical numbering has exactly one correct labelling.
"""
from __future__ import annotations

import hashlib
import json
import os
from pathlib import Path

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import make_blobs, make_config, make_mixed, quantise

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


def gpu_labels(ctx, pts, eps, min_pts, core=False, stats=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(pts, np.int32)).cuda()
    out = ctx.cluster(t, eps, min_pts, core=core, stats=stats)
    if isinstance(out, tuple):
        return tuple(o.cpu().numpy() if hasattr(o, "cpu") else o for o in out)
    return out.cpu().numpy()


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype("<i4").tobytes()).hexdigest()


def check(ctx, pts, eps, mp, tag=""):
    print(f"[case] {tag} n={len(pts)} d={pts.shape[1]} eps={eps} minPts={mp}", flush=True)
    want = oracle.dbscan(pts, eps, mp)
    got = gpu_labels(ctx, pts, eps, mp)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{tag}: {len(bad)} labels differ, first at {bad[:10]} "
                             f"got {got[bad[:10]]} want {want[bad[:10]]}")


def test_small_workload(ctx):
    w = make_config(1)
    want, counts, _ = oracle.dbscan(w.points, w.eps, w.min_pts, details=True)
    got, core, stats = gpu_labels(ctx, w.points, w.eps, w.min_pts, core=True, stats=True)
    assert np.array_equal(core.astype(bool), counts >= w.min_pts)
    assert np.array_equal(got, want)
    assert stats["n_clusters"] == want.max() + 1
    assert stats["n_noise"] == (want < 0).sum()
    assert stats["n_core_points"] == (counts >= w.min_pts).sum()


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_blobs_every_dimension(ctx, d):
    rng = np.random.default_rng(100 + d)
    for n in (1, 2, 63, 64, 65, 2047, 2049, 5000):
        x = make_blobs(rng, n, d, 4, 0.04, 0.1)
        pts = quantise(x, 10)
        eps = (0.06 + 0.01 * d) * 2 ** 10
        for mp in (1, 4, 9):
            check(ctx, pts, eps, mp, f"blobs d={d}")


@pytest.mark.parametrize("mode", ["cube", "group"])
@pytest.mark.parametrize("reps", ["1", "0"])
def test_search_modes_agree(ctx, mode, reps, monkeypatch):
    monkeypatch.setenv("HCA_SEARCH", mode)
    monkeypatch.setenv("HCA_REPS", reps)
    for d in (2, 3, 4, 5):
        rng = np.random.default_rng(7 * d)
        x = make_blobs(rng, 4000, d, 5, 0.03, 0.1)
        pts = quantise(x, 12)
        check(ctx, pts, 0.05 * 2 ** 12, 5, f"mode={mode} reps={reps} d={d}")


@pytest.mark.parametrize("split", ["0", "1", "2", "5"])
def test_merge_split(ctx, split, monkeypatch):
    """Cube-mode merging in one launch, or the nearest 1, 2 or 5 forward
    neighbours first and the rest after a flattening of the forest: the
    oracle's labels in one to four axes (lane path, stencil and lists)."""
    monkeypatch.setenv("HCA_MERGE_SPLIT", split)
    monkeypatch.setenv("HCA_SEARCH", "cube")
    for d in (1, 2, 3, 4):
        rng = np.random.default_rng(23 * d)
        pts = quantise(make_blobs(rng, 8000, d, 4, 0.03, 0.1), 12)
        for eps, mp in ((0.02 * 2 ** 12, 3), (0.06 * 2 ** 12, 8)):
            check(ctx, pts, eps, mp, f"merge split={split} d={d}")


@pytest.mark.parametrize("lists", ["1", "0"])
def test_cube_lists_on_off(ctx, lists, monkeypatch):
    """Cube mode in three and four axes with neighbour lists built once, or
    the stencil walked in every phase (the tuner's lists knob): the oracle's
    labels either way."""
    monkeypatch.setenv("HCA_SEARCH", "cube")
    monkeypatch.setenv("HCA_CUBE_LISTS", lists)
    for d in (3, 4):
        rng = np.random.default_rng(17 * d)
        pts = quantise(make_blobs(rng, 6000, d, 5, 0.03, 0.1), 12)
        for eps, mp in ((0.03 * 2 ** 12, 4), (0.08 * 2 ** 12, 9)):
            check(ctx, pts, eps, mp, f"cube lists={lists} d={d}")


@pytest.mark.parametrize("slab", ["0", "16", "64"])
def test_group_lists_fallback(ctx, slab, monkeypatch):
    """Group mode with no neighbour lists (stencil walk) and with slabs so small
    that most groups fall back to the stencil while the rest use their lists."""
    monkeypatch.setenv("HCA_SEARCH", "group")
    monkeypatch.setenv("HCA_LIST_SLAB", slab)
    for d in (3, 5, 6):
        rng = np.random.default_rng(70 + d)
        x = make_blobs(rng, 6000, d, 6, 0.04, 0.1)
        pts = quantise(x, 12)
        eps, mp = 0.08 * 2 ** 12, 5
        print(f"[case] lists slab={slab} d={d}", flush=True)
        want = oracle.dbscan(pts, eps, mp)
        got, stats = gpu_labels(ctx, pts, eps, mp, stats=True)
        assert np.array_equal(got, want), f"slab={slab} d={d}"
        if slab == "16" and d >= 5:
            assert stats["list_overflow"] > 0
        if slab == "0":
            assert stats["list_overflow"] == 0


@pytest.mark.parametrize("record", ["0", "1"])
def test_group_recorded_pairs(ctx, record, monkeypatch):
    """With and without the neighbours recorded by core marking (joined
    before the merge tiles of search groups, and deciding the border points
    whose neighbours were all recorded): the same labels."""
    monkeypatch.setenv("HCA_SEARCH", "group")
    monkeypatch.setenv("HCA_RECORD", record)
    for d in (3, 5, 8):
        rng = np.random.default_rng(80 + d)
        x = make_blobs(rng, 8000, d, 6, 0.03, 0.1)
        pts = quantise(x, 12)
        for f, mp in ((0.06, 5), (0.09, 12), (0.12, 1)):
            print(f"[case] recorded pairs={record} d={d} eps={f} minPts={mp}", flush=True)
            want = oracle.dbscan(pts, f * 2 ** 12, mp)
            assert np.array_equal(gpu_labels(ctx, pts, f * 2 ** 12, mp), want), (record, d, f, mp)
    # cubes as search groups: the records decide most border points
    monkeypatch.delenv("HCA_SEARCH")
    for d in (2, 4):
        rng = np.random.default_rng(90 + d)
        pts = quantise(make_blobs(rng, 20000, d, 8, 0.02, 0.15), 12)
        for f, mp in ((0.01, 4), (0.02, 9), (0.03, 12)):
            print(f"[case] recorded neighbours={record} d={d} eps={f} minPts={mp}", flush=True)
            want = oracle.dbscan(pts, f * 2 ** 12, mp)
            assert np.array_equal(gpu_labels(ctx, pts, f * 2 ** 12, mp), want), (record, d, f, mp)


def test_eps_past_int32(ctx):
    """eps^2 between 2^31 and 2^32 over small spans: 32-bit squared distances
    with a threshold past int32 (the data then sits in one cube per axis),
    here and through the batch path (one cluster per data set)."""
    rng = np.random.default_rng(91)
    for d, mode in ((2, None), (3, "group"), (8, None)):
        pts = rng.integers(0, 1000, size=(3000, d)).astype(np.int32)
        pts[:50] += 20000                               # a second, distant clump
        for eps in (50_000.0, 60_000.0, 65_000.0):      # eps^2 = 2.5e9, 3.6e9, 4.2e9
            os.environ.pop("HCA_SEARCH", None)
            if mode:
                os.environ["HCA_SEARCH"] = mode
            try:
                print(f"[case] eps past int32 d={d} eps={eps}", flush=True)
                want = oracle.dbscan(pts, eps, 5)
                assert np.array_equal(gpu_labels(ctx, pts, eps, 5), want), (d, eps)
            finally:
                os.environ.pop("HCA_SEARCH", None)
    # the batch path with the same data sets
    from paper_1912_00323_amd.datagen import Workload
    jobs = [Workload(f"big{d}", rng.integers(0, 1000, size=(2000, d)).astype(np.int32), 60_000.0, 4, 0)
            for d in (1, 2, 3, 4)]
    import torch
    flat = torch.from_numpy(np.concatenate([j.points.ravel() for j in jobs]).astype(np.int32)).cuda()
    got = ctx.cluster_batch(flat, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                            [j.min_pts for j in jobs]).cpu().numpy()
    assert (got == 0).all()


@pytest.mark.parametrize("prefix", ["0", "1"])
def test_group_prefix_ranges(ctx, prefix, monkeypatch):
    """Group-mode lists built by scanning the groups of each first-half
    prefix, or by looking every offset up: the same labels, also when the
    data varies along one half of the axes only (long prefix ranges fall back
    to lookups) or along the other."""
    monkeypatch.setenv("HCA_SEARCH", "group")
    monkeypatch.setenv("HCA_PREFIX", prefix)
    for d in (4, 6, 8):
        rng = np.random.default_rng(120 + d)
        pts = quantise(make_blobs(rng, 8000, d, 6, 0.03, 0.1), 12)
        flat_first = pts.copy()
        flat_first[:, : d // 2] = 7                     # one prefix: every range is the whole set
        flat_second = pts.copy()
        flat_second[:, d // 2:] = 7
        for name, p in (("blobs", pts), ("first half constant", flat_first), ("second half constant", flat_second)):
            for f, mp in ((0.07, 5), (0.1, 1)):
                print(f"[case] prefix={prefix} d={d} {name} eps={f} minPts={mp}", flush=True)
                want = oracle.dbscan(p, f * 2 ** 12, mp)
                assert np.array_equal(gpu_labels(ctx, p, f * 2 ** 12, mp), want), (prefix, d, name, f, mp)
    # cubes as search groups with lists over offsets -R..R (3-D and 4-D)
    monkeypatch.delenv("HCA_SEARCH")
    for d in (3, 4):
        rng = np.random.default_rng(130 + d)
        pts = quantise(make_blobs(rng, 20000, d, 8, 0.02, 0.1), 12)
        for f, mp in ((0.012, 4), (0.02, 9)):
            print(f"[case] prefix={prefix} cubes d={d} eps={f} minPts={mp}", flush=True)
            want = oracle.dbscan(pts, f * 2 ** 12, mp)
            assert np.array_equal(gpu_labels(ctx, pts, f * 2 ** 12, mp), want), (prefix, "cubes", d, f, mp)


def test_prefix_scan_far_groups(ctx, monkeypatch):
    """4-D search groups whose prefix ranges hold groups far beyond the
    stencil (gaps of about 50,000 units along the second half of the axes,
    whose squares pass 2^31) while every tested pair is narrow: the list
    build must drop them (no slab overflow from a wrapped box test) and the
    labels equal the oracle's."""
    monkeypatch.setenv("HCA_SEARCH", "group")
    rng = np.random.default_rng(141)
    parts = []
    for k in range(10):
        # wide along the prefix axes (0, 1), one or two groups along 2 and 3:
        # each prefix range holds a few groups of every clump, under the
        # 64-group limit above which the offsets are looked up instead
        c = rng.integers(0, 300, size=(300, 4))
        c[:, 2:] = rng.integers(0, 30, size=(300, 2))
        c[:, 3] += 50_000 * k
        parts.append(c)
    pts = np.ascontiguousarray(np.concatenate(parts)[rng.permutation(3000)], np.int32)
    for eps, mp in ((30.0, 4), (45.0, 8)):
        print(f"[case] far prefix groups eps={eps} minPts={mp}", flush=True)
        want = oracle.dbscan(pts, eps, mp)
        got, st = gpu_labels(ctx, pts, eps, mp, stats=True)
        assert np.array_equal(got, want), eps
        assert st["wide"] == 0 and st["list_overflow"] == 0, st


def test_unaligned_rows(ctx):
    """Rows that start off their vector alignment (views one to three
    elements into a tensor) are clustered like aligned ones, in 2-, 4- and
    8-D."""
    import torch
    for d, cfg in ((2, 1), (4, None), (8, 3)):
        if cfg is None:
            rng = np.random.default_rng(151)
            pts, eps, mp = quantise(make_blobs(rng, 5000, 4, 5, 0.03, 0.1), 12), 0.05 * 2 ** 12, 5
        else:
            w = make_config(cfg, n=5000)
            pts, eps, mp = w.points, w.eps, w.min_pts
        n = len(pts)
        flat = torch.zeros(n * d + 3, dtype=torch.int32, device="cuda")
        for off in (1, 2, 3):
            view = flat[off:off + n * d].view(n, d)
            view.copy_(torch.from_numpy(pts).cuda())
            assert view.data_ptr() % 16 != 0 or d == 2
            print(f"[case] unaligned rows d={d} offset={off}", flush=True)
            got = ctx.cluster(view, eps, mp).cpu().numpy()
            assert np.array_equal(got, oracle.dbscan(pts, eps, mp)), (d, off)


@pytest.mark.parametrize("lanes,budget", [("1", "1"), ("1", "16"), ("1", ""), ("0", "")])
def test_core_list_lane_walk(ctx, lanes, budget, monkeypatch):
    """Cube-mode core marking for three and four axes over the cube
    neighbour lists: one lane per point of a sparse cube (budgets so small
    that most points go on to the wave walk, and the default), or a wave per
    cube; the same labels and core flags as the oracle, also through the
    batch path and with the lists overflowing into the stencil."""
    monkeypatch.setenv("HCA_SEARCH", "cube")
    monkeypatch.setenv("HCA_CORE_LANES", lanes)
    if budget:
        monkeypatch.setenv("HCA_CORE_BUDGET", budget)
    for d in (3, 4):
        rng = np.random.default_rng(190 + d)
        pts = quantise(make_blobs(rng, 12000, d, 6, 0.02, 0.3), 12)
        for f, mp in ((0.02, 4), (0.04, 9), (0.08, 20)):
            eps = f * 2 ** 12
            print(f"[case] list lanes={lanes} budget={budget} d={d} eps={eps} minPts={mp}", flush=True)
            want, counts, _ = oracle.dbscan(pts, eps, mp, details=True)
            got, core, st = gpu_labels(ctx, pts, eps, mp, core=True, stats=True)
            assert np.array_equal(core.astype(bool), counts >= mp), (d, f, mp)
            assert np.array_equal(got, want), (d, f, mp)
            if lanes == "1" and budget == "1" and f == 0.04:
                assert st["core_rest"] > 0, st
    import torch
    jobs = [make_mixed(1300 + k, 3000 + 2000 * k, 3 + k % 2) for k in range(4)]
    flat = torch.from_numpy(np.concatenate([j.points.ravel() for j in jobs]).astype(np.int32)).cuda()
    got = ctx.cluster_batch(flat, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                            [j.min_pts for j in jobs]).cpu().numpy()
    at = 0
    for j in jobs:
        assert np.array_equal(got[at:at + j.n], oracle.dbscan(j.points, j.eps, j.min_pts)), j.name
        at += j.n
    monkeypatch.setenv("HCA_LIST_SLAB", "16")
    rng = np.random.default_rng(199)
    pts = quantise(make_blobs(rng, 8000, 3, 4, 0.03, 0.2), 12)
    check(ctx, pts, 0.05 * 2 ** 12, 6, f"list lanes={lanes} overflowing lists")


@pytest.mark.parametrize("lanes,budget", [("1", "1"), ("1", "24"), ("1", "512"), ("0", "512")])
def test_core_lane_walk(ctx, lanes, budget, monkeypatch):
    """Cube-mode core marking for one and two axes: one lane per point of a
    sparse cube (budgets so small that most points go on to the wave-wide
    walk, and the default), or a wave per cube; the same labels and core
    flags as the oracle, also through the batch path."""
    monkeypatch.setenv("HCA_CORE_LANES", lanes)
    monkeypatch.setenv("HCA_CORE_BUDGET", budget)
    for d in (1, 2):
        rng = np.random.default_rng(170 + d)
        pts = quantise(make_blobs(rng, 30000, d, 8, 0.01, 0.2), 14)
        for f, mp in ((0.002, 4), (0.004, 8), (0.01, 20)):
            eps = f * 2 ** 14
            print(f"[case] core lanes={lanes} budget={budget} d={d} eps={eps} minPts={mp}", flush=True)
            want, counts, _ = oracle.dbscan(pts, eps, mp, details=True)
            got, core, st = gpu_labels(ctx, pts, eps, mp, core=True, stats=True)
            assert np.array_equal(core.astype(bool), counts >= mp), (d, f, mp)
            assert np.array_equal(got, want), (d, f, mp)
            if lanes == "1" and budget == "1" and d == 2 and f == 0.004:
                assert st["core_rest"] > 0, st
    w = make_config(2, n=300_000)
    print(f"[case] core lanes={lanes} budget={budget} 2-D 300k", flush=True)
    assert np.array_equal(gpu_labels(ctx, w.points, w.eps, w.min_pts),
                          oracle.hca_grid(w.points, w.eps, w.min_pts, threads=0))
    import torch
    jobs = [make_mixed(1200 + k, 4000 + 3000 * k, 2) for k in range(4)]
    flat = torch.from_numpy(np.concatenate([j.points.ravel() for j in jobs]).astype(np.int32)).cuda()
    got = ctx.cluster_batch(flat, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                            [j.min_pts for j in jobs]).cpu().numpy()
    at = 0
    for j in jobs:
        assert np.array_equal(got[at:at + j.n], oracle.dbscan(j.points, j.eps, j.min_pts)), j.name
        at += j.n


@pytest.mark.parametrize("order", ["reverse", "permute"])
def test_schedule_orders(ctx, order, monkeypatch):
    """The wave-dealt units of every neighbour phase taken in reverse or in a
    permuted order (another schedule of the same atomics and unions): labels
    and core flags still equal the oracle's, in 2-D and 8-D, and in a batch."""
    monkeypatch.setenv("HCA_ORDER", order)
    for cfg, n in ((2, 200_000), (3, 100_000)):
        w = make_config(cfg, n=n)
        print(f"[case] order={order} {w.name} n={n}", flush=True)
        want = oracle.hca_grid(w.points, w.eps, w.min_pts, threads=0)
        got, core = gpu_labels(ctx, w.points, w.eps, w.min_pts, core=True)
        assert np.array_equal(got, want), (order, cfg)
        _, wcore, _ = oracle.hca_grid(w.points, w.eps, w.min_pts, threads=0, details=True)
        assert np.array_equal(core.astype(bool), wcore), (order, cfg)
    for mode in ("group", "cube"):
        monkeypatch.setenv("HCA_SEARCH", mode)
        rng = np.random.default_rng(181)
        pts = quantise(make_blobs(rng, 20000, 4, 6, 0.03, 0.1), 12)
        check(ctx, pts, 0.05 * 2 ** 12, 6, f"order={order} {mode} 4-D")
    monkeypatch.delenv("HCA_SEARCH")
    import torch
    jobs = [make_mixed(1300 + k, 3000 + 2000 * k, (2, 3, 4)[k % 3]) for k in range(6)]
    flat = torch.from_numpy(np.concatenate([j.points.ravel() for j in jobs]).astype(np.int32)).cuda()
    got = ctx.cluster_batch(flat, [j.n for j in jobs], [j.d for j in jobs], [j.eps for j in jobs],
                            [j.min_pts for j in jobs]).cpu().numpy()
    at = 0
    for j in jobs:
        assert np.array_equal(got[at:at + j.n], oracle.dbscan(j.points, j.eps, j.min_pts)), (order, j.name)
        at += j.n


def test_dense_groups(ctx):
    """Search groups holding tens of thousands of points (dense blobs in 5
    and 6 axes with eps near their spread): their cubes are linked pair by
    pair instead of point by point; labels equal the oracle's."""
    rng = np.random.default_rng(191)
    for d, n, std, f, mp in ((5, 60000, 0.006, 0.028, 8), (6, 40000, 0.01, 0.05, 10), (5, 30000, 0.004, 0.03, 4)):
        pts = quantise(make_blobs(rng, n, d, 3, std, 0.05), 14)
        check(ctx, pts, f * 2 ** 14, mp, f"dense groups d={d}")


def test_mixed_family(ctx):
    for seed in range(6):
        d = (2, 3, 4)[seed % 3]
        n = int(np.exp(np.random.default_rng(seed).uniform(np.log(1000), np.log(20000))))
        w = make_mixed(1000 + seed, n, d)
        check(ctx, w.points, w.eps, w.min_pts, f"mixed seed={seed}")


def test_degenerate_cases(ctx):
    same = np.full((300, 3), 77, np.int32)
    check(ctx, same, 0.5, 300, "identical, minPts=n")
    check(ctx, same, 0.5, 301, "identical, minPts>n")
    check(ctx, np.array([[5, -7]], np.int32), 3.0, 1, "single point")
    check(ctx, np.array([[5, -7]], np.int32), 3.0, 2, "single point noise")
    rng = np.random.default_rng(3)
    pts = rng.integers(-5000, 5000, size=(3000, 2)).astype(np.int32)
    check(ctx, pts, 0.3, 1, "eps < 1: only duplicates connect")
    check(ctx, pts, 1e6, 5, "eps beyond the diameter")
    k = 9
    lat = np.array([(i * k, j * k) for i in range(40) for j in range(40)], np.int32)
    check(ctx, lat, float(k), 5, "lattice on the eps boundary")
    check(ctx, lat, k - 1e-9, 2, "lattice just outside eps")
    line = np.stack([np.arange(5000) * 3, np.zeros(5000)], 1).astype(np.int32)
    check(ctx, line, 3.0, 3, "collinear chain")
    neg = quantise(make_blobs(rng, 3000, 4, 3, 0.05, 0.1), 10) - 100_000
    check(ctx, neg, 70.0, 4, "negative coordinates")
    # golden fixtures
    for name in ("closed_ball_core", "representative_split", "border_ties"):
        g = json.loads((GOLDEN / f"{name}.json").read_text())
        for case in g["cases"]:
            pts = np.array(case.get("points", g.get("points")), np.int32)
            got = gpu_labels(ctx, pts, case["eps"], case["min_pts"])
            assert got.tolist() == case["labels"], (name, case)


def test_chains(ctx):
    """Chains whose only links are consecutive points exactly eps apart: no
    redundant edge, so a single lost union-find link changes the labels."""
    rng = np.random.default_rng(5)
    for n in (5000, 60000):
        i = np.arange(n)
        line = np.stack([i * 3, np.zeros(n)], 1).astype(np.int32)
        diag = np.stack([i, i], 1).astype(np.int32)
        cube8 = np.zeros((n, 8), np.int32)
        cube8[:, 0] = cube8[:, 1] = i * 2                # steps of dist^2 = 8 in 8-D
        for name, pts, eps in (("line", line, 3.0), ("diagonal", diag, 2 ** 0.5),
                               ("8-D diagonal", cube8, 8 ** 0.5)):
            for order in ("sorted", "reversed", "shuffled"):
                p = pts[::-1] if order == "reversed" else (
                    pts[rng.permutation(n)] if order == "shuffled" else pts)
                p = np.ascontiguousarray(p)
                check(ctx, p, eps, 3, f"chain {name} {order}")
                check(ctx, p, eps, 1, f"chain {name} {order} minPts=1")


def test_wide_distances(ctx):
    """Coordinates and eps large enough that squared distances need 64 bits."""
    rng = np.random.default_rng(11)
    x = make_blobs(rng, 4000, 3, 4, 0.03, 0.1)
    pts = quantise(x, 26)                          # spans ~2^26
    eps = 0.05 * 2 ** 26
    got, stats = gpu_labels(ctx, pts, eps, 5, stats=True)
    assert stats["wide"] == 1
    assert np.array_equal(got, oracle.dbscan(pts, eps, 5))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_sort_digit_widths(ctx, d):
    """Cube keys from a few bits to past 32 (9-bit digits for 32-bit keys, 8-bit
    ones for 64-bit keys, the pass count evened out over the key): the same
    labels as the oracle at every width."""
    rng = np.random.default_rng(300 + d)
    pts = quantise(make_blobs(rng, 1500, d, 4, 0.01, 0.3), 14)
    for eps in (3.0, 10.0, 40.0, 160.0, 640.0):
        check(ctx, pts, eps, 3, f"digit widths d={d}")
        _, st = gpu_labels(ctx, pts, eps, 3, stats=True)
        kb = st["key_bits"]
        rb = 9 if kb <= 32 else 8
        assert st["sort_passes"] == max(1, -(-kb // rb)), (kb, st["sort_passes"])


@pytest.mark.parametrize("tile,threads", [("4096", "256"), ("4096", "512"), ("4096", "1024"), ("8192", "")])
def test_sort_tiles(ctx, tile, threads, monkeypatch):
    """Radix tiles ranked by 256, 512 or 1024 threads, and tiles of 8192 keys
    (chosen from 8M keys on), with rows of one and two axes carried through
    the passes and wider rows gathered: the oracle's labels, on inputs whose
    length leaves a ragged last tile."""
    monkeypatch.setenv("HCA_SORT_TILE", tile)
    if threads:
        monkeypatch.setenv("HCA_SORT_THREADS", threads)
    rng = np.random.default_rng(410)
    for d, n, eps in ((1, 30_001, 2.0), (2, 50_003, 60.0), (3, 20_011, 300.0)):
        pts = quantise(make_blobs(rng, n, d, 6, 0.01, 0.1), 16)
        check(ctx, pts, eps, 5, f"sort tiles {tile}/{threads or 'default'} d={d}")


def test_large_sort_tiles_agree(ctx, monkeypatch):
    """At 9M points (tiles of 8192 keys by default) the labels equal those
    of tiles of 4096 keys, and core points of a sample pass the brute-force
    check of the definition."""
    import torch
    w = make_config(2, n=9_000_000)
    pts = torch.from_numpy(w.points).cuda()
    print("[case] 9M 2-D, tiles of 8192 vs 4096", flush=True)
    big, core = ctx.cluster(pts, w.eps, w.min_pts, core=True)
    monkeypatch.setenv("HCA_SORT_TILE", "4096")
    small = ctx.cluster(pts, w.eps, w.min_pts)
    assert torch.equal(big, small)
    rng = np.random.default_rng(5)
    core = core.cpu().numpy()
    e2 = oracle.exact_eps2(w.eps)
    for i in rng.choice(w.n, 40, replace=False):
        d2 = ((w.points.astype(np.int64) - w.points[i].astype(np.int64)) ** 2).sum(1)
        assert bool(core[i]) == (int((d2 <= e2).sum()) >= w.min_pts), i


def test_errors(ctx):
    from paper_1912_00323_amd import hca
    import torch
    big = torch.tensor([[0, 0], [1 << 30, 0]], dtype=torch.int32, device="cuda")
    with pytest.raises(hca.HcaError) as e:
        ctx.cluster(big, 1.0, 1)
    assert e.value.status == hca.HCA_E_RANGE
    wide = torch.tensor([[0] * 8, [(1 << 29)] * 8], dtype=torch.int32, device="cuda")
    with pytest.raises(hca.HcaError) as e:
        ctx.cluster(wide, 1.0, 1)
    assert e.value.status == hca.HCA_E_RANGE
    ok = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    for eps, mp in ((0.0, 1), (float("nan"), 1), (1.0, 0)):
        with pytest.raises(hca.HcaError) as e:
            ctx.cluster(ok, eps, mp)
        assert e.value.status == hca.HCA_E_INVAL
    # the context stays usable after errors
    assert ctx.cluster(ok, 1.0, 1).cpu().tolist() == [0, 0, 0, 0]
    empty = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    assert ctx.cluster(empty, 1.0, 1).numel() == 0


def test_host_pointer_entry(ctx):
    w = make_config(1)
    assert np.array_equal(ctx.cluster_host(w.points, w.eps, w.min_pts),
                          oracle.dbscan(w.points, w.eps, w.min_pts))


def test_side_stream(ctx):
    import torch
    w = make_config(1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t = torch.from_numpy(w.points).to("cuda", non_blocking=False)
        lab = ctx.cluster(t, w.eps, w.min_pts)
    s.synchronize()
    assert np.array_equal(lab.cpu().numpy(), oracle.dbscan(w.points, w.eps, w.min_pts))


def _sampled_checks(w, got, core, samples=300):
    """One-by-one oracle checks on sampled points: |N(i)| by brute force over
    all points decides core; a sampled non-core point with a core neighbour
    must carry the label of its nearest core point (ties: smaller index)."""
    rng = np.random.default_rng(99)
    p = w.points.astype(np.int64)
    e2 = oracle.exact_eps2(w.eps)
    for i in rng.choice(w.n, size=min(samples, w.n), replace=False):
        d2 = ((p - p[i]) ** 2).sum(1)
        nb = d2 <= e2
        assert core[i] == (nb.sum() >= w.min_pts), i
        if not core[i]:
            cand = np.flatnonzero(nb & core)
            if len(cand) == 0:
                assert got[i] == -1, i
            else:
                j = cand[np.lexsort((cand, d2[cand]))[0]]
                assert got[i] == got[j] and got[i] >= 0, i
        else:
            cn = np.flatnonzero(nb & core)
            assert (got[cn] == got[i]).all(), i


@pytest.mark.parametrize("k", [2, 3])
def test_full_size_workloads(ctx, k):
    exp = json.loads((GOLDEN / "full_size_expected.json").read_text())
    w = make_config(k)
    e = exp["workloads"][w.name]
    assert digest(w.points.reshape(-1)) == e["points_sha256"], "input generator drifted"
    print(f"[case] full-size {w.name}", flush=True)
    got, core, stats = gpu_labels(ctx, w.points, w.eps, w.min_pts, core=True, stats=True)
    core = core.astype(bool)
    assert int(core.sum()) == e["n_core"]
    assert digest(core.astype(np.int32)) == e["core_sha256"]
    assert stats["n_clusters"] == e["n_clusters"] and stats["n_noise"] == e["n_noise"]
    assert digest(got) == e["labels_sha256"]
    _sampled_checks(w, got, core)


def test_repeatable(ctx):
    w = make_config(2, n=200_000)
    first = gpu_labels(ctx, w.points, w.eps, w.min_pts)
    for _ in range(5):
        assert np.array_equal(gpu_labels(ctx, w.points, w.eps, w.min_pts), first)
    assert np.array_equal(first, oracle.dbscan(w.points, w.eps, w.min_pts))


def test_prepared_call(ctx):
    """A call prepared once on fixed tensors and made repeatedly (the form the
    benchmark times) against the oracle, including after the data change in
    place."""
    import torch
    w = make_config(1)
    pts = torch.from_numpy(w.points).cuda()
    out = torch.empty(w.n, dtype=torch.int32, device="cuda")
    call = ctx.prepared(pts, w.eps, w.min_pts, out)
    want = oracle.dbscan(w.points, w.eps, w.min_pts)
    for _ in range(3):
        out.fill_(-7)
        call()
        assert np.array_equal(out.cpu().numpy(), want)
    moved = w.points[::-1].copy()
    moved[:, 1] += 77
    pts.copy_(torch.from_numpy(moved))
    call()
    assert np.array_equal(out.cpu().numpy(), oracle.dbscan(moved, w.eps, w.min_pts))


def test_plan_reuse(ctx):
    """Calls planned ahead from the box of the previous calls: the same data
    again (planned ahead, its box compared on the device), data of the same
    shape with another box (the comparison fails and the call runs again from
    its own box), a span past 2^30 once a plan is armed again (the error of the
    call planned from its own box), and reuse switched off."""
    import torch
    from paper_1912_00323_amd import hca
    ctx.set_plan_reuse(True)
    for d in (2, 3, 5, 8):
        rng = np.random.default_rng(300 + d)
        pts = quantise(make_blobs(rng, 6000, d, 5, 0.04, 0.1), 10)
        eps, mp = (0.06 + 0.01 * d) * 2 ** 10, 6
        want = oracle.dbscan(pts, eps, mp)
        t = torch.from_numpy(pts).cuda()
        print(f"[case] plan reuse d={d} same box", flush=True)
        c0, r0 = ctx.plan_reuse_counts()
        for _ in range(4):
            assert np.array_equal(ctx.cluster(t, eps, mp).cpu().numpy(), want)
        c1, r1 = ctx.plan_reuse_counts()
        assert c1 - c0 == 2 and r1 == r0, (d, c0, c1, r0, r1)
        print(f"[case] plan reuse d={d} other box", flush=True)
        other = pts.copy()
        other[:, 0] += 1234
        other[7] -= 3000
        got = ctx.cluster(torch.from_numpy(other).cuda(), eps, mp).cpu().numpy()
        assert np.array_equal(got, oracle.dbscan(other, eps, mp))
        c2, r2 = ctx.plan_reuse_counts()
        assert (c2, r2) == (c1 + 1, r1 + 1), (d, c1, c2, r1, r2)
        print(f"[case] plan reuse d={d} span past 2^30", flush=True)
        for _ in range(2):
            ctx.cluster(t, eps, mp)
        bad = pts.copy()
        bad[0, 0] += 1 << 30
        with pytest.raises(hca.HcaError) as e:
            ctx.cluster(torch.from_numpy(bad).cuda(), eps, mp)
        assert e.value.status == hca.HCA_E_RANGE
        assert ctx.plan_reuse_counts() == (c2 + 1, r2 + 1)
        assert np.array_equal(ctx.cluster(t, eps, mp).cpu().numpy(), want)
    ctx.set_plan_reuse(False)
    counts = ctx.plan_reuse_counts()
    for _ in range(3):
        assert np.array_equal(ctx.cluster(t, eps, mp).cpu().numpy(), want)
    assert ctx.plan_reuse_counts() == counts
    ctx.set_plan_reuse(True)


def test_representative_only_mode(ctx):
    """The paper's merge as printed (facing representatives alone) against the
    oracle's representative-only mode, including the fixture where it splits a
    DBSCAN cluster; then back to exact."""
    from paper_1912_00323_amd import hca
    import torch
    g = json.loads((GOLDEN / "representative_split.json").read_text())
    ctx.set_exact(False)
    try:
        for case in g["cases"]:
            pts = np.array(g["points"], np.int32)
            got = gpu_labels(ctx, pts, case["eps"], case["min_pts"])
            assert got.tolist() == case["rep_only_labels"]
        faces = json.loads((GOLDEN / "representative_faces.json").read_text())
        for case in faces["cases"]:
            pts = np.array(case["points"], np.int32)
            print(f"[case] representatives only, fixture {case['name']}", flush=True)
            got = gpu_labels(ctx, pts, case["eps"], case["min_pts"])
            assert got.tolist() == case["rep_only_labels"], case["name"]
        for d in (2, 3, 4):
            for seed in range(3):
                rng = np.random.default_rng(300 + 10 * d + seed)
                x = make_blobs(rng, 6000, d, 6, 0.04, 0.15)
                pts = quantise(x, 12)
                eps, mp = (0.03 + 0.01 * d) * 2 ** 12, 5
                print(f"[case] representatives only d={d} seed={seed}", flush=True)
                want = oracle.hca_grid(pts, eps, mp, rep_mode=1)
                got = gpu_labels(ctx, pts, eps, mp)
                assert np.array_equal(got, want), (d, seed)
        w = make_config(2, n=200_000)
        assert np.array_equal(gpu_labels(ctx, w.points, w.eps, w.min_pts),
                              oracle.hca_grid(w.points, w.eps, w.min_pts, rep_mode=1))
        with pytest.raises(hca.HcaError) as e:                 # d = 8: search groups, no representatives
            w8 = make_config(3, n=2000)
            ctx.cluster(torch.from_numpy(w8.points).cuda(), w8.eps, w8.min_pts)
        assert e.value.status == hca.HCA_E_INVAL
    finally:
        ctx.set_exact(True)
    pts = np.array(g["points"], np.int32)
    assert gpu_labels(ctx, pts, 14.15, 1).tolist() == [0, 0, 0]
