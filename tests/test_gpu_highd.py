"""GPU parity for data with more than eight axes (d up to 64; the paper's data
sets reach 54 dimensions, Table 1): the HIP path against the oracle's DBSCAN
definition, label for label."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import make_blobs, quantise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no HIP device visible"
    from paper_1912_00323_amd import hca
    c = hca.Context(0)
    yield c
    c.close()


def gpu_run(ctx, pts, eps, min_pts, core=False, stats=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(pts, np.int32)).cuda()
    out = ctx.cluster(t, eps, min_pts, core=core, stats=stats)
    if isinstance(out, tuple):
        return tuple(o.cpu().numpy() if hasattr(o, "cpu") else o for o in out)
    return out.cpu().numpy()


def check(ctx, pts, eps, mp, tag=""):
    print(f"[case] {tag} n={len(pts)} d={pts.shape[1]} eps={eps:.3f} minPts={mp}", flush=True)
    want, counts, _ = oracle.dbscan(pts, eps, mp, details=True)
    got, core = gpu_run(ctx, pts, eps, mp, core=True)
    assert np.array_equal(core.astype(bool), counts >= mp), f"{tag}: core flags differ"
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{tag}: {len(bad)} labels differ, first at {bad[:10]} "
                             f"got {got[bad[:10]]} want {want[bad[:10]]}")


def blobs(seed, n, d, k=5, std=0.03, noise=0.1, q=10):
    return quantise(make_blobs(np.random.default_rng(seed), n, d, k, std, noise), q)


@pytest.mark.parametrize("d", [9, 12, 16, 27, 54, 64])
def test_blobs_many_axes(ctx, d):
    for n in (1, 2, 63, 65, 3000):
        pts = blobs(500 + d + n, n, d)
        for f in (0.7, 0.8, 1.0):
            eps = 0.03 * math.sqrt(2 * d) * f * 2 ** 10
            for mp in (1, 4, 9):
                check(ctx, pts, eps, mp, f"blobs d={d} f={f}")


# shapes of the paper's data sets (Table 1): Vicon action (5045 x 27 and
# 3853 x 54), leaf (340 x 16); synthetic blobs stand in for their records
@pytest.mark.parametrize("n,d", [(5045, 27), (3853, 54), (340, 16)])
def test_paper_shapes(ctx, n, d):
    pts = blobs(40 + d, n, d, k=8, std=0.025)
    for f, mp in ((0.75, 5), (0.9, 10)):
        check(ctx, pts, 0.025 * math.sqrt(2 * d) * f * 2 ** 10, mp, f"paper shape {n}x{d}")


@pytest.mark.parametrize("budget", ["64", "256"])
def test_second_core_pass(ctx, budget, monkeypatch):
    """A candidate budget so small that the first core-marking pass leaves
    many points undecided: the second pass walks them to the end, and labels
    and core flags still equal the oracle's, on the paper's shapes and on
    blobs at 9 to 64 axes."""
    monkeypatch.setenv("HCA_HD_BUDGET", budget)
    cases = [(blobs(40 + d, n, d, k=8, std=0.025), 0.025 * math.sqrt(2 * d) * f * 2 ** 10, mp, f"{n}x{d}")
             for n, d in ((5045, 27), (3853, 54), (340, 16)) for f, mp in ((0.75, 5), (0.9, 10))]
    cases += [(blobs(600 + d, 3000, d), 0.03 * math.sqrt(2 * d) * 0.8 * 2 ** 10, 9, f"blobs 3000x{d}")
              for d in (9, 12, 64)]
    rest = 0
    for pts, eps, mp, tag in cases:
        print(f"[case] second core pass budget={budget} {tag} eps={eps:.3f} minPts={mp}", flush=True)
        want, counts, _ = oracle.dbscan(pts, eps, mp, details=True)
        got, core, st = gpu_run(ctx, pts, eps, mp, core=True, stats=True)
        assert np.array_equal(core.astype(bool), counts >= mp), tag
        assert np.array_equal(got, want), tag
        rest += st["core_rest"]
        if len(pts) > 1000:
            assert st["core_rest"] > 0, tag
    assert rest > 0


def test_stats_many_axes(ctx):
    pts = blobs(7, 4000, 20)
    eps, mp = 0.03 * math.sqrt(40) * 0.8 * 2 ** 10, 6
    want, counts, _ = oracle.dbscan(pts, eps, mp, details=True)
    got, st = gpu_run(ctx, pts, eps, mp, stats=True)
    assert np.array_equal(got, want)
    assert st["n_clusters"] == want.max() + 1
    assert st["n_noise"] == (want < 0).sum()
    assert st["n_core_points"] == (counts >= mp).sum()
    assert st["list_overflow"] == 0 and st["n_groups"] >= 1 and st["n_cells"] >= st["n_groups"]


def test_degenerate_many_axes(ctx):
    rng = np.random.default_rng(31)
    # every point the same: one cluster, or all noise when minPts > n
    same = np.full((500, 20), 123, np.int32)
    check(ctx, same, 1.0, 3, "identical points")
    check(ctx, same, 1.0, 501, "identical points, minPts > n")
    # eps below 1: only duplicates are neighbours
    dup = rng.integers(0, 4, size=(800, 12)).astype(np.int32)
    check(ctx, dup, 0.5, 2, "duplicates only")
    # a single point, two far apart
    check(ctx, np.zeros((1, 33), np.int32), 3.0, 1, "one point")
    two = np.zeros((2, 40), np.int32)
    two[1, 17] = 1000
    check(ctx, two, 10.0, 1, "two points")
    # data that varies along two axes only: the same labels as in 2-D
    p2 = blobs(9, 3000, 2, std=0.02)
    pad = np.concatenate([p2, np.full((3000, 30), -5, np.int32)], axis=1)
    perm = np.random.default_rng(3).permutation(32)
    padded = np.ascontiguousarray(pad[:, perm])
    eps, mp = 0.015 * 2 ** 10, 4
    check(ctx, padded, eps, mp, "two varying axes of 32")
    assert np.array_equal(gpu_run(ctx, padded, eps, mp), gpu_run(ctx, p2, eps, mp))


def test_wide_distances_many_axes(ctx):
    # 2^16 fixed point over 12 axes: squared spans add past 2^31 (64-bit sums)
    pts = blobs(11, 3000, 12, q=16)
    for f, mp in ((0.8, 4), (1.0, 8)):
        check(ctx, pts, 0.03 * math.sqrt(24) * f * 2 ** 16, mp, "wide sums")


@pytest.mark.parametrize("bits", ["1", "3"])
def test_hash_collisions(ctx, bits, monkeypatch):
    # so few cube-hash bits that cubes share keys: they are told apart after
    # the sort, a cube may come out in several runs, and nothing changes
    monkeypatch.setenv("HCA_HASH_BITS", bits)
    pts = blobs(13, 3000, 10, std=0.02, q=8)
    for f, mp in ((0.8, 3), (1.2, 6)):
        check(ctx, pts, 0.02 * math.sqrt(20) * f * 2 ** 8, mp, f"hash bits {bits}")


@pytest.mark.parametrize("slab", ["1", "4"])
def test_list_capacity_retry(ctx, slab, monkeypatch):
    # neighbour lists far too small at first: the call grows them and reruns
    monkeypatch.setenv("HCA_LIST_SLAB", slab)
    pts = blobs(17, 3000, 16)
    check(ctx, pts, 0.03 * math.sqrt(32) * 0.9 * 2 ** 10, 5, f"list slab {slab}")


def test_errors_many_axes(ctx):
    import torch
    from paper_1912_00323_amd import hca
    with pytest.raises(hca.HcaError) as e:
        gpu_run(ctx, np.zeros((4, 65), np.int32), 1.0, 1)
    assert e.value.status == hca.HCA_E_INVAL
    wide = np.zeros((2, 9), np.int32)
    wide[1] = (1 << 30) - 1
    with pytest.raises(hca.HcaError) as e:
        gpu_run(ctx, wide, 1.0, 1)
    assert e.value.status == hca.HCA_E_RANGE
    ctx.set_exact(False)
    try:
        with pytest.raises(hca.HcaError) as e:
            gpu_run(ctx, blobs(1, 100, 12), 50.0, 2)
        assert e.value.status == hca.HCA_E_INVAL
    finally:
        ctx.set_exact(True)
    check(ctx, blobs(1, 100, 12), 50.0, 2, "after errors")
    del torch


@pytest.mark.parametrize("packed", ["0", "1"])
def test_row_forms(ctx, packed, monkeypatch):
    # spans below 2^15: packed int16 rows (default) or plain 32-bit rows; a
    # span of 2^15 or more always takes the plain form
    monkeypatch.setenv("HCA_PACKED", packed)
    for d in (16, 54):
        pts = blobs(60 + d, 4000, d)
        for f, mp in ((0.75, 4), (0.9, 9)):
            check(ctx, pts, 0.03 * math.sqrt(2 * d) * f * 2 ** 10, mp, f"rows packed={packed}")
        _, st = gpu_run(ctx, pts, 0.03 * math.sqrt(2 * d) * 2 ** 10, 4, stats=True)
        assert st["packed_rows"] == int(packed) and 1 <= st["key_axes"] <= 8
    big = blobs(61, 3000, 20, q=15)
    big[0, 0] = 0
    big[1, 0] = (1 << 15) + 7
    check(ctx, big, 0.03 * math.sqrt(40) * 0.8 * 2 ** 15, 5, "span past 2^15")
    assert gpu_run(ctx, big, 100.0, 5, stats=True)[1]["packed_rows"] == 0


def test_full_size_54_axes_sampled():
    """The 54-axis workload at full size (the shape of the paper's PAMAP2
    set, 3,850,505 points): the core flag of sampled points against their
    brute-force neighbour counts, every core neighbour of a sampled core point
    in its cluster, a sampled non-core point in the cluster of its nearest
    core point (ties to the smaller index) or noise, and canonical numbering
    over all labels.  Squared distances come from float64 products, exact
    here (every product below 2^24, every sum below 2^31)."""
    import torch
    from paper_1912_00323_amd import hca
    from paper_1912_00323_amd.datagen import make_high
    w = make_high(54, 3_850_505)
    print(f"[case] {w.name} eps={w.eps:.3f} minPts={w.min_pts}", flush=True)
    c = hca.Context(0)
    try:
        t = torch.from_numpy(w.points).cuda()
        lab, core = c.cluster(t, w.eps, w.min_pts, core=True)
        lab, core = lab.cpu().numpy(), core.cpu().numpy().astype(bool)
        del t
    finally:
        c.close()
    eps2 = oracle.exact_eps2(w.eps)
    # canonical: the first occurrences of the labels come in the order 0, 1, 2, ...
    seen = lab[lab >= 0]
    _, first = np.unique(seen, return_index=True)
    assert np.array_equal(np.argsort(first), np.arange(len(first)))
    rng = np.random.default_rng(99)
    pick = np.concatenate([rng.choice(np.flatnonzero(core), 16, replace=False),
                           rng.choice(np.flatnonzero(~core), 16, replace=False)])
    S = w.points[pick].astype(np.float64)
    s2 = (S * S).sum(1)
    d2 = np.empty((len(pick), w.n), np.float64)
    for a in range(0, w.n, 500_000):
        X = w.points[a:a + 500_000].astype(np.float64)
        d2[:, a:a + len(X)] = (X * X).sum(1)[None, :] + s2[:, None] - 2.0 * (S @ X.T)
    for r, i in enumerate(pick):
        nb = np.flatnonzero(d2[r] <= eps2)
        assert core[i] == (len(nb) >= w.min_pts), ("core flag", i, len(nb))
        cn = nb[core[nb]]
        if core[i]:
            assert (lab[cn] == lab[i]).all(), ("core neighbour in another cluster", i)
        elif len(cn):
            j = cn[np.lexsort((cn, d2[r][cn]))[0]]
            assert lab[i] == lab[j], ("border owner", i, j)
        else:
            assert lab[i] == -1, ("noise", i)
