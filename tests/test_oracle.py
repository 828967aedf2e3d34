"""Pins for the CPU oracle (no GPU needed).

Every check here compares the oracle with something other than itself: exact
rational arithmetic, hand-derived fixtures under ``tests/golden/``, a 1-D closed
form, scikit-learn's DBSCAN and KD-tree, scipy's connected components, the
original expand-cluster procedure of DBSCAN, and invariances of the
definitions.  ``test_planted_mistakes_are_caught`` builds copies of the oracle
with one deliberate mistake each and checks that some pin fails on every one.
"""
from __future__ import annotations

import bisect
import json
import math
from collections import deque
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd.datagen import make_blobs, make_config, quantise

GOLDEN = Path(__file__).resolve().parent / "golden"


# --------------------------------------------------------------------------
# independent helpers (none of them calls the oracle)
# --------------------------------------------------------------------------
def rational_eps2(eps: float) -> int:
    """floor(eps^2) by exact rational arithmetic, saturated at 2^63 - 1 (no
    int64 squared distance can exceed that)."""
    return min(math.floor(Fraction(eps) ** 2), 2 ** 63 - 1)


def canonical(labels) -> np.ndarray:
    """Renumber a labelling so clusters are ranked by smallest member index."""
    out = np.full(len(labels), -1, np.int32)
    seen = {}
    for i, c in enumerate(labels):
        if c < 0:
            continue
        if c not in seen:
            seen[c] = len(seen)
        out[i] = seen[c]
    return out


def exact_dist2(p, q) -> int:
    return int(sum((int(a) - int(b)) ** 2 for a, b in zip(p, q)))


def dbscan_1d(x, eps2: int, min_pts: int) -> np.ndarray:
    """Closed form in one dimension.  Sorted values; |N(i)| by two binary
    searches; core points split into clusters wherever two consecutive core
    values are more than sqrt(eps2) apart; a border point takes the nearest
    core value within eps (ties to the smaller index)."""
    x = [int(v) for v in x]
    n = len(x)
    e = math.isqrt(eps2)                      # |dx| <= e  <=>  dx^2 <= eps2
    xs = sorted(x)
    cnt = [bisect.bisect_right(xs, v + e) - bisect.bisect_left(xs, v - e) for v in x]
    core = [c >= min_pts for c in cnt]
    core_vals = sorted(set(x[i] for i in range(n) if core[i]))
    run_of = {}
    run = -1
    prev = None
    for v in core_vals:
        if prev is None or v - prev > e:
            run += 1
        run_of[v] = run
        prev = v
    core_idx_by_val = {}
    for i in range(n):
        if core[i]:
            core_idx_by_val.setdefault(x[i], []).append(i)
    lab = [-1] * n
    for i in range(n):
        if core[i]:
            lab[i] = run_of[x[i]]
            continue
        best = None
        for v in core_vals:
            dd = (v - x[i]) ** 2
            if dd <= eps2:
                key = (dd, min(core_idx_by_val[v]))
                if best is None or key < best[0]:
                    best = (key, run_of[v])
        lab[i] = best[1] if best else -1
    return canonical(lab)


def dbscan_expand(points, eps2: int, min_pts: int) -> np.ndarray:
    """The original DBSCAN procedure (appendix, last paragraph): start from an
    unvisited point; if it is core, grow a cluster by repeatedly retrieving the
    neighbourhoods of the core points reached.  Border points are then given
    to their nearest core point (ties to the smaller index).  Pure Python,
    for tiny inputs only."""
    pts = [tuple(int(v) for v in p) for p in points]
    n = len(pts)
    nbr = [[j for j in range(n) if exact_dist2(pts[i], pts[j]) <= eps2] for i in range(n)]
    core = [len(nbr[i]) >= min_pts for i in range(n)]
    cl = [-1] * n
    c = 0
    for i in range(n):
        if not core[i] or cl[i] >= 0:
            continue
        cl[i] = c
        q = deque([i])
        while q:
            u = q.popleft()
            for v in nbr[u]:
                if core[v] and cl[v] < 0:
                    cl[v] = c
                    q.append(v)
        c += 1
    lab = list(cl)
    for i in range(n):
        if core[i]:
            continue
        cands = [(exact_dist2(pts[i], pts[j]), j) for j in nbr[i] if core[j]]
        lab[i] = cl[min(cands)[1]] if cands else -1
    return canonical(lab)


def same_partition(a, b) -> bool:
    """Do two labellings of the same items define the same partition?"""
    fwd, bwd = {}, {}
    for x, y in zip(a.tolist(), b.tolist()):
        if fwd.setdefault(x, y) != y or bwd.setdefault(y, x) != x:
            return False
    return True


def rand_points(rng, n, d, span, dup_frac=0.1):
    p = rng.integers(-span, span + 1, size=(n, d)).astype(np.int32)
    k = int(dup_frac * n)
    if k and n > 1:
        p[rng.integers(0, n, k)] = p[rng.integers(0, n, k)]
    return p


# --------------------------------------------------------------------------
# pins: each takes an oracle library handle (None = the real build)
# --------------------------------------------------------------------------
def pin_eps2_rational(lib):
    rng = np.random.default_rng(11)
    vals = [81.92, 262.144, 245.76, 14.15, 5.0, 2.0, 7.0, 0.75, 1.0, 1e-3, 3.999999999,
            float(2 ** 20) + 0.5, 46340.95, 123456.789]
    vals += list(rng.uniform(0.5, 5000.0, 200)) + list(np.exp(rng.uniform(-5, 25, 100)))
    for v in vals:
        assert oracle.exact_eps2(v, lib=lib) == rational_eps2(v), v
    assert oracle.exact_eps2(0.02 * 2 ** 12, lib=lib) == 6710
    assert oracle.exact_eps2(0.004 * 2 ** 16, lib=lib) == 68719
    assert oracle.exact_eps2(0.06 * 2 ** 12, lib=lib) == 60397


def pin_golden(lib):
    for name in ("closed_ball_core", "representative_split", "border_ties"):
        g = json.loads((GOLDEN / f"{name}.json").read_text())
        for case in g["cases"]:
            pts = np.array(case.get("points", g.get("points")), np.int32)
            got = oracle.dbscan(pts, case["eps"], case["min_pts"], lib=lib)
            assert got.tolist() == case["labels"], (name, case)


def pin_closed_form_1d(lib):
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(1, 400))
        span = int(rng.integers(1, 300))
        x = rand_points(rng, n, 1, span, 0.2)
        eps = float(rng.uniform(0.5, 12.0)) if trial % 4 else float(rng.integers(1, 10))
        mp = int(rng.integers(1, 8))
        want = dbscan_1d(x[:, 0], rational_eps2(eps), mp)
        got = oracle.dbscan(x, eps, mp, lib=lib)
        assert np.array_equal(got, want), (trial, n, eps, mp)


def _sklearn_check(points, eps, min_pts, lib):
    from sklearn.cluster import DBSCAN
    from sklearn.neighbors import KDTree
    eps2 = rational_eps2(eps)
    # dist2 is an integer, so dist <= sqrt(eps2 + 0.5) <=> dist2 <= eps2; the
    # half-unit margin dwarfs float64 rounding for these coordinate ranges.
    r = math.sqrt(eps2 + 0.5)
    x = points.astype(np.float64)
    sk = DBSCAN(eps=r, min_samples=min_pts, algorithm="kd_tree").fit(x)
    got, counts, owner = oracle.dbscan(points, eps, min_pts, details=True, lib=lib)
    core = np.zeros(len(x), bool)
    core[sk.core_sample_indices_] = True
    assert np.array_equal(counts >= min_pts, core), "core set differs"
    assert np.array_equal(got < 0, sk.labels_ < 0), "noise set differs"
    assert same_partition(got[core], sk.labels_[core]), "core partition differs"
    # border rule: nearest core point by exact dist2, then smaller index
    border = np.flatnonzero(~core & (got >= 0))
    if len(border):
        cidx = np.flatnonzero(core)
        tree = KDTree(x[cidx])
        hits = tree.query_radius(x[border], r)
        for b, h in zip(border, hits):
            cand = cidx[h]
            d2 = ((points[cand].astype(np.int64) - points[b].astype(np.int64)) ** 2).sum(1)
            j = cand[np.lexsort((cand, d2))[0]]
            assert got[b] == got[j], ("border owner", b, j)
    assert np.array_equal(got, canonical(got)), "labels not canonical"


def pin_sklearn(lib):
    rng = np.random.default_rng(7)
    for d, n, span, eps, mp in [(2, 600, 60, 4.5, 4), (3, 500, 30, 5.0, 5), (5, 400, 12, 6.3, 3),
                                (8, 300, 6, 7.9, 4), (2, 800, 100, 6.0, 1), (4, 400, 10, 4.0, 6)]:
        pts = rand_points(rng, n, d, span)
        _sklearn_check(pts, eps, mp, lib)
    w = make_config(1)
    _sklearn_check(w.points, w.eps, w.min_pts, lib)
    # the paper's data sets reach 16, 27 and 54 dimensions (Table 1)
    for d, n, k, std, eps, mp in [(16, 500, 5, 0.03, 0.16, 4), (27, 400, 4, 0.03, 0.2, 4),
                                  (54, 300, 3, 0.02, 0.17, 3)]:
        pts = quantise(make_blobs(np.random.default_rng(23), n, d, k, std, 0.1), 8)
        _sklearn_check(pts, eps * 2 ** 8, mp, lib)


def pin_scipy_min_pts_1(lib):
    """minPts = 1: every point is core, clusters are the components of the
    eps-graph, no noise."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    for d, n, span, eps in [(2, 700, 80, 3.5), (3, 500, 20, 3.0), (6, 300, 5, 4.2)]:
        pts = rand_points(rng, n, d, span)
        r = math.sqrt(rational_eps2(eps) + 0.5)
        pairs = cKDTree(pts.astype(np.float64)).query_pairs(r, output_type="ndarray")
        g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
        _, comp = connected_components(g, directed=False)
        got = oracle.dbscan(pts, eps, 1, lib=lib)
        assert (got >= 0).all()
        assert np.array_equal(got, canonical(comp))


def pin_expand_cluster(lib):
    rng = np.random.default_rng(13)
    for trial in range(30):
        d = int(rng.integers(1, 9))
        n = int(rng.integers(1, 70))
        pts = rand_points(rng, n, d, int(rng.integers(2, 12)), 0.15)
        eps = float(rng.uniform(1.0, 9.0))
        mp = int(rng.integers(1, 6))
        want = dbscan_expand(pts, rational_eps2(eps), mp)
        got = oracle.dbscan(pts, eps, mp, lib=lib)
        assert np.array_equal(got, want), (trial, d, n, eps, mp)
    for trial, d in enumerate((12, 27, 54)):
        pts = rand_points(rng, 60, d, 2, 0.2)
        eps = float(rng.uniform(3.0, 9.0))
        want = dbscan_expand(pts, rational_eps2(eps), 3)
        got = oracle.dbscan(pts, eps, 3, lib=lib)
        assert np.array_equal(got, want), (trial, d, eps)


def pin_special_cases(lib):
    rng = np.random.default_rng(17)
    pts = rand_points(rng, 200, 3, 50)
    # minPts > n: nothing is core, everything is noise
    assert (oracle.dbscan(pts, 10.0, 201, lib=lib) == -1).all()
    # eps at least the diameter: one cluster
    assert (oracle.dbscan(pts, 200.0, 5, lib=lib) == 0).all()
    # square lattice with spacing k and eps = k exactly: the 4-neighbours are
    # on the boundary of the ball.  minPts = 5 -> interior core, edges border,
    # corners (only 2 non-core neighbours) noise.
    k = 7
    g = np.array([(i * k, j * k) for i in range(5) for j in range(5)], np.int32)
    lab = oracle.dbscan(g, float(k), 5, lib=lib).reshape(5, 5)
    want = np.zeros((5, 5), np.int32)
    want[0, 0] = want[0, 4] = want[4, 0] = want[4, 4] = -1
    assert np.array_equal(lab, want)
    # eps just below the spacing: all isolated
    assert (oracle.dbscan(g, k - 1e-9, 2, lib=lib) == -1).all()
    # the same lattice shifted along x only separates <= from < on dimension 0
    line = np.array([(i * k, 0) for i in range(6)], np.int32)
    assert (oracle.dbscan(line, float(k), 2, lib=lib) == 0).all()
    assert (oracle.dbscan(line, float(k), 3, lib=lib) == 0).all()
    # duplicates count separately: 3 copies of one point with minPts = 3
    dup = np.array([[5, 5]] * 3 + [[100, 100]], np.int32)
    assert oracle.dbscan(dup, 0.5, 3, lib=lib).tolist() == [0, 0, 0, -1]


def pin_invariances(lib):
    rng = np.random.default_rng(19)
    for d in (2, 4, 8):
        x = make_blobs(rng, 600, d, 4, 0.05, 0.1)
        pts = quantise(x, 8)
        eps, mp = 0.08 * 2 ** 8, 5
        base = oracle.dbscan(pts, eps, mp, lib=lib)
        shift = rng.integers(-10_000, 10_000, size=d).astype(np.int32)
        assert np.array_equal(oracle.dbscan(pts + shift, eps, mp, lib=lib), base)
        assert np.array_equal(oracle.dbscan(pts * 4, eps * 4, mp, lib=lib), base)
    # axes permuted and constant axes added change no distance
    x = make_blobs(rng, 500, 6, 4, 0.04, 0.1)
    pts = quantise(x, 8)
    eps, mp = 0.07 * 2 ** 8, 4
    base = oracle.dbscan(pts, eps, mp, lib=lib)
    pad = np.concatenate([pts, np.full((500, 48), 77, np.int32)], axis=1)
    perm = rng.permutation(54)
    assert np.array_equal(oracle.dbscan(np.ascontiguousarray(pad[:, perm]), eps, mp, lib=lib), base)


def pin_representative_faces(lib):
    """The grid part's representative-only merge (the paper's merge as printed)
    on hand-derived cases: the facing rule (sign of the offset against its
    opposite) along an axis, on a diagonal and on a knight offset, the ideal
    position on the upper face for +1 and the lower face for -1, and ties
    kept by the first point (Algorithm 2; Depth First Search paragraph)."""
    g = json.loads((GOLDEN / "representative_faces.json").read_text())
    for case in g["cases"]:
        pts = np.array(case["points"], np.int32)
        got = oracle.hca_grid(pts, case["eps"], case["min_pts"], rep_mode=1, lib=lib)
        assert got.tolist() == case["rep_only_labels"], case["name"]
        for mode in (0, 2):
            got = oracle.hca_grid(pts, case["eps"], case["min_pts"], rep_mode=mode, lib=lib)
            assert got.tolist() == case["labels"], (case["name"], mode)
    split = json.loads((GOLDEN / "representative_split.json").read_text())
    c = split["cases"][0]
    pts = np.array(split["points"], np.int32)
    assert oracle.hca_grid(pts, c["eps"], c["min_pts"], rep_mode=1, lib=lib).tolist() == c["rep_only_labels"]


PINS = [pin_eps2_rational, pin_golden, pin_closed_form_1d, pin_sklearn, pin_scipy_min_pts_1,
        pin_expand_cluster, pin_special_cases, pin_invariances, pin_representative_faces]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(None)


N_MUTANTS = 14


def test_planted_mistakes_are_caught(tmp_path):
    """Each planted mistake in a copy of the oracle must fail at least one pin."""
    survivors = []
    for k in range(1, N_MUTANTS + 1):
        so = oracle.build(out=tmp_path / f"mut{k}.so", mutant=k)
        lib = oracle.load_variant(so)
        caught = False
        for pin in PINS:
            try:
                pin(lib)
            except (AssertionError, ValueError):
                caught = True
                break
        if not caught:
            survivors.append(k)
    assert not survivors, f"mutants not caught by any pin: {survivors}"


# --------------------------------------------------------------------------
# the two oracle parts against each other, and the grid geometry
# --------------------------------------------------------------------------
def test_grid_part_matches_definition_random():
    rng = np.random.default_rng(23)
    for trial in range(120):
        d = int(rng.integers(1, 9))
        n = int(rng.integers(0, 400))
        pts = rand_points(rng, n, d, int(rng.integers(2, 60)), 0.1)
        eps = float(rng.uniform(0.5, 25.0))
        mp = int(rng.integers(1, 9))
        want = oracle.dbscan(pts, eps, mp)
        for mode in (0, 2):
            got = oracle.hca_grid(pts, eps, mp, rep_mode=mode)
            assert np.array_equal(got, want), (trial, d, n, eps, mp, mode)


def test_representative_only_refines_exact():
    """Representative-only merging joins two cubes only when two of their core
    points are within eps, so it can split exact clusters but never join two:
    core and noise points are the same, every representative-only cluster of
    core points lies inside one exact cluster, and on 1-D data (one facing
    pair per cube pair: the last point of the left cube, the first of the
    right) it equals the exact result whenever the cubes hold one point."""
    rng = np.random.default_rng(31)
    for trial in range(80):
        d = int(rng.integers(1, 5))
        n = int(rng.integers(1, 300))
        pts = rand_points(rng, n, d, int(rng.integers(2, 60)), 0.1)
        eps = float(rng.uniform(0.5, 25.0))
        mp = int(rng.integers(1, 6))
        exact, core_e, _ = oracle.hca_grid(pts, eps, mp, details=True)
        approx, core_a, _ = oracle.hca_grid(pts, eps, mp, rep_mode=1, details=True)
        assert np.array_equal(core_e, core_a)
        assert np.array_equal(exact < 0, approx < 0), trial
        where = {}
        for i in np.flatnonzero(core_a):
            assert where.setdefault(int(approx[i]), int(exact[i])) == int(exact[i]), trial
    # 1-D, minPts = 1, cube side s = floor(sqrt(eps2)): every point is core and
    # sits alone in its cube when points are spaced at least s apart; then the
    # facing representatives are the points themselves
    for trial in range(20):
        eps = float(rng.uniform(3.0, 20.0))
        s = oracle.grid_geometry(eps, 1)[0]
        x = np.cumsum(rng.integers(s, 2 * s + 10, size=60)).reshape(-1, 1).astype(np.int32)
        x = x[rng.permutation(60)]
        want = oracle.dbscan(x, eps, 1)
        assert np.array_equal(oracle.hca_grid(x, eps, 1, rep_mode=1), want), trial


def test_grid_part_matches_definition_small_workload():
    w = make_config(1)
    want = oracle.dbscan(w.points, w.eps, w.min_pts)
    got, core, stats = oracle.hca_grid(w.points, w.eps, w.min_pts, details=True)
    assert np.array_equal(got, want)
    _, counts, _ = oracle.dbscan(w.points, w.eps, w.min_pts, details=True)
    assert np.array_equal(core, counts >= w.min_pts)
    assert stats["cubes"] > 0 and stats["rep_accepts"] > 0


def test_representative_only_merge_is_not_exact():
    g = json.loads((GOLDEN / "representative_split.json").read_text())
    c = g["cases"][0]
    pts = np.array(g["points"], np.int32)
    assert oracle.hca_grid(pts, c["eps"], c["min_pts"], rep_mode=0).tolist() == c["labels"]
    assert oracle.hca_grid(pts, c["eps"], c["min_pts"], rep_mode=1).tolist() == c["rep_only_labels"]


def test_paper_neighbourhood_counts():
    g = json.loads((GOLDEN / "grid_neighbourhood.json").read_text())
    for eps in g["eps_values_2d"]:
        assert oracle.stencil_size(eps, 2) == g["neighbours_2d"], eps
    # brute force: count the cube offsets whose closest pair of integer points
    # (enumerated per axis, the squared distance being separable) is within
    # eps; offsets up to R + 1 are enumerated so that a too-small R shows up.
    for eps, d in [(5.5, 3), (9.0, 2), (4.2, 4), (3.0, 1), (12.5, 2)]:
        s, R = oracle.grid_geometry(eps, d)
        e2 = rational_eps2(eps)
        axis_min = {}
        for o in range(-(R + 1), R + 2):
            axis_min[o] = min((x - y) ** 2 for x in range(s) for y in range(o * s, o * s + s))
        count = 0
        for off in np.ndindex(*([2 * R + 3] * d)):
            o = [v - (R + 1) for v in off]
            if any(o) and sum(axis_min[v] for v in o) <= e2:
                count += 1
                assert max(abs(v) for v in o) <= R
        assert oracle.stencil_size(eps, d) == count, (eps, d)


def test_same_cube_points_within_eps():
    """The hypercube side keeps every pair of points of one cube within eps."""
    rng = np.random.default_rng(29)
    for d in range(1, 9):
        for eps in rng.uniform(1.0, 500.0, 20):
            s, _ = oracle.grid_geometry(eps, d)
            assert d * (s - 1) ** 2 <= rational_eps2(eps)


def test_domain_errors():
    pts = np.array([[0, 0], [1 << 30, 0]], np.int32)
    with pytest.raises(ValueError):
        oracle.dbscan(pts, 1.0, 1)
    with pytest.raises(ValueError):
        oracle.dbscan(np.zeros((3, 65), np.int32), 1.0, 1)
    # d > 8: the sum of squared spans must stay below 2^63
    wide = np.zeros((2, 9), np.int32)
    wide[1] = (1 << 30) - 1
    with pytest.raises(ValueError):
        oracle.dbscan(wide, 1.0, 1)
    wide[1, :8] = (1 << 30) - 1
    wide[1, 8] = 0
    assert oracle.dbscan(wide, 1.0, 1).tolist() == [0, 1]
    with pytest.raises(ValueError):
        oracle.dbscan(np.zeros((3, 2), np.int32), 0.0, 1)
    with pytest.raises(ValueError):
        oracle.dbscan(np.zeros((3, 2), np.int32), 1.0, 0)
    assert oracle.dbscan(np.zeros((0, 2), np.int32), 1.0, 1).shape == (0,)
    ok = np.array([[0, 0], [(1 << 30) - 1, 0]], np.int32)
    assert oracle.dbscan(ok, 1.0, 1).tolist() == [0, 1]
