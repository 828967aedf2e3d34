"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and its host-only logic (exact eps^2, grid geometry, argument checks) agrees
with exact arithmetic, the oracle's independent geometry and the paper."""
from __future__ import annotations

import ctypes
import json
import math
import re
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest

import oracle
from paper_1912_00323_amd import hca

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib():
    if not hca.LIB_PATH.exists():
        from paper_1912_00323_amd import build
        build.build()
    return hca.load_library()


def declared_functions():
    src = (ROOT / "include" / "hca.h").read_text()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hca_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name


def test_exact_eps2_rational(lib):
    rng = np.random.default_rng(1)
    vals = [81.92, 262.144, 245.76, 14.15, 1.0, 0.5, 2.0 ** -1074, 1e300, 46340.95]
    vals += list(rng.uniform(0.1, 1e6, 300)) + list(np.exp(rng.uniform(-30, 40, 300)))
    for v in vals:
        want = min(math.floor(Fraction(float(v)) ** 2), 2 ** 63 - 1)
        assert hca.exact_eps2(v) == want, v
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(hca.HcaError):
            hca.exact_eps2(bad)


def test_geometry_matches_oracle_and_paper(lib):
    g = json.loads((ROOT / "tests" / "golden" / "grid_neighbourhood.json").read_text())
    for eps in g["eps_values_2d"]:
        assert hca.geometry(eps, 2)["stencil"] == g["neighbours_2d"]
    for d in range(1, 5):
        assert hca.geometry(81.92, d)["reps"] == g["representatives"][str(d)]
    rng = np.random.default_rng(2)
    for _ in range(60):
        d = int(rng.integers(1, 9))
        eps = float(np.exp(rng.uniform(0, 8)))
        geo = hca.geometry(eps, d)
        s, r = oracle.grid_geometry(eps, d)
        assert (geo["side"], geo["radius"]) == (s, r), (eps, d)
        if (2 * r + 1) ** d <= 200_000:
            assert geo["stencil"] == oracle.stencil_size(eps, d), (eps, d)


def test_geometry_of_the_workloads(lib):
    assert hca.geometry(0.02 * 2 ** 12, 2) | {} == hca.geometry(81.92, 2)
    g2 = hca.geometry(0.004 * 2 ** 16, 2)
    assert (g2["eps2"], g2["side"], g2["radius"], g2["stencil"], g2["group"]) == (68719, 185, 2, 20, 1)
    g8 = hca.geometry(0.06 * 2 ** 12, 8)
    assert (g8["eps2"], g8["side"], g8["radius"]) == (60397, 86, 3)
    assert g8["stencil"] == oracle.stencil_size(0.06 * 2 ** 12, 8) == 1601696
    assert g8["group"] == 3 and g8["group_stencil"] == 3 ** 8 and g8["reps"] == 0


def test_argument_checks_without_device(lib):
    null = ctypes.c_void_p()
    assert lib.hca_cluster(null, None, 10, 2, 1.0, 1, None) == hca.HCA_E_INVAL
    assert lib.hca_cluster_ex(null, None, 10, 2, 1.0, 1, None, None, None) == hca.HCA_E_INVAL
    assert lib.hca_cluster_host(null, None, 10, 2, 1.0, 1, None) == hca.HCA_E_INVAL
    assert lib.hca_set_stream(null, None) == hca.HCA_E_INVAL
    assert lib.hca_last_error(null) == b""
    lib.hca_destroy(null)
    assert lib.hca_create(None, 0) == hca.HCA_E_INVAL
    geo = hca.Geometry()
    assert lib.hca_get_geometry(1.0, 0, ctypes.byref(geo)) == hca.HCA_E_INVAL
    assert lib.hca_get_geometry(1.0, 65, ctypes.byref(geo)) == hca.HCA_E_INVAL
    assert lib.hca_get_geometry(-1.0, 2, ctypes.byref(geo)) == hca.HCA_E_INVAL


def test_geometry_many_axes(lib):
    """d > 8: cube side floor(sqrt(floor(eps^2 / d))) (space diagonal at most
    eps, Overlaying Hypercubes), groups of ceil(sqrt(eps2) / side) cubes so
    their side reaches eps, no enumerable stencil."""
    geo = hca.Geometry()
    for d in (9, 16, 27, 54, 64):
        for eps in (0.5, 1.0, 7.3, 61.44, 245.76, 4096.0, 123456.7):
            assert lib.hca_get_geometry(eps, d, ctypes.byref(geo)) == hca.HCA_OK
            e2 = math.floor(Fraction(eps) ** 2)
            side = max(1, math.isqrt(e2 // d))
            assert geo.eps2 == e2 and geo.side == side
            assert d * side * side <= max(e2, d)
            assert geo.group == max(1, -(-math.isqrt(e2) // side))
            assert geo.group * side >= math.isqrt(e2)
            assert geo.stencil == -1 and geo.group_stencil == -1 and geo.reps == 0


def test_no_cpu_fallback_in_binding():
    """The product binding never imports the oracle."""
    src = (ROOT / "paper_1912_00323_amd" / "hca.py").read_text()
    assert "oracle" not in src
    for f in (ROOT / "paper_1912_00323_amd" / "csrc").glob("*.*"):
        if f.is_file():
            assert "oracle" not in f.read_text(errors="ignore"), f


def test_bench_disagreement_measure():
    """The label-disagreement figure the bench reports for the approximate
    merge: points outside the largest fragment of their exact cluster."""
    import sys
    sys.path.insert(0, str(Path(__file__).resolve().parents[1]))
    import bench
    e = np.array([0, 0, 0, 1, 1, -1, 2, 2, 3])
    a = np.array([0, 0, 1, 2, 2, -1, 3, 4, 5])
    r = bench.disagreement(e, a)
    assert r["points_differing"] == 2 and r["exact_clusters_split"] == 2
    assert r["clusters_exact"] == 4 and r["clusters_approx"] == 6 and r["noise_differing"] == 0
    assert bench.disagreement(e, e)["points_differing"] == 0
    # the fixture on which representatives alone split a cluster
    g = json.loads((Path(__file__).parent / "golden" / "representative_split.json").read_text())
    pts = np.array(g["points"], np.int32)
    exact = oracle.dbscan(pts, 14.15, 1)
    approx = oracle.hca_grid(pts, 14.15, 1, rep_mode=1)
    assert bench.disagreement(exact, approx)["points_differing"] == 1


def test_label_tensor_checks():
    """Label arrays the library writes are checked before any C call: CUDA,
    int32, on the points' device, contiguous and exactly n elements."""
    import torch

    class FakeCuda:                     # stands in for a CUDA tensor on a GPU-less host
        is_cuda = True

        def __init__(self, n, dtype=torch.int32, device="cuda:0", contiguous=True):
            self.dtype, self.device, self._n, self._c = dtype, torch.device(device), n, contiguous

        def is_contiguous(self):
            return self._c

        def numel(self):
            return self._n

    dev = torch.device("cuda:0")
    hca.check_labels(FakeCuda(10), 10, dev)
    with pytest.raises(TypeError):
        hca.check_labels(torch.zeros(10, dtype=torch.int32), 10, dev)       # host tensor
    with pytest.raises(TypeError):
        hca.check_labels(FakeCuda(10, dtype=torch.int64), 10, dev)
    with pytest.raises(ValueError):
        hca.check_labels(FakeCuda(9), 10, dev)
    with pytest.raises(ValueError):
        hca.check_labels(FakeCuda(11), 10, dev)
    with pytest.raises(ValueError):
        hca.check_labels(FakeCuda(10, contiguous=False), 10, dev)
    with pytest.raises(ValueError):
        hca.check_labels(FakeCuda(10, device="cuda:1"), 10, dev)
