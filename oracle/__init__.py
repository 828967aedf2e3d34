"""CPU oracle for exact DBSCAN -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and the two share no
code: this side is plain C (``dbscan_def.c``: the DBSCAN definition written
out; ``hca_grid.c``: the paper's hypercube method run sequentially with an
exact fallback), built with gcc into ``liboracle.so`` and loaded by ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SO = _HERE / "liboracle.so"
_SOURCES = ["dbscan_def.c", "hca_grid.c"]
_lib = None

ERRORS = {1: "invalid argument", 2: "coordinate span out of range", 3: "out of memory"}


def build(force: bool = True, out: Path | None = None, mutant: int = 0) -> Path:
    """Compile the C oracle with gcc (-O2, OpenMP) into ``oracle/liboracle.so``.

    ``mutant`` > 0 builds a copy with one planted mistake (into ``out``), used
    only by the test that checks that the pins catch it."""
    so = Path(out) if out is not None else _SO
    if not force and so.exists():
        return so
    tmp = so.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-Wall",
           f"-DORACLE_MUTANT={int(mutant)}",
           *[str(_HERE / s) for s in _SOURCES], "-o", str(tmp), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, so)
    return so


def _load():
    global _lib
    if _lib is None:
        if not _SO.exists():
            build()
        _lib = _bind(ctypes.CDLL(str(_SO)))
    return _lib


def load_variant(path) -> ctypes.CDLL:
    """Load another build of the oracle (see ``build(mutant=...)``); pass the
    handle as ``lib=`` to the functions below."""
    return _bind(ctypes.CDLL(str(path)))


def _bind(lib):
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_exact_eps2.argtypes = [ctypes.c_double, i64p]
    lib.oracle_dbscan.argtypes = [i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32]
    lib.oracle_hca_grid.argtypes = [i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_int32, i32p, i32p, i64p,
                                    ctypes.c_int32]
    lib.oracle_grid_geometry.argtypes = [ctypes.c_double, ctypes.c_int32, i64p, i64p]
    lib.oracle_stencil_size.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int64, i64p]
    return lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t)) if a is not None else None


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle error {rc}: {ERRORS.get(rc, 'unknown')}")


def _points(points):
    p = np.ascontiguousarray(points, dtype=np.int32)
    if p.ndim != 2:
        raise ValueError("points must be a 2-D [n, d] array")
    return p


def exact_eps2(eps: float, lib=None) -> int:
    """floor(eps**2), computed exactly from the binary value of ``eps``."""
    out = ctypes.c_int64()
    _check((lib or _load()).oracle_exact_eps2(float(eps), ctypes.byref(out)))
    return int(out.value)


def grid_geometry(eps: float, d: int) -> tuple[int, int]:
    """(cube side s, neighbour radius R) of the integer hypercube grid."""
    s, r = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().oracle_grid_geometry(float(eps), int(d), ctypes.byref(s), ctypes.byref(r)))
    return int(s.value), int(r.value)


def stencil_size(eps: float, d: int, max_count: int = 50_000_000) -> int:
    """Number of neighbour cube offsets of the integer hypercube grid."""
    out = ctypes.c_int64()
    _check(_load().oracle_stencil_size(float(eps), int(d), int(max_count), ctypes.byref(out)))
    return int(out.value)


def dbscan(points, eps: float, min_pts: int, threads: int = 0, details: bool = False,
           lib=None):
    """Exact DBSCAN from the definition.  Returns int32 labels (-1 noise),
    canonical (clusters ranked by smallest member index).  With ``details`` also
    returns (counts |N(i)|, owner index of each border point or -1)."""
    p = _points(points)
    n, d = p.shape
    labels = np.empty(n, np.int32)
    counts = np.empty(n, np.int32) if details else None
    owner = np.empty(n, np.int32) if details else None
    _check((lib or _load()).oracle_dbscan(_ptr(p, ctypes.c_int32), n, d, float(eps), int(min_pts),
                                 _ptr(labels, ctypes.c_int32), _ptr(counts, ctypes.c_int32),
                                 _ptr(owner, ctypes.c_int32), int(threads)))
    if details:
        return labels, counts, owner
    return labels


def hca_grid(points, eps: float, min_pts: int, rep_mode: int = 0, threads: int = 1,
             details: bool = False, lib=None):
    """The paper's hypercube method on the CPU (exact unless ``rep_mode == 1``).
    Returns int32 canonical labels; with ``details`` also (core flags, stats dict)."""
    p = _points(points)
    n, d = p.shape
    labels = np.empty(n, np.int32)
    core = np.empty(n, np.int32)
    stats = np.zeros(8, np.int64)
    _check((lib or _load()).oracle_hca_grid(_ptr(p, ctypes.c_int32), n, d, float(eps), int(min_pts),
                                   int(rep_mode), _ptr(labels, ctypes.c_int32),
                                   _ptr(core, ctypes.c_int32), _ptr(stats, ctypes.c_int64),
                                   int(threads)))
    if details:
        keys = ["cubes", "core_cubes", "dense_cubes", "core_points", "rep_accepts",
                "exact_accepts", "exact_rejects", "pair_tests"]
        return labels, core.astype(bool), dict(zip(keys, stats.tolist()))
    return labels
