"""Python binding of libhca.so (ctypes).  Argument marshalling only: every step
of the clustering runs in the library's HIP kernels.  There is no CPU path; if
the library is missing or no GPU is usable, calls raise.

Names follow the C ABI in ``include/hca.h``.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libhca.so"

HCA_OK, HCA_E_INVAL, HCA_E_RANGE, HCA_E_NOMEM, HCA_E_DEVICE = 0, 1, 2, 3, 4
PHASES = ["bbox", "sort", "cells", "lists", "core", "reps", "intra", "merge", "border", "labels"]
STATUS_NAMES = {0: "HCA_OK", 1: "HCA_E_INVAL", 2: "HCA_E_RANGE", 3: "HCA_E_NOMEM",
                4: "HCA_E_DEVICE"}


class HcaError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class Geometry(ctypes.Structure):
    _fields_ = [("eps2", ctypes.c_int64), ("side", ctypes.c_int64), ("radius", ctypes.c_int32),
                ("group", ctypes.c_int32), ("stencil", ctypes.c_int64),
                ("group_stencil", ctypes.c_int64), ("reps", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Stats(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_core_points", ctypes.c_int64), ("n_clusters", ctypes.c_int64),
                ("n_noise", ctypes.c_int64), ("exact_pairs", ctypes.c_int64),
                ("key_bits", ctypes.c_int32), ("sort_passes", ctypes.c_int32),
                ("group", ctypes.c_int32), ("wide", ctypes.c_int32),
                ("dense_table", ctypes.c_int32), ("list_overflow", ctypes.c_int32),
                ("tests_core", ctypes.c_int64), ("tests_merge", ctypes.c_int64),
                ("tests_border", ctypes.c_int64), ("tests_intra", ctypes.c_int64),
                ("packed_rows", ctypes.c_int32), ("key_axes", ctypes.c_int32),
                ("core_rest", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def load_library(path: str | Path | None = None) -> ctypes.CDLL:
    """Load libhca.so (built in-tree by ``paper_1912_00323_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path is not None else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1912_00323_amd.build`")
    lib = ctypes.CDLL(str(p))
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.hca_exact_eps2.argtypes = [dbl, ctypes.POINTER(i64)]
    lib.hca_exact_eps2.restype = ctypes.c_int
    lib.hca_get_geometry.argtypes = [dbl, i32, ctypes.POINTER(Geometry)]
    lib.hca_get_geometry.restype = ctypes.c_int
    lib.hca_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.hca_create.restype = ctypes.c_int
    lib.hca_destroy.argtypes = [vp]
    lib.hca_destroy.restype = None
    lib.hca_last_error.argtypes = [vp]
    lib.hca_last_error.restype = ctypes.c_char_p
    lib.hca_set_stream.argtypes = [vp, vp]
    lib.hca_set_stream.restype = ctypes.c_int
    lib.hca_set_plan_reuse.argtypes = [vp, i32]
    lib.hca_set_plan_reuse.restype = ctypes.c_int
    lib.hca_plan_reuse_counts.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.hca_plan_reuse_counts.restype = ctypes.c_int
    lib.hca_cluster.argtypes = [vp, vp, i64, i32, dbl, i32, vp]
    lib.hca_cluster.restype = ctypes.c_int
    lib.hca_cluster_noalloc.argtypes = [vp, vp, i64, i32, dbl, i32, vp]
    lib.hca_cluster_noalloc.restype = ctypes.c_int
    lib.hca_batch_create.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp]
    lib.hca_batch_create.restype = ctypes.c_int
    lib.hca_batch_run.argtypes = [vp, vp, vp]
    lib.hca_batch_run.restype = ctypes.c_int
    lib.hca_batch_stats.argtypes = [vp, vp, vp, i32]
    lib.hca_batch_stats.restype = ctypes.c_int
    lib.hca_batch_destroy.argtypes = [vp]
    lib.hca_batch_destroy.restype = None
    lib.hca_cluster_ex.argtypes = [vp, vp, i64, i32, dbl, i32, vp, vp, ctypes.POINTER(Stats)]
    lib.hca_cluster_ex.restype = ctypes.c_int
    lib.hca_cluster_host.argtypes = [vp, vp, i64, i32, dbl, i32, vp]
    lib.hca_cluster_host.restype = ctypes.c_int
    lib.hca_cluster_batch.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    lib.hca_cluster_batch.restype = ctypes.c_int
    lib.hca_cluster_sets.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.hca_cluster_sets.restype = ctypes.c_int
    lib.hca_server_create.argtypes = [ctypes.POINTER(vp), i32, i32, i64, i32]
    lib.hca_server_create.restype = ctypes.c_int
    lib.hca_server_submit.argtypes = [vp, vp, i64, i32, dbl, i32, vp, ctypes.c_uint64, vp]
    lib.hca_server_submit.restype = ctypes.c_int
    lib.hca_server_set_batch_time.argtypes = [vp, dbl]
    lib.hca_server_set_batch_time.restype = ctypes.c_int
    lib.hca_server_poll.argtypes = [vp, vp, vp, vp, i32]
    lib.hca_server_poll.restype = i32
    lib.hca_server_drain.argtypes = [vp]
    lib.hca_server_drain.restype = ctypes.c_int
    lib.hca_server_destroy.argtypes = [vp]
    lib.hca_server_destroy.restype = None
    lib.hca_clock.argtypes = []
    lib.hca_clock.restype = dbl
    lib.hca_set_exact.argtypes = [vp, i32]
    lib.hca_set_exact.restype = ctypes.c_int
    lib.hca_set_profiling.argtypes = [vp, i32]
    lib.hca_set_profiling.restype = ctypes.c_int
    lib.hca_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    lib.hca_phase_times.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


class BatchInfo(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_int64), ("graph_replays", ctypes.c_int64), ("plans", ctypes.c_int64),
                ("groups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchGroupInfo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("sets", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("key_bits", ctypes.c_int32), ("sort_passes", ctypes.c_int32), ("wide", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("lanes", ctypes.c_int32), ("prefix", ctypes.c_int32),
                ("wave_blocks", ctypes.c_int32), ("hash_load", ctypes.c_int32), ("digit_cap", ctypes.c_int32),
                ("sort_items", ctypes.c_int32), ("tuned", ctypes.c_int32), ("lists", ctypes.c_int32),
                ("merge_split", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tuned_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Batch:
    """A batch handle (hca_batch_*): batches of one fixed shape, the first run
    planned, tuned and captured in a HIP graph, every later run one graph
    launch.  tune: 0 default knobs, 1 cache then tune, 2 always tune."""

    def __init__(self, ctx: "Context", rows, dims, eps, min_pts, tune: int = 1):
        self._lib = ctx._lib
        self._ctx = ctx
        self.rows = [int(r) for r in rows]
        self.dims = [int(d) for d in dims]
        r = np.ascontiguousarray(self.rows, dtype=np.int64)
        dm = np.ascontiguousarray(self.dims, dtype=np.int32)
        ep = np.ascontiguousarray(eps, dtype=np.float64)
        mp = np.ascontiguousarray(min_pts, dtype=np.int32)
        if not (len(r) == len(dm) == len(ep) == len(mp)):
            raise ValueError("rows, dims, eps and min_pts must have one entry per data set")
        self._h = ctypes.c_void_p()
        ctx._check(self._lib.hca_batch_create(ctx._ctx, len(r), r.ctypes.data_as(ctypes.c_void_p),
                                              dm.ctypes.data_as(ctypes.c_void_p),
                                              ep.ctypes.data_as(ctypes.c_void_p),
                                              mp.ctypes.data_as(ctypes.c_void_p), int(tune), ctypes.byref(self._h)))

    def run(self, points, labels):
        """Cluster one batch: points[i] a contiguous CUDA int32 tensor
        [rows[i], dims[i]], labels[i] a CUDA int32 tensor of rows[i]."""
        import torch
        n = len(self.rows)
        if len(points) != n or len(labels) != n:
            raise ValueError(f"{n} data sets expected")
        for i, (p, o) in enumerate(zip(points, labels)):
            if not (isinstance(p, torch.Tensor) and p.is_cuda and p.dtype == torch.int32 and p.is_contiguous()
                    and p.numel() == self.rows[i] * self.dims[i]):
                raise TypeError(f"points[{i}] must be a contiguous CUDA int32 tensor of {self.rows[i]} x "
                                f"{self.dims[i]}")
            check_labels(o, self.rows[i], p.device, f"labels[{i}]")
        pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in points])
        ll = (ctypes.c_void_p * n)(*[o.data_ptr() for o in labels])
        self._ctx.set_stream(torch.cuda.current_stream(points[0].device).cuda_stream)
        self._ctx._check(self._lib.hca_batch_run(self._h, pp, ll))

    def stats(self) -> dict:
        info = BatchInfo()
        groups = (BatchGroupInfo * 8)()
        self._ctx._check(self._lib.hca_batch_stats(self._h, ctypes.byref(info), groups, 8))
        return {"runs": info.runs, "graph_replays": info.graph_replays, "plans": info.plans,
                "groups": [groups[i].as_dict() for i in range(info.groups)]}

    def close(self):
        if self._h:
            self._lib.hca_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_labels(t, n: int, device, what: str = "out"):
    """A label array the library will write: a contiguous int32 CUDA tensor of
    exactly n elements on the points' device (raises TypeError / ValueError)."""
    import torch
    if not getattr(t, "is_cuda", False) or getattr(t, "dtype", None) != torch.int32:
        raise TypeError(f"{what} must be a CUDA int32 tensor")
    if t.device != device:
        raise ValueError(f"{what} is on {t.device}, the points on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} elements, {n} are needed")


def clock() -> float:
    """Seconds of the steady clock the server stamps completions with."""
    return float(load_library().hca_clock())


class Server:
    """The served form (hca_server_*): submit requests on device tensors,
    poll completions.  Keep every submitted tensor alive until its request
    completes."""

    def __init__(self, device: int = 0, workers: int = 2, budget_bytes: int = 32 << 30,
                 max_batch: int = 64, batch_ms: float | None = None):
        self._lib = load_library()
        self._srv = ctypes.c_void_p()
        st = self._lib.hca_server_create(ctypes.byref(self._srv), int(device), int(workers),
                                         int(budget_bytes), int(max_batch))
        if st != HCA_OK:
            raise HcaError(st, "hca_server_create failed")
        self._keep = {}
        if batch_ms is not None:
            st = self._lib.hca_server_set_batch_time(self._srv, float(batch_ms))
            if st != HCA_OK:
                raise HcaError(st, "batch_ms must be > 0")

    def submit(self, points, eps: float, min_pts: int, labels, tag: int):
        """Queue one request.  It runs after the work already queued on the
        current torch stream of the points' device (so tensors written or
        filled there are ready); its labels are final once poll() returns its
        tag."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.int32
                and points.dim() == 2 and points.is_contiguous()):
            raise TypeError("points must be a contiguous CUDA int32 tensor [n, d]")
        n, d = points.shape
        check_labels(labels, n, points.device, "labels")
        stream = torch.cuda.current_stream(points.device).cuda_stream
        self._keep[int(tag)] = (points, labels)
        st = self._lib.hca_server_submit(self._srv, ctypes.c_void_p(points.data_ptr()), n, d, float(eps),
                                         int(min_pts), ctypes.c_void_p(labels.data_ptr()), int(tag),
                                         ctypes.c_void_p(stream))
        if st != HCA_OK:
            self._keep.pop(int(tag), None)
            raise HcaError(st, "hca_server_submit failed")

    def poll(self, max_items: int = 4096):
        """Completed requests: list of (tag, status, t_done)."""
        tags = (ctypes.c_uint64 * max_items)()
        status = (ctypes.c_int32 * max_items)()
        tdone = (ctypes.c_double * max_items)()
        k = self._lib.hca_server_poll(self._srv, tags, status, tdone, max_items)
        out = [(int(tags[i]), int(status[i]), float(tdone[i])) for i in range(k)]
        for t, _, _ in out:
            self._keep.pop(t, None)
        return out

    def drain(self):
        self._lib.hca_server_drain(self._srv)

    def close(self):
        if self._srv:
            self._lib.hca_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exact_eps2(eps: float) -> int:
    out = ctypes.c_int64()
    st = load_library().hca_exact_eps2(float(eps), ctypes.byref(out))
    if st != HCA_OK:
        raise HcaError(st, "eps must be finite and > 0")
    return int(out.value)


def geometry(eps: float, d: int) -> dict:
    g = Geometry()
    st = load_library().hca_get_geometry(float(eps), int(d), ctypes.byref(g))
    if st != HCA_OK:
        raise HcaError(st, "bad eps or d")
    return g.as_dict()


class Context:
    """One hca_ctx on a HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        self._ctx = ctypes.c_void_p()
        st = self._lib.hca_create(ctypes.byref(self._ctx), int(device))
        if st != HCA_OK:
            raise HcaError(st, f"hca_create(device={device}) failed")
        self.device = device

    def close(self):
        if self._ctx:
            self._lib.hca_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != HCA_OK:
            msg = self._lib.hca_last_error(self._ctx)
            raise HcaError(st, msg.decode() if msg else "")

    def set_stream(self, stream_handle: int | None):
        self._check(self._lib.hca_set_stream(self._ctx, ctypes.c_void_p(stream_handle or 0)))

    def set_exact(self, exact: bool):
        """True (default): exact DBSCAN.  False: the paper's merge on facing
        representatives alone (approximate; cubes as search groups, d <= 4)."""
        self._check(self._lib.hca_set_exact(self._ctx, 1 if exact else 0))

    def set_plan_reuse(self, on: bool):
        """True (default): a call whose shape and bounding box repeat those of
        the previous calls is launched without waiting for its own box (which
        is still checked on the device; a differing box runs the call again)."""
        self._check(self._lib.hca_set_plan_reuse(self._ctx, 1 if on else 0))

    def plan_reuse_counts(self) -> tuple:
        """(calls planned ahead, of which ran again) on this context."""
        calls, reruns = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.hca_plan_reuse_counts(self._ctx, ctypes.byref(calls), ctypes.byref(reruns)))
        return calls.value, reruns.value

    def set_profiling(self, phase: int | str | None):
        """Time later calls with HIP events: None = off, "all", or one phase."""
        code = -1 if phase is None else -2 if phase == "all" else (
            PHASES.index(phase) if isinstance(phase, str) else int(phase))
        self._check(self._lib.hca_set_profiling(self._ctx, code))

    def phase_times(self) -> dict:
        """Milliseconds per phase of the last call (timed phases only)."""
        buf = (ctypes.c_float * len(PHASES))()
        self._check(self._lib.hca_phase_times(self._ctx, buf, len(PHASES)))
        return {name: float(buf[i]) for i, name in enumerate(PHASES)}

    def phase_time(self, index: int) -> float:
        """Milliseconds of phase PHASES[index] in the last call (0 when not
        timed), through a buffer kept by the context: cheap enough to call
        after every call of a timed loop."""
        buf = getattr(self, "_phase_buf", None)
        if buf is None:
            buf = self._phase_buf = (ctypes.c_float * len(PHASES))()
        self._check(self._lib.hca_phase_times(self._ctx, buf, len(PHASES)))
        return float(buf[index])

    def cluster(self, points, eps: float, min_pts: int, core: bool = False, stats: bool = False,
                out=None):
        """Cluster a CUDA int32 tensor [n, d].  Returns an int32 tensor of labels
        (and, if asked, a uint8 core-flag tensor and a stats dict).  Runs on the
        current torch stream and blocks until done."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda):
            raise TypeError("points must be a CUDA (HIP) torch tensor")
        if points.dtype != torch.int32 or points.dim() != 2:
            raise TypeError("points must be int32 with shape [n, d]")
        pts = points.contiguous()
        n, d = pts.shape
        if out is not None:
            check_labels(out, n, pts.device)
        labels = out if out is not None else torch.empty(n, dtype=torch.int32, device=pts.device)
        core_t = torch.empty(n, dtype=torch.uint8, device=pts.device) if core else None
        st_obj = Stats() if stats else None
        self.set_stream(torch.cuda.current_stream(pts.device).cuda_stream)
        st = self._lib.hca_cluster_ex(self._ctx, ctypes.c_void_p(pts.data_ptr()), n, d, float(eps),
                                      int(min_pts), ctypes.c_void_p(labels.data_ptr()),
                                      ctypes.c_void_p(core_t.data_ptr()) if core else None,
                                      ctypes.byref(st_obj) if stats else None)
        self._check(st)
        res = [labels]
        if core:
            res.append(core_t)
        if stats:
            res.append(st_obj.as_dict())
        return res[0] if len(res) == 1 else tuple(res)

    def prepared(self, points, eps: float, min_pts: int, out):
        """A repeated call on fixed tensors: the arguments are checked and
        marshalled once, on the current torch stream, and the returned function
        calls hca_cluster with them (blocking; raises HcaError on failure).  The
        tensors must stay alive and in place while it is used."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.is_contiguous()):
            raise TypeError("points must be a contiguous CUDA (HIP) torch tensor")
        if points.dtype != torch.int32 or points.dim() != 2:
            raise TypeError("points must be int32 with shape [n, d]")
        n, d = points.shape
        check_labels(out, n, points.device)
        self.set_stream(torch.cuda.current_stream(points.device).cuda_stream)
        f, ctx = self._lib.hca_cluster, self._ctx
        args = (ctx, ctypes.c_void_p(points.data_ptr()), n, d, float(eps), int(min_pts),
                ctypes.c_void_p(out.data_ptr()))

        def call():
            st = f(*args)
            if st != HCA_OK:
                self._check(st)
        return call

    def cluster_batch(self, points, rows, dims, eps, min_pts, out=None):
        """Cluster the data sets packed one after the other in the CUDA int32
        tensor ``points`` (flat, data set i being rows[i] x dims[i]).  Returns
        an int32 tensor with every data set's own labels at its rows."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.int32):
            raise TypeError("points must be a CUDA (HIP) int32 torch tensor")
        pts = points.contiguous()
        nseg = len(rows)
        r = np.ascontiguousarray(rows, dtype=np.int64)
        dm = np.ascontiguousarray(dims, dtype=np.int32)
        ep = np.ascontiguousarray(eps, dtype=np.float64)
        mp = np.ascontiguousarray(min_pts, dtype=np.int32)
        if not (len(dm) == len(ep) == len(mp) == nseg):
            raise ValueError("rows, dims, eps and min_pts must have one entry per data set")
        if int((r * dm).sum()) != pts.numel():
            raise ValueError("points does not hold sum(rows * dims) coordinates")
        total = int(r.sum())
        if out is not None:
            check_labels(out, total, pts.device)
        labels = out if out is not None else torch.empty(total, dtype=torch.int32, device=pts.device)
        self.set_stream(torch.cuda.current_stream(pts.device).cuda_stream)
        self._check(self._lib.hca_cluster_batch(
            self._ctx, ctypes.c_void_p(pts.data_ptr()), nseg, r.ctypes.data_as(ctypes.c_void_p),
            dm.ctypes.data_as(ctypes.c_void_p), ep.ctypes.data_as(ctypes.c_void_p),
            mp.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(labels.data_ptr())))
        return labels

    def cluster_noalloc(self, points, eps: float, min_pts: int, out):
        """hca_cluster_noalloc: cluster a CUDA int32 tensor [n, d] (d <= 8,
        contiguous, vector-aligned rows) into the caller's int32 tensor
        ``out`` without any allocation by the library or by this binding;
        runs on the current torch stream and blocks until done."""
        import torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.int32
                and points.dim() == 2 and points.is_contiguous()):
            raise TypeError("points must be a contiguous CUDA int32 tensor [n, d]")
        n, d = points.shape
        check_labels(out, n, points.device)
        self.set_stream(torch.cuda.current_stream(points.device).cuda_stream)
        self._check(self._lib.hca_cluster_noalloc(self._ctx, ctypes.c_void_p(points.data_ptr()), n, d,
                                                  float(eps), int(min_pts), ctypes.c_void_p(out.data_ptr())))
        return out

    def cluster_ptr(self, points_ptr: int, n: int, d: int, eps: float, min_pts: int,
                    labels_ptr: int):
        """hca_cluster on raw device pointers (no tensor checks)."""
        self._check(self._lib.hca_cluster(self._ctx, ctypes.c_void_p(points_ptr), int(n), int(d),
                                          float(eps), int(min_pts), ctypes.c_void_p(labels_ptr)))

    def cluster_host(self, points: np.ndarray, eps: float, min_pts: int) -> np.ndarray:
        """Cluster a host int32 array [n, d] (copied in and out by the library)."""
        p = np.ascontiguousarray(points, dtype=np.int32)
        if p.ndim != 2:
            raise TypeError("points must have shape [n, d]")
        labels = np.empty(p.shape[0], np.int32)
        st = self._lib.hca_cluster_host(self._ctx, p.ctypes.data_as(ctypes.c_void_p), p.shape[0],
                                        p.shape[1], float(eps), int(min_pts),
                                        labels.ctypes.data_as(ctypes.c_void_p))
        self._check(st)
        return labels


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    """A cached context per device."""
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def cluster(points, eps: float, min_pts: int, **kw):
    """Cluster a CUDA int32 tensor [n, d] on its device; see Context.cluster."""
    dev = points.device.index or 0
    return context(dev).cluster(points, eps, min_pts, **kw)
