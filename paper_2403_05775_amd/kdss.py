"""Python binding of the kdss C-ABI (argument marshalling only).

Every step of the method runs in libkdss.so: the clique tree is built by its
host code and every iteration and extraction runs in its HIP kernels.  PyTorch
only provides device memory and the stream.  The library must have been built
(``__graft_entry__.build()``); a missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkdss.so")

OK, EINVAL, EGRAPH, ERANGE, EOVERFLOW, EWORKSPACE, EHIP, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8


class KdssError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("n", C.c_uint32), ("nnz", C.c_uint64), ("row_ptr", C.POINTER(C.c_uint64)),
                ("col", C.POINTER(C.c_uint32))]


class U128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]

    @property
    def value(self) -> int:
        return (self.hi << 64) | self.lo


class TreeStats(C.Structure):
    _fields_ = [("k", C.c_uint32), ("n", C.c_uint32), ("leaves", C.c_uint64), ("members", C.c_uint64),
                ("s_max", C.c_uint32), ("degeneracy", C.c_uint32), ("c_k", U128),
                ("build_seconds", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("width", C.c_int), ("use_graph", C.c_int), ("extract_every", C.c_uint32),
                ("time_kernels", C.c_int), ("gather", C.c_int), ("update", C.c_int), ("schedule", C.c_int),
                ("heavy", C.c_int)]


class Timing(C.Structure):
    _fields_ = [("leaf_launches", C.c_uint64), ("leaf_ms", C.c_double), ("heavy_ms", C.c_double),
                ("reduce_ms", C.c_double), ("apply_launches", C.c_uint64), ("apply_ms", C.c_double),
                ("heavy_leaves", C.c_uint64)]


class TuneResult(C.Structure):
    _fields_ = [("tried", C.c_uint32), ("best_leaf_blocks", C.c_uint32), ("best_heavy_blocks", C.c_uint32),
                ("best_ms", C.c_double), ("leaf_blocks", C.c_uint32 * 32), ("heavy_blocks", C.c_uint32 * 32),
                ("ms", C.c_double * 32), ("best_gather", C.c_int), ("gather_ms", C.c_double * 2),
                ("best_schedule", C.c_int), ("schedule_ms", C.c_double * 2), ("best_heavy", C.c_int),
                ("heavy_ms", C.c_double * 3)]


class PlanStats(C.Structure):
    _fields_ = [("workspace_bytes", C.c_uint64), ("stream_bytes", C.c_uint64), ("width", C.c_int),
                ("key_mode", C.c_int), ("id_bits", C.c_uint32), ("T_max", C.c_uint32),
                ("tiles", C.c_uint64 * 5), ("leaves", C.c_uint64 * 5), ("members", C.c_uint64 * 5),
                ("gather", C.c_int), ("update", C.c_int), ("schedule", C.c_int), ("hot_nodes", C.c_uint32),
                ("hot_share", C.c_double), ("heavy", C.c_int)]


class SampleInfo(C.Structure):
    _fields_ = [("samples", C.c_uint64), ("cliques", C.c_uint64), ("distinct", C.c_uint64), ("paths", U128),
                ("colors", C.c_uint32), ("device_seconds", C.c_double), ("host_seconds", C.c_double)]


class Result(C.Structure):
    _fields_ = [("T", C.c_uint32), ("size", C.c_uint32), ("n", C.c_uint32), ("width", C.c_int),
                ("dens_num", U128), ("ub_num", U128), ("c_k", U128), ("density", C.c_double),
                ("upper_bound", C.c_double), ("bound_num", U128), ("bound_den", C.c_uint64),
                ("bound_kind", C.c_int), ("certified", C.c_int), ("bound", C.c_double)]


class TraceRow(C.Structure):
    _fields_ = [("t", C.c_uint32), ("size", C.c_uint32), ("dens_num", U128), ("ub_num", U128)]


EXPORTS = [
    "kdss_status_string", "kdss_last_error", "kdss_csr_validate", "kdss_sct_build", "kdss_sct_info",
    "kdss_sct_export", "kdss_sct_core_numbers", "kdss_sct_free", "kdss_plan_create", "kdss_plan_info",
    "kdss_plan_free", "kdss_plan_upload", "kdss_run", "kdss_leaf_credit", "kdss_extract", "kdss_plan_timing",
    "kdss_batch_create", "kdss_batch_offsets", "kdss_batch_run", "kdss_plan_set_launch", "kdss_plan_autotune",
    "kdss_sample_build", "kdss_sct_build_gpu", "kdss_workspace_size", "kdss_solve", "kdss_run_resume",
    "kdss_extract_counts", "kdss_batch_free", "kdss_run_static", "kdss_sct_count", "kdss_plan_tune_key",
    "kdss_plan_autotune_cached", "kdss_plan_set_timing", "kdss_sample_workspace", "kdss_sct_build_gpu_workspace",
]

TUNE_CACHE = os.path.join(_HERE, "tune_cache.txt")   # launches tuned on MI355X, keyed by plan shape

STATIC_WORKSPACE_BYTES = 64 << 20   # KDSS_STATIC_WORKSPACE_BYTES

_lib = None


def lib():
    """Load libkdss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    # torch supplies the device memory and streams; its HIP runtime must be the
    # one libkdss binds to, so it is loaded first (a second runtime loaded
    # beside it finds no device)
    import torch  # noqa: F401
    _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def lib_at(path: str):
    """Another build of the library (e.g. the fault-injection test build), bound the same way."""
    import torch  # noqa: F401
    return _bind(C.CDLL(path))


def _bind(L):
    vp, p64, p32 = C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
    L.kdss_status_string.restype = C.c_char_p
    L.kdss_status_string.argtypes = [C.c_int]
    L.kdss_last_error.restype = C.c_char_p
    L.kdss_csr_validate.argtypes = [C.POINTER(Csr)]
    L.kdss_sct_build.argtypes = [C.POINTER(Csr), C.c_uint32, C.c_uint32, C.POINTER(vp)]
    L.kdss_sct_info.argtypes = [vp, C.POINTER(TreeStats)]
    L.kdss_sct_count.argtypes = [C.POINTER(Csr), C.c_uint32, C.c_uint32, C.POINTER(TreeStats)]
    L.kdss_sct_export.argtypes = [vp, p32, p32, p32, C.c_uint64, C.c_uint64]
    L.kdss_sct_core_numbers.argtypes = [vp, p32, C.c_uint32]
    L.kdss_sct_free.argtypes = [vp]
    L.kdss_sct_build_gpu.argtypes = [C.POINTER(Csr), C.c_uint32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.kdss_sct_build_gpu_workspace.argtypes = [C.POINTER(Csr), C.c_uint32, C.POINTER(C.c_size_t)]
    L.kdss_sample_build.argtypes = [C.POINTER(Csr), C.c_uint32, C.c_uint64, p64, vp, C.c_size_t, vp,
                                    C.POINTER(SampleInfo), C.POINTER(vp)]
    L.kdss_sample_workspace.argtypes = [C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint64, C.POINTER(C.c_size_t)]
    L.kdss_sct_free.restype = None
    L.kdss_plan_create.argtypes = [vp, C.c_uint32, C.c_uint64, C.POINTER(Opts), C.POINTER(vp)]
    L.kdss_plan_info.argtypes = [vp, C.POINTER(PlanStats)]
    L.kdss_plan_free.argtypes = [vp]
    L.kdss_plan_free.restype = None
    L.kdss_plan_upload.argtypes = [vp, vp, C.c_size_t, vp]
    L.kdss_plan_timing.argtypes = [vp, C.POINTER(Timing), C.c_int]
    L.kdss_run.argtypes = [vp, vp, C.c_size_t, C.c_uint32, vp, vp, vp, C.POINTER(TraceRow), C.c_uint32,
                           C.POINTER(Result), vp]
    L.kdss_leaf_credit.argtypes = [vp, vp, C.c_size_t, vp, vp, vp]
    L.kdss_batch_create.argtypes = [C.POINTER(vp), C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(Opts),
                                    C.POINTER(vp)]
    L.kdss_batch_offsets.argtypes = [vp, p64, C.c_uint32]
    L.kdss_batch_run.argtypes = [vp, vp, C.c_size_t, C.c_uint32, vp, vp, vp, C.POINTER(Result), C.c_uint32, vp]
    L.kdss_plan_set_launch.argtypes = [vp, C.c_uint32, C.c_uint32]
    L.kdss_plan_autotune.argtypes = [vp, vp, C.c_size_t, vp, C.c_uint32, C.c_uint32, C.POINTER(TuneResult), vp]
    L.kdss_plan_tune_key.argtypes = [vp, C.c_char_p, C.c_size_t]
    L.kdss_plan_set_timing.argtypes = [vp, C.c_int]
    L.kdss_plan_autotune_cached.argtypes = [vp, vp, C.c_size_t, vp, C.c_uint32, C.c_uint32, C.c_char_p,
                                            C.POINTER(C.c_int), C.POINTER(TuneResult), vp]
    L.kdss_extract.argtypes = [vp, vp, C.c_size_t, vp, vp, C.c_uint32, vp, C.POINTER(Result), vp]
    L.kdss_extract_counts.argtypes = [vp, vp, C.c_size_t, vp, vp, C.c_uint32, vp, vp, C.POINTER(Result), vp]
    L.kdss_workspace_size.argtypes = [vp, C.c_uint32, C.c_uint64, C.POINTER(Opts), C.POINTER(C.c_size_t)]
    L.kdss_solve.argtypes = [C.POINTER(Csr), C.c_uint32, C.c_uint32, C.POINTER(Opts), vp, C.c_uint64, vp,
                             C.c_size_t, C.POINTER(C.c_size_t), vp, C.c_size_t, vp, C.POINTER(Result), vp]
    L.kdss_run_resume.argtypes = [vp, vp, C.c_size_t, C.c_uint32, C.c_uint32, vp, vp, vp, vp, C.POINTER(TraceRow),
                                  C.c_uint32, C.POINTER(Result), vp]
    L.kdss_run_static.argtypes = [vp, C.c_uint32, vp, vp, vp, C.POINTER(Result), vp]
    L.kdss_batch_free.argtypes = [vp]
    L.kdss_batch_free.restype = None
    return L


def _check(status: int, where: str):
    if status != OK:
        detail = lib().kdss_last_error().decode(errors="replace")
        raise KdssError(status, where, detail or lib().kdss_status_string(status).decode())


def _csr(graph):
    rp = np.ascontiguousarray(graph.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(graph.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    c = Csr(graph.n, int(rp[graph.n]), rp.ctypes.data_as(C.POINTER(C.c_uint64)),
            col.ctypes.data_as(C.POINTER(C.c_uint32)))
    return c, (rp, col)


def validate(graph) -> int:
    c, keep = _csr(graph)
    return lib().kdss_csr_validate(C.byref(c))


def tree_count(graph, k: int, threads: int = 0) -> TreeStats:
    """The k-pruned tree's sizes without building it (kdss_sct_count)."""
    c, keep = _csr(graph)
    s = TreeStats()
    _check(lib().kdss_sct_count(C.byref(c), k, threads, C.byref(s)), "kdss_sct_count")
    return s


class Tree:
    """The k-pruned succinct clique tree of a graph, built by the library's host code."""

    def __init__(self, graph, k: int, threads: int = 0):
        c, keep = _csr(graph)
        h = C.c_void_p()
        _check(lib().kdss_sct_build(C.byref(c), k, threads, C.byref(h)), "kdss_sct_build")
        self._h = h
        self.n, self.k = graph.n, k

    def stats(self) -> TreeStats:
        s = TreeStats()
        _check(lib().kdss_sct_info(self._h, C.byref(s)), "kdss_sct_info")
        return s

    def workspace_size(self, T_max: int, r0_max: int = 0, width: int = 0, update: int = 0) -> int:
        """Device workspace a plan of this tree would need (kdss_workspace_size)."""
        o = Opts(width, 0, 0, 0, 0, update)
        b = C.c_size_t(0)
        _check(lib().kdss_workspace_size(self._h, T_max, r0_max, C.byref(o), C.byref(b)), "kdss_workspace_size")
        return b.value

    def export(self):
        """(h, p, members) of the kept leaves."""
        s = self.stats()
        h = np.zeros(max(s.leaves, 1), dtype=np.uint32)
        p = np.zeros(max(s.leaves, 1), dtype=np.uint32)
        m = np.zeros(max(s.members, 1), dtype=np.uint32)
        P32 = C.POINTER(C.c_uint32)
        _check(lib().kdss_sct_export(self._h, h.ctypes.data_as(P32), p.ctypes.data_as(P32), m.ctypes.data_as(P32),
                                     h.size, m.size), "kdss_sct_export")
        return h[: s.leaves], p[: s.leaves], m[: s.members]

    def core_numbers(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.uint32)
        _check(lib().kdss_sct_core_numbers(self._h, out.ctypes.data_as(C.POINTER(C.c_uint32)), self.n),
               "kdss_sct_core_numbers")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().kdss_sct_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GpuTree(Tree):
    """The k-pruned succinct clique tree built on the GPU (kdss_sct_build_gpu),
    in a workspace of ws_bytes (default: kdss_sct_build_gpu_workspace's size)."""

    def __init__(self, graph, k: int, stream=None, ws_bytes: int | None = None):
        import torch
        c, keep = _csr(graph)
        h = C.c_void_p()
        need = C.c_size_t(0)
        _check(lib().kdss_sct_build_gpu_workspace(C.byref(c), k, C.byref(need)), "kdss_sct_build_gpu_workspace")
        nbytes = need.value if ws_bytes is None else ws_bytes
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        _check(lib().kdss_sct_build_gpu(C.byref(c), k, _ptr(ws), nbytes,
                                        _stream(stream) if stream is not None else None, C.byref(h)),
               "kdss_sct_build_gpu")
        del ws
        self._h = h
        self.n, self.k = graph.n, k


class SampleTree(Tree):
    """Algorithm 4's sample set as a clique tree: t colour-increasing k-node
    paths sampled on the GPU with the given draws (uint64[t, k, 2]); the
    distinct ones that are k-cliques become leaves (C, {})."""

    def __init__(self, graph, k: int, draws, stream=None):
        c, keep = _csr(graph)
        d = np.ascontiguousarray(draws, dtype=np.uint64)
        t = d.shape[0] if d.size else 0
        h = C.c_void_p()
        info = SampleInfo()
        need = C.c_size_t(0)
        _check(lib().kdss_sample_workspace(graph.n, int(c.nnz), k, t, C.byref(need)), "kdss_sample_workspace")
        ws = None
        if need.value:
            import torch
            ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        _check(lib().kdss_sample_build(C.byref(c), k, t, d.ctypes.data_as(C.POINTER(C.c_uint64)) if t else None,
                                       _ptr(ws), need.value, _stream(stream) if t else None, C.byref(info),
                                       C.byref(h)),
               "kdss_sample_build")
        self._h = h
        self.n, self.k = graph.n, k
        self.info = info


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Plan:
    """Device layout of a tree; owns nothing on the device."""

    def __init__(self, tree: Tree, T_max: int, r0_max: int = 0, width: int = 0, use_graph: bool = False,
                 extract_every: int = 0, time_kernels: bool = False, gather: int = 0, update: int = 0,
                 schedule: int = 0, heavy: int = 0):
        o = Opts(width, int(use_graph), extract_every, 1 if time_kernels else 0, gather, update, schedule, heavy)
        h = C.c_void_p()
        _check(lib().kdss_plan_create(tree._h, T_max, r0_max, C.byref(o), C.byref(h)), "kdss_plan_create")
        self._h = h
        self.n, self.k, self.T_max = tree.n, tree.k, T_max
        self.extract_every = extract_every
        st = self.stats()
        self.width = st.width
        self.workspace_bytes = st.workspace_bytes

    def stats(self) -> PlanStats:
        s = PlanStats()
        _check(lib().kdss_plan_info(self._h, C.byref(s)), "kdss_plan_info")
        return s

    def set_launch(self, leaf_blocks: int, heavy_blocks: int):
        _check(lib().kdss_plan_set_launch(self._h, leaf_blocks, heavy_blocks), "kdss_plan_set_launch")

    def autotune(self, ws, r, warm: int = 3, iters: int = 3, stream=None) -> TuneResult:
        """Time candidate grid sizes on this plan's data and keep the fastest."""
        out = TuneResult()
        _check(lib().kdss_plan_autotune(self._h, _ptr(ws), ws.numel(), _ptr(r), warm, iters, C.byref(out),
                                        _stream(stream)), "kdss_plan_autotune")
        return out

    def tune_key(self) -> str:
        buf = C.create_string_buffer(512)
        _check(lib().kdss_plan_tune_key(self._h, buf, 512), "kdss_plan_tune_key")
        return buf.value.decode()

    def autotune_cached(self, ws, r, warm: int, iters: int, cache_path: str = TUNE_CACHE, stream=None):
        """Tuned launch from the cache file, or tuned now and filed there; returns (result, from_cache)."""
        out = TuneResult()
        hit = C.c_int(0)
        _check(lib().kdss_plan_autotune_cached(self._h, _ptr(ws), ws.numel(), _ptr(r), warm, iters,
                                               cache_path.encode(), C.byref(hit), C.byref(out), _stream(stream)),
               "kdss_plan_autotune_cached")
        return out, bool(hit.value)

    def set_timing(self, on: bool):
        _check(lib().kdss_plan_set_timing(self._h, 1 if on else 0), "kdss_plan_set_timing")

    def timing(self, reset: bool = False) -> Timing:
        t = Timing()
        _check(lib().kdss_plan_timing(self._h, C.byref(t), 1 if reset else 0), "kdss_plan_timing")
        return t

    def alloc_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def alloc_loads(self, device="cuda"):
        import torch
        words = self.n * (2 if self.width == 128 else 1)
        return torch.empty(max(words, 1), dtype=torch.int64, device=device)

    def upload(self, ws, stream=None):
        _check(lib().kdss_plan_upload(self._h, _ptr(ws), ws.numel(), _stream(stream)), "kdss_plan_upload")

    def run(self, ws, T: int, r, order, r0=None, trace_cap: int = 0, stream=None):
        res = Result()
        rows = (TraceRow * trace_cap)() if trace_cap else None
        _check(lib().kdss_run(self._h, _ptr(ws), ws.numel(), T, _ptr(r0), _ptr(r), _ptr(order),
                              C.cast(rows, C.POINTER(TraceRow)) if rows is not None else None, trace_cap,
                              C.byref(res), _stream(stream)), "kdss_run")
        trace = None
        if rows is not None:
            trace = [dict(t=x.t, size=x.size, dens_num=x.dens_num.value, ub_num=x.ub_num.value)
                     for x in rows if x.t]
        return res, trace

    def resume(self, ws, T: int, t_offset: int, start, r, order, r0=None, trace_cap: int = 0, stream=None):
        """T more iterations from checkpoint loads `start` (u64[n]) of a run that
        began at r0 (nullable) t_offset iterations earlier (kdss_run_resume)."""
        res = Result()
        rows = (TraceRow * trace_cap)() if trace_cap else None
        _check(lib().kdss_run_resume(self._h, _ptr(ws), ws.numel(), T, t_offset, _ptr(start), _ptr(r0), _ptr(r),
                                     _ptr(order), C.cast(rows, C.POINTER(TraceRow)) if rows is not None else None,
                                     trace_cap, C.byref(res), _stream(stream)), "kdss_run_resume")
        trace = None
        if rows is not None:
            trace = [dict(t=x.t, size=x.size, dens_num=x.dens_num.value, ub_num=x.ub_num.value)
                     for x in rows if x.t]
        return res, trace

    def extract_counts(self, ws, r, order, counts, T: int, r0=None, stream=None) -> Result:
        """The extraction with every prefix count K_i into counts (u64[n])."""
        res = Result()
        _check(lib().kdss_extract_counts(self._h, _ptr(ws), ws.numel(), _ptr(r), _ptr(r0), T, _ptr(order),
                                         _ptr(counts), C.byref(res), _stream(stream)), "kdss_extract_counts")
        return res

    def run_static(self, T: int, r, order, r0=None, stream=None) -> Result:
        """kdss_run on the library's static device workspace (no device allocation)."""
        res = Result()
        _check(lib().kdss_run_static(self._h, T, _ptr(r0), _ptr(r), _ptr(order), C.byref(res), _stream(stream)),
               "kdss_run_static")
        return res

    def leaf_credit(self, ws, r, out, stream=None):
        _check(lib().kdss_leaf_credit(self._h, _ptr(ws), ws.numel(), _ptr(r), _ptr(out), _stream(stream)),
               "kdss_leaf_credit")

    def extract(self, ws, r, order, T: int, r0=None, stream=None) -> Result:
        res = Result()
        _check(lib().kdss_extract(self._h, _ptr(ws), ws.numel(), _ptr(r), _ptr(r0), T, _ptr(order),
                                  C.byref(res), _stream(stream)), "kdss_extract")
        return res

    def close(self):
        if getattr(self, "_h", None):
            lib().kdss_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(Plan):
    """Many (graph, k) problems laid out as one plan: one launch per iteration
    covers every problem; each problem's result equals its solo run."""

    def __init__(self, trees, T_max: int, r0_max: int = 0, use_graph: bool = False, time_kernels: bool = False,
                 gather: int = 0, update: int = 0, schedule: int = 0, heavy: int = 0):
        o = Opts(0, int(use_graph), 0, 1 if time_kernels else 0, gather, update, schedule, heavy)
        arr = (C.c_void_p * len(trees))(*[t._h for t in trees])
        h = C.c_void_p()
        _check(lib().kdss_batch_create(arr, len(trees), T_max, r0_max, C.byref(o), C.byref(h)), "kdss_batch_create")
        self._h = h
        self.count = len(trees)
        self.T_max = T_max
        self.extract_every = 0
        off = np.zeros(self.count + 1, dtype=np.uint64)
        _check(lib().kdss_batch_offsets(h, off.ctypes.data_as(C.POINTER(C.c_uint64)), self.count),
               "kdss_batch_offsets")
        self.node_off = off
        self.n = int(off[-1])
        self.k = None
        st = self.stats()
        self.width = st.width
        self.workspace_bytes = st.workspace_bytes

    def close(self):
        if getattr(self, "_h", None):
            lib().kdss_batch_free(self._h)
            self._h = None

    def run(self, ws, T: int, r, order, r0=None, stream=None):
        res = (Result * self.count)()
        _check(lib().kdss_batch_run(self._h, _ptr(ws), ws.numel(), T, _ptr(r0), _ptr(r), _ptr(order), res,
                                    self.count, _stream(stream)), "kdss_batch_run")
        return list(res)


def loads_to_numpy(r_tensor, n: int, width: int):
    """Device loads -> numpy uint64 (width 64) or a list of Python ints (width 128)."""
    a = r_tensor.cpu().numpy().view(np.uint64)
    if width == 64:
        return a[:n].copy()
    lo, hi = a[0: 2 * n: 2], a[1: 2 * n: 2]
    if not np.any(hi):
        return lo.copy()
    return [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]


@dataclass
class Solution:
    r: object                 # numpy uint64[n] or list of ints
    order: np.ndarray         # uint32[n]
    size: int
    dens_num: int
    ub_num: int
    T: int
    c_k: int
    width: int
    trace: list | None
    tree_stats: TreeStats
    plan_stats: PlanStats
    bound_num: int = 0        # certified bound on rho*: bound_num / bound_den
    bound_den: int = 1
    bound_kind: int = 0       # 1: top-s bound, 0: max (r - r0) / T
    certified: bool = False   # the density is rho*

    @property
    def nodes(self) -> np.ndarray:
        return self.order[: self.size]


def solve(graph, k: int, T: int, r0=None, width: int = 0, use_graph: bool = False, extract_every: int = 0,
          threads: int = 0, device="cuda", gather: int = 0, update: int = 0, schedule: int = 0,
          heavy: int = 0) -> Solution:
    """Build the tree, lay it out, run T iterations and the extraction on the GPU."""
    import torch
    tree = Tree(graph, k, threads)
    r0_max = 0 if r0 is None else int(np.max(np.asarray(r0, dtype=np.uint64))) if graph.n else 0
    plan = Plan(tree, T, r0_max, width=width, use_graph=use_graph, extract_every=extract_every, gather=gather,
                update=update, schedule=schedule, heavy=heavy)
    ws = plan.alloc_workspace(device)
    plan.upload(ws)
    r = plan.alloc_loads(device)
    order = torch.empty(max(graph.n, 1), dtype=torch.int32, device=device)
    r0_t = None
    if r0 is not None:
        r0_t = torch.from_numpy(np.asarray(r0, dtype=np.uint64).view(np.int64).copy()).to(device)
    cap = (T // extract_every + 1) if extract_every else 0
    res, trace = plan.run(ws, T, r, order, r0=r0_t, trace_cap=cap)
    torch.cuda.synchronize()
    out = Solution(r=loads_to_numpy(r, graph.n, plan.width),
                   order=order.cpu().numpy().view(np.uint32)[: graph.n].copy(), size=res.size,
                   dens_num=res.dens_num.value, ub_num=res.ub_num.value, T=res.T, c_k=res.c_k.value,
                   width=res.width, trace=trace, tree_stats=tree.stats(), plan_stats=plan.stats(),
                   bound_num=res.bound_num.value, bound_den=res.bound_den, bound_kind=res.bound_kind,
                   certified=bool(res.certified))
    plan.close()
    tree.close()
    return out


def solve_one_shot(graph, k: int, T: int, r0=None, width: int = 0, device="cuda", stream=None):
    """kdss_solve: a first call sizes the buffers (nothing runs), the second
    builds, lays out, uploads and runs in one C call."""
    import torch
    c, keep = _csr(graph)
    o = Opts(width, 0, 0, 0, 0, 0)
    need = C.c_size_t(0)
    res = Result()
    r0_max = 0 if r0 is None or graph.n == 0 else int(np.max(np.asarray(r0, dtype=np.uint64)))
    r0_t = None
    if r0 is not None:
        r0_t = torch.from_numpy(np.asarray(r0, dtype=np.uint64).view(np.int64).copy()).to(device)
    st = _stream(stream)
    rc = lib().kdss_solve(C.byref(c), k, T, C.byref(o), _ptr(r0_t), r0_max, None, 0, C.byref(need), None, 0, None,
                          C.byref(res), st)
    if rc != EWORKSPACE:
        _check(rc, "kdss_solve (size query)")
    words = max(graph.n * (2 if res.width == 128 else 1), 1)
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    r = torch.empty(words, dtype=torch.int64, device=device)
    order = torch.empty(max(graph.n, 1), dtype=torch.int32, device=device)
    _check(lib().kdss_solve(C.byref(c), k, T, C.byref(o), _ptr(r0_t), r0_max, _ptr(ws), ws.numel(), C.byref(need),
                            _ptr(r), words, _ptr(order), C.byref(res), st), "kdss_solve")
    torch.cuda.synchronize()
    return res, loads_to_numpy(r, graph.n, res.width), order.cpu().numpy().view(np.uint32)[: graph.n].copy()
