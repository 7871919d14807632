"""MI355X random hyperbolic graph generator: Python binding of librhg.so.

The functions here carry the names of the C ABI in ``include/rhg.h`` and do
argument marshalling only: PyTorch supplies device memory and the current
HIP stream, and every step of the computation runs in the library's HIP
kernels.  There is no CPU fallback: if ``librhg.so`` is missing or fails to
load, importing a function raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librhg.so")

RHG_OK, RHG_EINVAL, RHG_ENOMEM, RHG_ECAPACITY, RHG_EDEVICE, RHG_ENOROOT, RHG_EINTERNAL, RHG_EBUSY = range(8)
_STATUS = {0: "RHG_OK", 1: "RHG_EINVAL", 2: "RHG_ENOMEM", 3: "RHG_ECAPACITY", 4: "RHG_EDEVICE",
           5: "RHG_ENOROOT", 6: "RHG_EINTERNAL", 7: "RHG_EBUSY"}


class RhgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


class rhg_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("avg_degree", C.c_double), ("gamma", C.c_double),
                ("seed", C.c_uint64), ("alpha", C.c_double), ("R", C.c_double),
                ("cosh_R", C.c_double), ("cosh_R_lo", C.c_double), ("cosh_aR_m1", C.c_double),
                ("cosh_aR_m1_lo", C.c_double)]


class rhg_tuning(C.Structure):
    _fields_ = [("band_width", C.c_double), ("inner_radius", C.c_double),
                ("cell_target", C.c_int32), ("heavy_points", C.c_int32), ("sweep_max", C.c_int32),
                ("sweep_linear", C.c_int32), ("fp64_only", C.c_int32), ("no_stream_stage", C.c_int32),
                ("exact_inline", C.c_int32), ("defer_cap", C.c_int32), ("stage", C.c_int32),
                ("stage_pct", C.c_int32)]


class rhg_stats(C.Structure):
    _fields_ = [("fp32_undecided", C.c_int64), ("dd_fallbacks", C.c_int64), ("ties", C.c_int64),
                ("swept", C.c_int64), ("tests", C.c_int64),
                ("register_streams", C.c_int64), ("temp_candidates", C.c_int64),
                ("temp_coins", C.c_int64), ("staged_waves", C.c_int64), ("stage_overflows", C.c_int64)]


class rhg_graph_summary(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("max_degree", C.c_int64), ("hist", C.c_int64 * 33),
                ("kmin", C.c_double), ("tail_count", C.c_int64), ("gamma_mle", C.c_double),
                ("assortativity", C.c_double), ("triads", C.c_int64), ("triangles", C.c_int64),
                ("transitivity", C.c_double), ("avg_local_clustering", C.c_double),
                ("ascending_rows", C.c_int32), ("reserved", C.c_int32)]


class rhg_completion(C.Structure):
    _fields_ = [("req_id", C.c_int64), ("status", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64),
                ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("r", C.c_void_p),
                ("theta", C.c_void_p), ("latency_ms", C.c_double), ("params", rhg_params)]


class rhg_server_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "failed", "rejected", "refills", "edges",
                                         "max_inflight", "max_reserved_bytes", "reserved_bytes", "inflight",
                                         "queued")]


class rhg_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("r", C.c_void_p), ("theta", C.c_void_p), ("params", rhg_params)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)

_lib = None


def load():
    """Load librhg.so (built by ``build.py``); raises if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librhg.so is not built (run paper_1501_03545_amd/build.py or "
                           "__graft_entry__.build()); there is no fallback path")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one.  Loading torch first makes librhg.so bind to that same runtime, so
    # that torch's streams and allocations are valid handles for the library.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i64, d, u64, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_uint64, C.c_int
    P = C.POINTER
    sig = {
        "rhg_plan": (i32, [i64, d, d, u64, P(rhg_params)]),
        "rhg_plan_radius": (i32, [i64, d, d, u64, P(rhg_params)]),
        "rhg_sample_points": (i32, [P(rhg_params), vp, vp, vp]),
        "rhg_index_workspace_bytes": (C.c_size_t, [P(rhg_params), P(rhg_tuning)]),
        "rhg_layout_bands": (i32, [P(rhg_params), P(rhg_tuning), P(C.c_double), i32, P(C.c_int)]),
        "rhg_build_index": (i32, [P(rhg_params), vp, vp, P(rhg_tuning), vp, C.c_size_t, i32, P(vp), vp]),
        "rhg_count_edges": (i32, [vp, vp, vp]),
        "rhg_emit_edges": (i32, [vp, vp, vp, i64, i32, vp]),
        "rhg_sort_rows_workspace_bytes": (C.c_size_t, [i64, i64]),
        "rhg_sort_rows": (i32, [i64, vp, vp, i64, vp, C.c_size_t, vp]),
        "rhg_long_range_workspace_bytes": (C.c_size_t, [i64, i64]),
        "rhg_graph_stats_workspace_bytes": (C.c_size_t, [i64, i64, i32]),
        "rhg_graph_stats": (i32, [i64, vp, vp, i64, d, i32, vp, C.c_size_t, P(rhg_graph_summary), vp]),
        "rhg_long_range": (i32, [i64, vp, vp, i64, i64, u64, vp, C.c_size_t, vp, vp, i64, vp, vp]),
        "rhg_index_stats": (i32, [vp, P(rhg_stats), vp]),
        "rhg_index_free": (None, [vp]),
        "rhg_generate": (i32, [i64, d, d, u64, P(rhg_tuning), ALLOC_FN, vp, i32, P(rhg_csr), vp]),
        "rhg_generate_async": (i32, [P(rhg_params), P(rhg_tuning), vp, vp, vp, C.c_size_t, vp, vp, i64, vp, vp]),
        "rhg_generate_async_noalloc": (i32, [P(rhg_params), P(rhg_tuning), vp, vp, vp, vp, i64, vp, vp]),
        "rhg_server_create": (i32, [C.c_size_t, i32, P(vp)]),
        "rhg_server_submit": (i32, [vp, i64, i64, C.c_double, C.c_double, C.c_uint64, P(rhg_tuning)]),
        "rhg_server_poll": (i32, [vp, P(rhg_completion), i32, P(i32)]),
        "rhg_server_release": (i32, [vp, i64]),
        "rhg_server_get_stats": (i32, [vp, P(rhg_server_stats)]),
        "rhg_server_destroy": (None, [vp]),
        "rhg_batch_create": (i32, [i32, P(rhg_params), P(rhg_tuning), P(vp), P(vp), P(vp), P(C.c_size_t), P(vp),
                                   P(vp), P(i64), vp, i32, P(vp)]),
        "rhg_batch_launch": (i32, [vp, vp]),
        "rhg_batch_destroy": (None, [vp]),
        "rhg_temp_count_edges": (i32, [vp, d, vp, vp]),
        "rhg_temp_emit_edges": (i32, [vp, d, vp, vp, i64, i32, vp]),
        "rhg_temp_generate": (i32, [i64, d, d, d, u64, P(rhg_tuning), ALLOC_FN, vp, i32, P(rhg_csr), vp]),
        "rhg_dyn_create": (i32, [P(rhg_params), P(rhg_tuning), vp, vp, P(vp), vp]),
        "rhg_dyn_move": (i32, [vp, i64, vp, vp, vp, vp]),
        "rhg_dyn_graph": (i32, [vp, P(rhg_csr)]),
        "rhg_dyn_last_step": (i32, [vp, P(i64), P(i64)]),
        "rhg_dyn_set_regenerate_share": (i32, [vp, d]),
        "rhg_dyn_free": (None, [vp]),
        "rhg_set_profiling": (i32, [i32]),
        "rhg_phase_times": (i32, [P(C.c_double), P(C.c_int64), i32]),
        "rhg_phase_name": (C.c_char_p, [i32]),
        "rhg_last_error": (C.c_char_p, []),
        "rhg_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != RHG_OK:
        raise RhgError(status, load().rhg_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _tuning(t: Optional[dict]):
    if not t:
        return None
    tu = rhg_tuning()
    tu.band_width = float(t.get("band_width", 0.0))
    tu.inner_radius = float(t.get("inner_radius", 0.0))
    tu.cell_target = int(t.get("cell_target", 0))
    tu.heavy_points = int(t.get("heavy_points", 0))
    tu.sweep_max = int(t.get("sweep_max", 0))
    tu.sweep_linear = 1 if t.get("sweep_linear") else 0
    tu.fp64_only = 1 if t.get("fp64_only") else 0
    tu.no_stream_stage = 1 if t.get("no_stream_stage") else 0
    tu.exact_inline = 1 if t.get("exact_inline") else 0
    tu.defer_cap = int(t.get("defer_cap", 0))
    tu.stage = int(t.get("stage", 0))
    tu.stage_pct = int(t.get("stage_pct", 0))
    return C.byref(tu)


def version() -> str:
    return load().rhg_version().decode()


def rhg_plan(n: int, avg_degree: float, gamma: float, seed: int) -> rhg_params:
    p = rhg_params()
    _check(load().rhg_plan(n, avg_degree, gamma, seed, C.byref(p)))
    return p


def rhg_plan_radius(n: int, alpha: float, R: float, seed: int = 0) -> rhg_params:
    p = rhg_params()
    _check(load().rhg_plan_radius(n, alpha, R, seed, C.byref(p)))
    return p


def rhg_sample_points(p: rhg_params, r, theta, stream=None):
    """Fill device float64 tensors r, theta (n each) with the graph's points."""
    assert r.dtype == theta.dtype and r.is_cuda and theta.is_cuda
    assert r.numel() >= p.n and theta.numel() >= p.n and r.is_contiguous() and theta.is_contiguous()
    _check(load().rhg_sample_points(C.byref(p), _ptr(r), _ptr(theta), _stream(stream)))


def rhg_layout_bands(p: rhg_params, tuning: Optional[dict] = None):
    """Band edges E[0..B] of the index layout for these parameters (host only)."""
    buf = (C.c_double * 65)()
    b = C.c_int()
    _check(load().rhg_layout_bands(C.byref(p), _tuning(tuning), buf, 65, C.byref(b)))
    return [buf[j] for j in range(b.value + 1)]


def rhg_index_workspace_bytes(p: rhg_params, tuning: Optional[dict] = None) -> int:
    return int(load().rhg_index_workspace_bytes(C.byref(p), _tuning(tuning)))


@dataclass
class Index:
    handle: C.c_void_p
    workspace: object  # torch tensor that backs the index
    params: rhg_params

    def free(self):
        if self.handle:
            load().rhg_index_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rhg_build_index(p: rhg_params, r, theta, tuning: Optional[dict] = None, workspace=None,
                    validate: bool = True, stream=None) -> Index:
    import torch
    nbytes = rhg_index_workspace_bytes(p, tuning)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=r.device)
    h = C.c_void_p()
    _check(load().rhg_build_index(C.byref(p), _ptr(r), _ptr(theta), _tuning(tuning), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), 1 if validate else 0,
                                  C.byref(h), _stream(stream)))
    return Index(h, workspace, p)


def rhg_count_edges(idx: Index, row_ptr, stream=None):
    """row_ptr: device int64 tensor of n + 1 entries."""
    import torch
    assert row_ptr.dtype == torch.int64 and row_ptr.numel() >= idx.params.n + 1
    _check(load().rhg_count_edges(idx.handle, _ptr(row_ptr), _stream(stream)))


def rhg_emit_edges(idx: Index, row_ptr, col_idx, canonical_rows: bool = False, stream=None):
    import torch
    assert col_idx.dtype == torch.int32
    _check(load().rhg_emit_edges(idx.handle, _ptr(row_ptr), _ptr(col_idx), col_idx.numel(),
                                 1 if canonical_rows else 0, _stream(stream)))


def rhg_sort_rows_workspace_bytes(n: int, nnz: int) -> int:
    return int(load().rhg_sort_rows_workspace_bytes(int(n), int(nnz)))


def rhg_sort_rows(row_ptr, col_idx, nnz: Optional[int] = None, workspace=None, stream=None):
    """Sorts every row of the CSR (row_ptr: device int64, n + 1; col_idx:
    device int32) ascending, in place.  nnz defaults to row_ptr[n] (read
    back); the workspace defaults to a new device tensor."""
    import torch
    assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32
    assert row_ptr.is_contiguous() and col_idx.is_contiguous()
    n = row_ptr.numel() - 1
    if nnz is None:
        nnz = int(row_ptr[n].item()) - int(row_ptr[0].item()) if n >= 0 else 0
    nbytes = rhg_sort_rows_workspace_bytes(n, nnz)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=col_idx.device)
    _check(load().rhg_sort_rows(n, _ptr(row_ptr), _ptr(col_idx), int(nnz), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)))


def rhg_long_range_workspace_bytes(n: int, k: int) -> int:
    return int(load().rhg_long_range_workspace_bytes(int(n), int(k)))


def long_range_count(m: int, fraction: float = 0.005) -> int:
    """k for a share `fraction` of m undirected edges: ceil(fraction * m)."""
    import math
    return int(math.ceil(fraction * m))


def rhg_long_range(row_ptr, col_idx, k: int, seed: int, nnz: Optional[int] = None, workspace=None,
                   out=None, stream=None):
    """Adds k random edges (see rhg.h).  Returns (row_ptr_out, col_out,
    added) with `added` a device int64 tensor of one entry."""
    import torch
    assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32
    n = row_ptr.numel() - 1
    if nnz is None:
        nnz = int(row_ptr[n].item())
    dev = row_ptr.device
    if workspace is None:
        workspace = torch.empty(max(rhg_long_range_workspace_bytes(n, k), 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = (torch.empty(n + 1, dtype=torch.int64, device=dev),
               torch.empty(max(nnz + 2 * k, 1), dtype=torch.int32, device=dev))
    rp_out, col_out = out
    added = torch.empty(1, dtype=torch.int64, device=dev)
    _check(load().rhg_long_range(n, _ptr(row_ptr), _ptr(col_idx), int(nnz), int(k), int(seed), _ptr(workspace),
                                 workspace.numel(), _ptr(rp_out), _ptr(col_out), col_out.numel(), _ptr(added),
                                 _stream(stream)))
    return rp_out, col_out, added


def rhg_graph_stats_workspace_bytes(n: int, nnz: int, triangles: bool = True) -> int:
    return int(load().rhg_graph_stats_workspace_bytes(int(n), int(nnz), 1 if triangles else 0))


def rhg_graph_stats(row_ptr, col_idx, kmin: float = 10.0, triangles: bool = True, nnz: Optional[int] = None,
                    workspace=None, stream=None) -> dict:
    """Validation statistics of a simple symmetric CSR (see rhg.h); triangles
    need ascending rows.  Synchronises."""
    import torch
    assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32
    n = row_ptr.numel() - 1
    if nnz is None:
        nnz = int(row_ptr[n].item())
    if workspace is None:
        workspace = torch.empty(rhg_graph_stats_workspace_bytes(n, nnz, triangles), dtype=torch.uint8,
                                device=row_ptr.device)
    out = rhg_graph_summary()
    _check(load().rhg_graph_stats(n, _ptr(row_ptr), _ptr(col_idx), int(nnz), float(kmin), 1 if triangles else 0,
                                  _ptr(workspace), workspace.numel(), C.byref(out), _stream(stream)))
    res = {f: getattr(out, f) for f, _ in rhg_graph_summary._fields_ if f not in ("hist", "reserved")}
    res["hist"] = list(out.hist)
    return res


def rhg_index_stats(idx: Index, stream=None) -> dict:
    st = rhg_stats()
    _check(load().rhg_index_stats(idx.handle, C.byref(st), _stream(stream)))
    return {"fp32_undecided": st.fp32_undecided, "dd_fallbacks": st.dd_fallbacks, "ties": st.ties,
            "swept": st.swept, "tests": st.tests, "register_streams": st.register_streams,
            "temp_candidates": st.temp_candidates, "temp_coins": st.temp_coins,
            "staged_waves": st.staged_waves, "stage_overflows": st.stage_overflows}


PHASES = ["sample", "keys+sort", "index", "gather", "plan", "count", "scan", "emit", "rows"]


def rhg_set_profiling(on: bool):
    """Record HIP events around each library phase (see rhg_phase_times)."""
    _check(load().rhg_set_profiling(1 if on else 0))


def rhg_phase_times() -> dict:
    """{phase name: (average ms per launch, launches)} since profiling was enabled."""
    k = len(PHASES)
    ms = (C.c_double * k)()
    cnt = (C.c_int64 * k)()
    _check(load().rhg_phase_times(ms, cnt, k))
    return {load().rhg_phase_name(i).decode(): (ms[i], cnt[i]) for i in range(k)}


@dataclass
class Graph:
    params: rhg_params
    row_ptr: object
    col_idx: object
    r: object
    theta: object

    @property
    def n(self):
        return self.params.n

    @property
    def nnz(self):
        return self.col_idx.numel()


def rhg_generate(n: int, avg_degree: float, gamma: float, seed: int, tuning: Optional[dict] = None,
                 canonical_rows: bool = False, device="cuda", stream=None) -> Graph:
    """Algorithm 1 end to end on the GPU; device memory from PyTorch."""
    import torch
    held = {}

    def _alloc(nbytes, _ctx):
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        held[t.data_ptr()] = t
        return t.data_ptr()

    cb = ALLOC_FN(_alloc)
    out = rhg_csr()
    _check(load().rhg_generate(n, avg_degree, gamma, seed, _tuning(tuning), cb, None,
                               1 if canonical_rows else 0, C.byref(out), _stream(stream)))

    def view(ptr, dtype, count):
        return held[ptr][: count * torch.empty((), dtype=dtype).element_size()].view(dtype)

    return Graph(params=out.params,
                 row_ptr=view(out.row_ptr, torch.int64, n + 1),
                 col_idx=view(out.col_idx, torch.int32, out.nnz),
                 r=view(out.r, torch.float64, n), theta=view(out.theta, torch.float64, n))


def rhg_temp_count_edges(idx: Index, T: float, row_ptr, stream=None):
    """Temperature model, count pass: row_ptr (device int64, n + 1)."""
    import torch
    assert row_ptr.dtype == torch.int64 and row_ptr.numel() >= idx.params.n + 1
    _check(load().rhg_temp_count_edges(idx.handle, float(T), _ptr(row_ptr), _stream(stream)))


def rhg_temp_emit_edges(idx: Index, T: float, row_ptr, col_idx, canonical_rows: bool = False, stream=None):
    import torch
    assert col_idx.dtype == torch.int32
    _check(load().rhg_temp_emit_edges(idx.handle, float(T), _ptr(row_ptr), _ptr(col_idx), col_idx.numel(),
                                      1 if canonical_rows else 0, _stream(stream)))


def rhg_temp_generate(n: int, avg_degree: float, gamma: float, T: float, seed: int,
                      tuning: Optional[dict] = None, canonical_rows: bool = False, device="cuda",
                      stream=None) -> Graph:
    """The temperature model end to end on the GPU; device memory from PyTorch."""
    import torch
    held = {}

    def _alloc(nbytes, _ctx):
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        held[t.data_ptr()] = t
        return t.data_ptr()

    cb = ALLOC_FN(_alloc)
    out = rhg_csr()
    _check(load().rhg_temp_generate(n, avg_degree, gamma, float(T), seed, _tuning(tuning), cb, None,
                                    1 if canonical_rows else 0, C.byref(out), _stream(stream)))

    def view(ptr, dtype, count):
        return held[ptr][: count * torch.empty((), dtype=dtype).element_size()].view(dtype)

    return Graph(params=out.params,
                 row_ptr=view(out.row_ptr, torch.int64, n + 1),
                 col_idx=view(out.col_idx, torch.int32, out.nnz),
                 r=view(out.r, torch.float64, n), theta=view(out.theta, torch.float64, n))


def rhg_generate_async(p: rhg_params, r, theta, workspace, row_ptr, col_idx, overflow, tuning=None, stream=None):
    """Whole pipeline into caller buffers; asynchronous and capturable."""
    _check(load().rhg_generate_async(C.byref(p), _tuning(tuning), _ptr(r), _ptr(theta), _ptr(workspace),
                                     workspace.numel(), _ptr(row_ptr), _ptr(col_idx), col_idx.numel(),
                                     _ptr(overflow), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # RHG_NOALLOC_SCRATCH_BYTES


def rhg_generate_async_noalloc(p: rhg_params, r, theta, row_ptr, col_idx, overflow, tuning=None, stream=None):
    """rhg_generate_async with the library's own per-GPU workspace (no
    device allocation; calls on one GPU must not overlap)."""
    _check(load().rhg_generate_async_noalloc(C.byref(p), _tuning(tuning), _ptr(r), _ptr(theta), _ptr(row_ptr),
                                             _ptr(col_idx), col_idx.numel(), _ptr(overflow), _stream(stream)))


class DeviceView:
    """A device array owned by the library, seen as a torch tensor (no copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr or 0), False),
                                         "version": 3, "strides": None}


def _view(ptr, n, typestr):
    import torch
    if n <= 0 or not ptr:
        dt = {"<i8": torch.int64, "<i4": torch.int32, "<f8": torch.float64}[typestr]
        return torch.empty(0, dtype=dt, device="cuda")
    return torch.as_tensor(DeviceView(ptr, n, typestr), device="cuda")


class DynGraph:
    """The dynamic model (rhg_dyn_*): a graph whose vertices move.  move()
    applies a batch of (id, r, theta) moves; graph() gives device views of
    the current CSR (ascending rows) and points, valid until the next move."""

    def __init__(self, p: rhg_params, r, theta, tuning: Optional[dict] = None, stream=None):
        self.handle = C.c_void_p()
        self.params = p
        _check(load().rhg_dyn_create(C.byref(p), _tuning(tuning), _ptr(r), _ptr(theta), C.byref(self.handle),
                                     _stream(stream)))

    def move(self, ids, r, theta, stream=None):
        import torch
        assert ids.dtype == torch.int32 and r.dtype == torch.float64 and theta.dtype == torch.float64
        k = ids.numel()
        assert r.numel() == k and theta.numel() == k
        _check(load().rhg_dyn_move(self.handle, k, _ptr(ids), _ptr(r), _ptr(theta), _stream(stream)))

    def graph(self) -> Graph:
        out = rhg_csr()
        _check(load().rhg_dyn_graph(self.handle, C.byref(out)))
        n = out.n
        return Graph(params=out.params, row_ptr=_view(out.row_ptr, n + 1, "<i8"),
                     col_idx=_view(out.col_idx, out.nnz, "<i4"), r=_view(out.r, n, "<f8"),
                     theta=_view(out.theta, n, "<f8"))

    def set_regenerate_share(self, share: float):
        """Batches with k (1 + mean degree) above share * n are applied by
        regeneration (0: always; a huge share: never)."""
        _check(load().rhg_dyn_set_regenerate_share(self.handle, float(share)))

    def last_step(self) -> dict:
        a, b = C.c_int64(), C.c_int64()
        _check(load().rhg_dyn_last_step(self.handle, C.byref(a), C.byref(b)))
        return {"changed_rows": a.value, "moved_entries": b.value}

    def close(self):
        if self.handle:
            load().rhg_dyn_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RhgServer:
    """The library's request server (rhg_server_*): continuous batching with
    its own device arena and streams.  submit() queues a request, poll()
    collects finished ones (as dicts holding device views of the CSR, valid
    until release())."""

    def __init__(self, budget_bytes: int, slots: int = 16):
        lib = load()
        h = C.c_void_p()
        _check(lib.rhg_server_create(int(budget_bytes), int(slots), C.byref(h)))
        self._h = h
        self._buf = (rhg_completion * 64)()

    def submit(self, req_id: int, n: int, avg_degree: float, gamma: float, seed: int, tuning=None):
        _check(load().rhg_server_submit(self._h, int(req_id), int(n), float(avg_degree), float(gamma), int(seed),
                                        _tuning(tuning)))

    def poll(self):
        lib = load()
        out = []
        while True:
            cnt = C.c_int(0)
            _check(lib.rhg_server_poll(self._h, self._buf, len(self._buf), C.byref(cnt)))
            for i in range(cnt.value):
                c = self._buf[i]
                d = {"req_id": c.req_id, "status": c.status, "n": c.n, "nnz": c.nnz,
                     "latency_ms": c.latency_ms, "params": rhg_params.from_buffer_copy(c.params)}
                if c.status == RHG_OK:
                    d["row_ptr"] = _view(c.row_ptr, c.n + 1, "<i8")
                    d["col_idx"] = _view(c.col_idx, c.nnz, "<i4")
                    d["r"] = _view(c.r, c.n, "<f8")
                    d["theta"] = _view(c.theta, c.n, "<f8")
                out.append(d)
            if cnt.value < len(self._buf):
                return out

    def release(self, req_id: int):
        _check(load().rhg_server_release(self._h, int(req_id)))

    def stats(self) -> dict:
        st = rhg_server_stats()
        _check(load().rhg_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in rhg_server_stats._fields_}

    def close(self):
        if self._h:
            load().rhg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def expected_col_capacity(p: rhg_params, slack: float = 1.3) -> int:
    """int32 slots to reserve for col_idx before counting: 2m in expectation
    (the target degree times n), with slack for the spread of the degree."""
    k = p.avg_degree if p.avg_degree == p.avg_degree else 16.0
    return int(p.n * k * slack) + 4096


class GraphBuffers:
    """Device buffers of one graph for rhg_generate_async / batches."""

    def __init__(self, p: rhg_params, tuning=None, col_capacity=None, device="cuda"):
        import torch
        n = max(int(p.n), 1)
        self.params = p
        self.tuning = tuning
        self.r = torch.empty(n, dtype=torch.float64, device=device)
        self.theta = torch.empty(n, dtype=torch.float64, device=device)
        self.ws = torch.empty(rhg_index_workspace_bytes(p, tuning), dtype=torch.uint8, device=device)
        self.row_ptr = torch.empty(int(p.n) + 1, dtype=torch.int64, device=device)
        cap = expected_col_capacity(p) if col_capacity is None else int(col_capacity)
        self.col = torch.empty(max(cap, 1), dtype=torch.int32, device=device)

    def graph(self) -> "Graph":
        nnz = int(self.row_ptr[-1].item())
        return Graph(params=self.params, row_ptr=self.row_ptr, col_idx=self.col[:nnz], r=self.r[:self.params.n],
                     theta=self.theta[:self.params.n])


class Batch:
    """Many graphs captured into one HIP graph (rhg_batch_create); launch()
    runs the whole batch as one submission."""

    def __init__(self, bufs, n_streams: int = 64):
        import torch
        self.bufs = bufs
        k = len(bufs)
        self.overflow = torch.zeros(max(k, 1), dtype=torch.int32, device=bufs[0].r.device if k else "cuda")
        ps = (rhg_params * k)(*[b.params for b in bufs])
        tus = (rhg_tuning * k)()
        for i, b in enumerate(bufs):
            if b.tuning:
                t = _tuning(b.tuning)._obj
                tus[i] = t
        arr = lambda vals, T: (T * k)(*vals)
        # the captured graph holds raw pointers: keep every buffer it writes
        # alive for the batch's lifetime, also after fix_overflows swaps col
        self._keep = (ps, tus, [(b.r, b.theta, b.ws, b.row_ptr, b.col) for b in bufs])
        self.capacity = [b.col.numel() for b in bufs]  # col_idx slots the graph was captured with
        h = C.c_void_p()
        _check(load().rhg_batch_create(
            k, ps, tus, arr([b.r.data_ptr() for b in bufs], C.c_void_p),
            arr([b.theta.data_ptr() for b in bufs], C.c_void_p), arr([b.ws.data_ptr() for b in bufs], C.c_void_p),
            arr([b.ws.numel() for b in bufs], C.c_size_t), arr([b.row_ptr.data_ptr() for b in bufs], C.c_void_p),
            arr([b.col.data_ptr() for b in bufs], C.c_void_p), arr([b.col.numel() for b in bufs], C.c_int64),
            _ptr(self.overflow), n_streams, C.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(load().rhg_batch_launch(self.handle, _stream(stream)))

    def fix_overflows(self, stream=None):
        """Re-run, with exact capacity, any graph whose col_idx was too small
        (its flag is set; its row_ptr is complete).  The graph keeps writing
        the original buffer on later launches, so call this after each."""
        import torch
        torch.cuda.synchronize()
        flags = self.overflow[:len(self.bufs)].cpu()
        broken = torch.nonzero(flags & 2).flatten().tolist()
        if broken:
            raise RhgError(RHG_EINTERNAL, "emit pass disagreed with the count pass for graphs %s" % broken)
        bad = torch.nonzero(flags & 1).flatten().tolist()
        for i in bad:
            b = self.bufs[i]
            b.col = torch.empty(int(b.row_ptr[-1].item()), dtype=torch.int32, device=b.r.device)
            flag = torch.zeros(1, dtype=torch.int32, device=b.r.device)
            rhg_generate_async(b.params, b.r, b.theta, b.ws, b.row_ptr, b.col, flag, tuning=b.tuning, stream=stream)
            torch.cuda.synchronize()
            if int(flag.item()) != 0:
                raise RhgError(RHG_EINTERNAL, "refill of graph %d reported flag %d" % (i, int(flag.item())))
        return bad

    def destroy(self):
        if self.handle:
            load().rhg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


__all__ = ["rhg_plan", "rhg_plan_radius", "rhg_sample_points", "rhg_index_workspace_bytes",
           "rhg_build_index", "rhg_count_edges", "rhg_emit_edges", "rhg_sort_rows",
           "rhg_sort_rows_workspace_bytes", "rhg_long_range", "rhg_long_range_workspace_bytes",
           "long_range_count", "rhg_graph_stats", "rhg_graph_stats_workspace_bytes", "rhg_index_stats",
           "rhg_generate",
           "rhg_set_profiling", "rhg_phase_times", "rhg_generate_async", "rhg_generate_async_noalloc",
           "GraphBuffers", "Batch", "RhgServer",
           "expected_col_capacity", "RhgError", "Graph", "Index", "load", "version",
           "LIB_PATH", "PHASES"]
