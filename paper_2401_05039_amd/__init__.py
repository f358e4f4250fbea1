"""MI355X maximal biclique enumeration: Python binding of ``libmbe.so``.

The functions here only marshal arguments to the C interface declared in
``include/mbe.h``; every step of the enumeration runs in the library's HIP kernels.
Graphs are passed as two sorted CSR arrays (see ``include/mbe.h``); host arrays (numpy)
are copied by the library, device arrays (torch tensors on a HIP device) are used in place.

The library must be built first (``python -m paper_2401_05039_amd.build`` or
``__graft_entry__.build()``); importing the binding fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Any, Dict, List, Optional, Tuple

import numpy as np

__all__ = ["mbe_count", "mbe_count_loads", "mbe_count_noalloc", "mbe_count_batch", "mbe_enumerate", "mbe_strerror", "mbe_version", "MbeError",
           "Options", "Server", "lib_path", "load"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# (MBE_LIB: another build of the same library, e.g. the sanitized host build of the CPU tests)
_LIB_PATH = os.environ.get("MBE_LIB") or os.path.join(_HERE, "libmbe.so")
_lib = None

MBE_OK = 0
MBE_ERR_INVALID_ARG = -1
MBE_ERR_INVALID_GRAPH = -2
MBE_ERR_BUFFER_TOO_SMALL = -3
MBE_ERR_OUT_OF_MEMORY = -4
MBE_ERR_DEVICE = -5
MBE_ERR_UNSUPPORTED = -6
MBE_ERR_SCRATCH_LIMIT = -7
MBE_ERR_TIMEOUT = -8
MBE_ERR_CANCELLED = -9
MBE_NOALLOC_SCRATCH_BYTES = 256 << 20
MBE_MAX_DEGREE = 1024


class _Graph(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("u_off", ctypes.c_void_p), ("u_adj", ctypes.c_void_p),
                ("v_off", ctypes.c_void_p), ("v_adj", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("hash", ctypes.c_uint64), ("out_ints", ctypes.c_uint64),
                ("nodes", ctypes.c_uint64), ("nonmaximal", ctypes.c_uint64),
                ("bytes_alg", ctypes.c_uint64), ("max_depth", ctypes.c_uint32),
                ("side", ctypes.c_uint32), ("kernel_ms", ctypes.c_double),
                ("phase_cycles", ctypes.c_uint64 * 6), ("shared_chunks", ctypes.c_uint64),
                ("attempts", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("bytes_design", ctypes.c_uint64)]


class _Options(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("wg_waves", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("diagnostics", ctypes.c_int32), ("no_validate", ctypes.c_int32),
                ("steal_k", ctypes.c_int32), ("root_lo", ctypes.c_int64),
                ("root_hi", ctypes.c_int64), ("stream", ctypes.c_void_p), ("prune", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64)]


@dataclasses.dataclass
class Options:
    """Mirror of ``mbe_options``; zero means default."""
    side: int = 0
    wg_waves: int = 0
    grid: int = 0
    diagnostics: int = 0  # 1: the method's tree tallies; 2: the production search's design bytes
    no_validate: bool = False
    steal_k: int = 0
    root_lo: int = 0
    root_hi: int = 0
    stream: Optional[int] = None  # hipStream_t as an integer; None = torch's current stream
    # pruning of section II-C (the same answer, the pruned tree's tallies): 0 / False none,
    # 1 / True iMBEA's candidate pruning, 2 the pivot rule
    prune: int = 0
    # mbe_count only: device memory of the caller (a torch tensor, or an address with
    # workspace_bytes) that every device buffer of the call is carved from
    workspace: Any = None
    workspace_bytes: int = 0


class _ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("small_edges", ctypes.c_int64), ("search", _Options), ("request_timeout_ms", ctypes.c_double)]


class MbeError(RuntimeError):
    def __init__(self, code: int, result: Optional[Dict[str, Any]] = None):
        super().__init__(f"mbe error {code}: {mbe_strerror(code)}")
        self.code = code
        self.result = result


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libmbe.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2401_05039_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.mbe_count.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Result)]
    lib.mbe_count.restype = ctypes.c_int
    lib.mbe_count_loads.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Result),
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.mbe_count_loads.restype = ctypes.c_int
    lib.mbe_count_noalloc.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Result)]
    lib.mbe_count_noalloc.restype = ctypes.c_int
    lib.mbe_workspace_size.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_size_t)]
    lib.mbe_workspace_size.restype = ctypes.c_int
    lib.mbe_enumerate.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Result),
                                  ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32]
    lib.mbe_enumerate.restype = ctypes.c_int
    lib.mbe_count_batch.argtypes = [ctypes.POINTER(_Graph), ctypes.c_int32, ctypes.POINTER(_Options),
                                     ctypes.POINTER(_Result)]
    lib.mbe_count_batch.restype = ctypes.c_int
    lib.mbe_tune_batch.argtypes = [ctypes.POINTER(_Graph), ctypes.c_int32, ctypes.POINTER(_Options),
                                   ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_double)]
    lib.mbe_tune_batch.restype = ctypes.c_int
    lib.mbe_server_create.argtypes = [ctypes.POINTER(_ServerOptions), ctypes.POINTER(ctypes.c_void_p)]
    lib.mbe_server_create.restype = ctypes.c_int
    lib.mbe_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Graph), ctypes.POINTER(ctypes.c_uint64)]
    lib.mbe_server_submit.restype = ctypes.c_int
    lib.mbe_server_submit_timeout.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Graph), ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_uint64)]
    lib.mbe_server_submit_timeout.restype = ctypes.c_int
    lib.mbe_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.mbe_server_cancel.restype = ctypes.c_int
    lib.mbe_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(_Result),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.mbe_server_wait.restype = ctypes.c_int
    lib.mbe_server_destroy.argtypes = [ctypes.c_void_p]
    lib.mbe_server_destroy.restype = ctypes.c_int
    lib.mbe_strerror.argtypes = [ctypes.c_int]
    lib.mbe_strerror.restype = ctypes.c_char_p
    lib.mbe_version.argtypes = []
    lib.mbe_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def mbe_strerror(code: int) -> str:
    return load().mbe_strerror(int(code)).decode()


def mbe_version() -> str:
    return load().mbe_version().decode()


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _marshal_graph(g) -> Tuple[_Graph, List[Any]]:
    """Build the C struct; keeps references to the arrays alive in the returned list."""
    arrs = [g.u_off, g.u_adj, g.v_off, g.v_adj]
    on_dev = all(_is_torch(a) and a.is_cuda for a in arrs)
    keep: List[Any] = []
    ptrs = []
    if on_dev:
        import torch
        for a in arrs:
            if a.dtype != torch.int32 or not a.is_contiguous():
                a = a.to(torch.int32).contiguous()
            keep.append(a)
            ptrs.append(a.data_ptr())
    else:
        for a in arrs:
            if _is_torch(a):
                a = a.cpu().numpy()
            a = np.ascontiguousarray(a, dtype=np.int32)
            keep.append(a)
            ptrs.append(a.ctypes.data)
    n_edges = int(keep[1].shape[0]) if hasattr(keep[1], "shape") else len(keep[1])
    cg = _Graph(int(g.n_u), int(g.n_v), n_edges, *[ctypes.c_void_p(p) for p in ptrs], 1 if on_dev else 0)
    return cg, keep


def _marshal_opts(opt: Optional[Options], on_device: bool) -> _Options:
    opt = opt or Options()
    stream = opt.stream
    if stream is None and on_device:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    ws, ws_bytes = opt.workspace, int(opt.workspace_bytes)
    if ws is not None and not isinstance(ws, int):  # a tensor: its device memory
        ws_bytes = ws_bytes or int(ws.numel()) * int(ws.element_size())
        ws = int(ws.data_ptr())
    return _Options(opt.side, opt.wg_waves, opt.grid, int(opt.diagnostics), int(bool(opt.no_validate)),
                    opt.steal_k, opt.root_lo, opt.root_hi, ctypes.c_void_p(stream or 0), int(opt.prune),
                    ctypes.c_void_p(ws or 0), ws_bytes)


PHASES = ("root", "light", "check", "expand", "child", "wait")


def _result_dict(r: _Result) -> Dict[str, Any]:
    d = {k: getattr(r, k) for k, _ in _Result._fields_ if k != "phase_cycles"}
    d["phase_cycles"] = dict(zip(PHASES, list(r.phase_cycles)))
    return d


def mbe_count(g, opt: Optional[Options] = None) -> Dict[str, Any]:
    """Count and hash the maximal bicliques of g; returns the fields of ``mbe_result``."""
    lib = load()
    cg, keep = _marshal_graph(g)
    co = _marshal_opts(opt, bool(cg.on_device))
    res = _Result()
    rc = lib.mbe_count(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(res))
    if rc != MBE_OK:
        raise MbeError(rc, _result_dict(res))
    return _result_dict(res)


def mbe_count_loads(g, opt: Optional[Options] = None, cap: int = 1 << 16) -> Tuple[Dict[str, Any], np.ndarray]:
    """``mbe_count`` with the design-byte tally, and one load record per workgroup of every
    search launch: an (n, 4) uint64 array of (mask words of its class, 0 = wide search;
    start ns; end ns; ns spent finding work)."""
    lib = load()
    cg, keep = _marshal_graph(g)
    co = _marshal_opts(opt, bool(cg.on_device))
    res = _Result()
    rec = np.zeros((max(1, cap), 4), dtype=np.uint64)
    n = ctypes.c_int64(0)
    rc = lib.mbe_count_loads(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(res), ctypes.c_void_p(rec.ctypes.data),
                             ctypes.c_int64(cap), ctypes.byref(n))
    if rc != MBE_OK:
        raise MbeError(rc, _result_dict(res))
    return _result_dict(res), rec[:n.value].copy()


def mbe_count_noalloc(g, opt: Optional[Options] = None) -> Dict[str, Any]:
    """``mbe_count`` without any device allocation: the call's buffers come from the library's
    fixed per-device scratch (``MBE_NOALLOC_SCRATCH_BYTES``); raises MbeError with
    ``MBE_ERR_SCRATCH_LIMIT`` when the graph needs more."""
    lib = load()
    cg, keep = _marshal_graph(g)
    co = _marshal_opts(opt, bool(cg.on_device))
    res = _Result()
    rc = lib.mbe_count_noalloc(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(res))
    if rc != MBE_OK:
        raise MbeError(rc, _result_dict(res))
    return _result_dict(res)


def mbe_workspace_size(g, opt: Optional[Options] = None) -> int:
    """Device bytes a ``mbe_count`` of g with these options holds (preparation runs, no search)."""
    lib = load()
    cg, keep = _marshal_graph(g)
    co = _marshal_opts(opt, bool(cg.on_device))
    out = ctypes.c_size_t(0)
    rc = lib.mbe_workspace_size(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(out))
    if rc != MBE_OK:
        raise MbeError(rc, {})
    return int(out.value)


def _marshal_batch(graphs):
    n = len(graphs)
    arr = (_Graph * max(1, n))()
    keep: List[Any] = []
    for i, g in enumerate(graphs):
        cg, k = _marshal_graph(g)
        if cg.on_device:
            raise ValueError("batched calls take host graphs")
        arr[i] = cg
        keep.append(k)
    return arr, keep


def mbe_tune_batch(graphs, opt: Optional[Options] = None):
    """Autotune the batched form on a sample of graphs (``mbe_tune_batch``); returns the
    fastest Options and its wall time in milliseconds."""
    lib = load()
    arr, keep = _marshal_batch(graphs)
    co = _marshal_opts(opt, False)
    best = _Options()
    ms = ctypes.c_double(0.0)
    rc = lib.mbe_tune_batch(arr, len(graphs), ctypes.byref(co), ctypes.byref(best), ctypes.byref(ms))
    if rc != MBE_OK:
        raise MbeError(rc)
    base = opt or Options()
    tuned = dataclasses.replace(base, wg_waves=best.wg_waves, steal_k=best.steal_k)
    return tuned, ms.value


def mbe_count_batch(graphs, opt: Optional[Options] = None) -> List[Dict[str, Any]]:
    """Count and hash the maximal bicliques of many host graphs in one batched pass; returns
    one result dict per graph (kernel_ms is the time of the whole batch)."""
    lib = load()
    n = len(graphs)
    arr, keep = _marshal_batch(graphs)
    co = _marshal_opts(opt, False)
    res = (_Result * max(1, n))()
    rc = lib.mbe_count_batch(arr, n, ctypes.byref(co), res)
    if rc != MBE_OK:
        raise MbeError(rc)
    return [_result_dict(res[i]) for i in range(n)]


class Server:
    """Continuous-batching request server (``mbe_server_*``): submit host graphs from any
    thread, wait for each result; results equal those of ``mbe_count`` on the graph alone."""

    def __init__(self, hbm_budget_bytes: int = 0, slots: int = 2, max_batch: int = 0,
                 opt: Optional[Options] = None, small_edges: int = 0, request_timeout_ms: float = 0.0):
        lib = load()
        so = _ServerOptions(hbm_budget_bytes, slots, max_batch, small_edges, _marshal_opts(opt, False),
                            request_timeout_ms)
        h = ctypes.c_void_p()
        rc = lib.mbe_server_create(ctypes.byref(so), ctypes.byref(h))
        if rc != MBE_OK:
            raise MbeError(rc)
        self._h = h

    def submit(self, g, timeout_ms: Optional[float] = None) -> int:
        """Queue g; timeout_ms (None: the server's request_timeout_ms) is its deadline."""
        cg, keep = _marshal_graph(g)
        t = ctypes.c_uint64()
        if timeout_ms is None:
            rc = load().mbe_server_submit(self._h, ctypes.byref(cg), ctypes.byref(t))
        else:
            rc = load().mbe_server_submit_timeout(self._h, ctypes.byref(cg), ctypes.c_double(timeout_ms),
                                                  ctypes.byref(t))
        if rc != MBE_OK:
            raise MbeError(rc)
        return int(t.value)

    def cancel(self, ticket: int) -> None:
        rc = load().mbe_server_cancel(self._h, ctypes.c_uint64(ticket))
        if rc != MBE_OK:
            raise MbeError(rc)

    def wait(self, ticket: int) -> Tuple[Dict[str, Any], float]:
        """(result dict, latency in ms from submission to completion)."""
        res = _Result()
        lat = ctypes.c_double()
        rc = load().mbe_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(res), ctypes.byref(lat))
        if rc != MBE_OK:
            raise MbeError(rc, _result_dict(res))
        return _result_dict(res), float(lat.value)

    def close(self) -> None:
        if self._h:
            load().mbe_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def mbe_enumerate(g, opt: Optional[Options] = None, cap_ints: Optional[int] = None,
                  out=None) -> Tuple[Dict[str, Any], Any]:
    """Enumerate the maximal bicliques of g as canonical records.

    out may be a torch int32 device tensor (records are written there) or None (a host numpy
    buffer of cap_ints ints is used; when cap_ints is None the count is taken first to size
    it exactly).  Returns (result dict, record array trimmed to out_ints)."""
    lib = load()
    cg, keep = _marshal_graph(g)
    co = _marshal_opts(opt, bool(cg.on_device))
    res = _Result()
    if out is not None:
        ptr, cap, on_dev = out.data_ptr(), int(out.numel()), 1
        buf = out
    else:
        if cap_ints is None:
            rc = lib.mbe_count(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(res))
            if rc != MBE_OK:
                raise MbeError(rc, _result_dict(res))
            cap_ints = int(res.out_ints)
        buf = np.zeros(max(1, cap_ints), dtype=np.int32)
        ptr, cap, on_dev = buf.ctypes.data, int(cap_ints), 0
    rc = lib.mbe_enumerate(ctypes.byref(cg), ctypes.byref(co), ctypes.byref(res), ctypes.c_void_p(ptr),
                           ctypes.c_uint64(cap), on_dev)
    if rc != MBE_OK:
        raise MbeError(rc, _result_dict(res))
    return _result_dict(res), buf[:res.out_ints]


def decode_records(flat) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """Split a flat record array into (A, B) tuples."""
    flat = flat.tolist() if hasattr(flat, "tolist") else list(flat)
    out = []
    i = 0
    while i < len(flat):
        na, nb = flat[i], flat[i + 1]
        out.append((tuple(flat[i + 2:i + 2 + na]), tuple(flat[i + 2 + na:i + 2 + na + nb])))
        i += 2 + na + nb
    return out
