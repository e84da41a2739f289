"""MI355X (gfx950) sketch-based facility location on graphs.

Python front of the HIP library ``libfl.so`` (C ABI in include/fl.h), after
"Scalable Facility Location for Massive Graphs on Pregel-like Systems"
(arXiv 1503.03635).  The functions here only marshal arguments: graphs are
moved to the GPU as torch tensors, their pointers go through the C ABI, and
the results come back as tensors and host scalars.
"""
import ctypes as C
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import (FL_FLAG_DIRECTED, FL_FLAG_LUBY_MIS, FL_FLAG_NO_DENSE, FL_NONE, FL_NOT_FACILITY, FL_RUNG_END, FL_RUNG_GUARD,
                   FL_RUNG_NONE, FlError, lib)

__all__ = ["DeviceGraph", "to_device", "solve", "solve_static", "release_workspace", "solve_batch", "Server", "ads_build", "rank_of", "priority_of",
           "use_torch_allocator",
           "FlError", "FL_NONE", "FL_NOT_FACILITY", "FL_RUNG_NONE", "FL_RUNG_GUARD", "FL_RUNG_END",
           "FL_FLAG_NO_DENSE", "FL_FLAG_LUBY_MIS", "FL_FLAG_DIRECTED", "lib"]


@dataclass
class DeviceGraph:
    n: int
    row_ptr: torch.Tensor                 # int64 [n+1] (read as uint64)
    col: torch.Tensor                     # int32 [m]   (read as uint32)
    w: Optional[torch.Tensor] = None      # int32 [m]
    fac_cost: Optional[torch.Tensor] = None   # int32 [n] (read as uint32)
    is_client: Optional[torch.Tensor] = None  # uint8 [n]
    directed: bool = False                # rows are out-arcs: FL_FLAG_DIRECTED is added to the flags

    @property
    def n_arcs(self):
        return int(self.col.numel())


def _t(a, dtype, device):
    import numpy as np
    if a is None:
        return None
    arr = np.ascontiguousarray(a)
    return torch.from_numpy(arr.view(dtype)).to(device)


def to_device(g, device="cuda") -> DeviceGraph:
    """Copy a host graph (numpy arrays: row_ptr uint64, col/w/fac_cost uint32,
    is_client uint8) to device tensors with the same bit patterns."""
    import numpy as np
    return DeviceGraph(
        n=int(g.n),
        row_ptr=_t(np.asarray(g.row_ptr, np.uint64), np.int64, device),
        col=_t(np.asarray(g.col, np.uint32), np.int32, device),
        w=None if g.w is None else _t(np.asarray(g.w, np.uint32), np.int32, device),
        fac_cost=None if getattr(g, "fac_cost", None) is None else
        _t(np.asarray(g.fac_cost, np.uint32), np.int32, device),
        is_client=None if getattr(g, "is_client", None) is None else
        _t(np.asarray(g.is_client, np.uint8), np.uint8, device),
        directed=bool(getattr(g, "directed", False)),
    )


def _flags(dg: DeviceGraph, flags: int) -> int:
    return flags | (_lib.FL_FLAG_DIRECTED if dg.directed else 0)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _problem(dg: DeviceGraph):
    return _lib.FlProblem(dg.n, dg.n_arcs, _ptr(dg.row_ptr), _ptr(dg.col), _ptr(dg.w),
                          _ptr(dg.fac_cost), _ptr(dg.is_client))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _alloc_outputs(n, device, diagnostics):
    out = {
        "open": torch.empty(n, dtype=torch.uint8, device=device),
        "assign": torch.empty(n, dtype=torch.int32, device=device),
        "dist": torch.empty(n, dtype=torch.int32, device=device),
    }
    if diagnostics:
        out["open_rung"] = torch.empty(n, dtype=torch.int32, device=device)
        out["freeze_rung"] = torch.empty(n, dtype=torch.int32, device=device)
        out["q"] = torch.empty(n, dtype=torch.float64, device=device)
    return out


def _result_struct(out):
    return _lib.FlResult(_ptr(out["open"]), _ptr(out["assign"]), _ptr(out["dist"]),
                         _ptr(out.get("open_rung")), _ptr(out.get("freeze_rung")), _ptr(out.get("q")))


def _collect(res, out):
    st = res.stats
    out["status"] = int(res.status)
    out["total_cost"] = int(res.total_cost)
    out["n_open"] = int(res.n_open)
    out["n_unreachable"] = int(res.n_unreachable)
    out["stats"] = {name: getattr(st, name) for name, _ in _lib.FlStats._fields_}
    return out


def _solve_with(fn, name, dg, k, seed, eps, flags, diagnostics, stream, outputs, check):
    device = dg.col.device if dg.n_arcs else dg.row_ptr.device
    out = outputs if outputs is not None else _alloc_outputs(dg.n, device, diagnostics)
    prob = _problem(dg)
    prm = _lib.FlParams(k, seed, eps, _flags(dg, flags))
    res = _result_struct(out)
    rc = fn(C.byref(prob), C.byref(prm), C.byref(res), C.c_void_p(_stream_ptr(stream)))
    out["rc"] = rc
    if rc != _lib.FL_OK:
        if check:
            raise FlError(rc, name)
        return out
    return _collect(res, out)


def solve(dg: DeviceGraph, k: int, seed: int, eps: float = 0.1, flags: int = 0,
          diagnostics: bool = False, stream=None, outputs=None, check=True):
    """One facility-location solve (fl_solve).  Returns a dict of device
    tensors (open, assign, dist[, open_rung, freeze_rung, q]) and host scalars
    (total_cost, n_open, n_unreachable, stats)."""
    return _solve_with(lib().fl_solve, "fl_solve", dg, k, seed, eps, flags, diagnostics, stream, outputs, check)


def solve_static(dg: DeviceGraph, k: int, seed: int, eps: float = 0.1, flags: int = 0,
                 diagnostics: bool = False, stream=None, outputs=None, check=True):
    """fl_solve_static: the same solve with the workspace in the library's
    fixed device array (no device allocation by the library; pass `outputs`
    to keep the call free of torch allocations too)."""
    return _solve_with(lib().fl_solve_static, "fl_solve_static", dg, k, seed, eps, flags, diagnostics, stream,
                       outputs, check)


def solve_batch(dgs, k, seed, eps=0.1, flags=0, diagnostics=False, stream=None, check=True, outputs=None):
    """fl_solve_batch over a list of device graphs; one dict per graph.  k,
    seed, eps and flags are scalars or per-graph sequences.  Each dict holds
    the element's own status (0 = FL_OK); with check=True any failing element
    raises."""
    count = len(dgs)

    def per(x):
        return list(x) if isinstance(x, (list, tuple)) else [x] * count
    ks, seeds, epss, flagss = per(k), per(seed), per(eps), per(flags)
    probs = (_lib.FlProblem * count)(*[_problem(d) for d in dgs])
    prms = (_lib.FlParams * count)(*[_lib.FlParams(ks[i], seeds[i], epss[i], _flags(dgs[i], flagss[i]))
                                     for i in range(count)])
    outs = outputs if outputs is not None else [
        _alloc_outputs(d.n, d.col.device if d.n_arcs else d.row_ptr.device, diagnostics) for d in dgs]
    ress = (_lib.FlResult * count)(*[_result_struct(o) for o in outs])
    rc = lib().fl_solve_batch(probs, prms, ress, count, C.c_void_p(_stream_ptr(stream)))
    for i in range(count):
        _collect(ress[i], outs[i])
        outs[i]["rc"] = outs[i]["status"]
    if rc != _lib.FL_OK and check:
        raise FlError(rc, "fl_solve_batch")
    return outs


class Server:
    """Continuous-batching solve server (fl_server_*): submit() queues a
    request and returns a ticket; wait()/poll() return the result dict.  The
    request's structs and output tensors are kept alive here until then."""

    def __init__(self, hbm_budget_bytes: int = 0, slots: int = 0):
        h = C.c_void_p()
        rc = lib().fl_server_create(hbm_budget_bytes, slots, C.byref(h))
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_server_create")
        self._h = h
        self._live = {}
        import threading
        self._lock = threading.Lock()

    def submit(self, dg: DeviceGraph, k: int, seed: int, eps: float = 0.1, flags: int = 0,
               diagnostics: bool = False, outputs=None) -> int:
        device = dg.col.device if dg.n_arcs else dg.row_ptr.device
        out = outputs if outputs is not None else _alloc_outputs(dg.n, device, diagnostics)
        torch.cuda.synchronize(device)  # inputs and outputs ready before another stream reads them
        prob = _problem(dg)
        prm = _lib.FlParams(k, seed, eps, _flags(dg, flags))
        res = _result_struct(out)
        t = C.c_uint64()
        rc = lib().fl_server_submit(self._h, C.byref(prob), C.byref(prm), C.byref(res), C.byref(t))
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_server_submit")
        with self._lock:
            self._live[t.value] = (dg, prob, prm, res, out)
        return t.value

    def _finish(self, ticket, st):
        with self._lock:
            dg, prob, prm, res, out = self._live.pop(ticket)
        out["rc"] = st
        _collect(res, out)
        return out

    def wait(self, ticket: int):
        st = C.c_int()
        rc = lib().fl_server_wait(self._h, ticket, C.byref(st))
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_server_wait")
        return self._finish(ticket, st.value)

    def poll(self, ticket: int):
        """The result dict when finished, else None."""
        st = C.c_int()
        rc = lib().fl_server_poll(self._h, ticket, C.byref(st))
        if rc == _lib.FL_EBUSY:
            return None
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_server_poll")
        return self._finish(ticket, st.value)

    def close(self):
        if self._h:
            lib().fl_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


_hooks = None  # the registered callbacks (kept alive while the library may call them)


def use_torch_allocator(enable: bool = True):
    """Back the library's device workspace and sketch handles with torch's
    caching allocator (fl_set_allocator), or go back to hipMalloc/hipFree.
    Not while a Server exists or a call is running."""
    global _hooks
    L = lib()
    if not enable:
        rc = L.fl_set_allocator(None, None, None)
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_set_allocator")
        _hooks = None
        return

    def _alloc(nbytes, device, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device))
        except Exception:  # out of memory: the library reports FL_ENOMEM
            return None

    def _free(ptr, nbytes, device, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    rc = L.fl_set_allocator(C.cast(hooks[0], C.c_void_p), C.cast(hooks[1], C.c_void_p), None)
    if rc != _lib.FL_OK:
        raise FlError(rc, "fl_set_allocator")
    _hooks = hooks


def release_workspace():
    """fl_release_workspace: frees the library's cached workspaces on the
    current device."""
    lib().fl_release_workspace()


def ads_build(dg: DeviceGraph, k: int, seed: int, flags: int = 0, stream=None):
    """Bottom-k sketches of every vertex (fl_ads_build), copied into fresh
    device tensors: off int64 [n+1], rank/dist/thresh int32 [total]."""
    prob = _problem(dg)
    prm = _lib.FlParams(k, seed, 0.1, _flags(dg, flags))
    h = C.c_void_p()
    rc = lib().fl_ads_build(C.byref(prob), C.byref(prm), C.byref(h), C.c_void_p(_stream_ptr(stream)))
    if rc != _lib.FL_OK:
        raise FlError(rc, "fl_ads_build")
    try:
        v = _lib.FlSketchView()
        rc = lib().fl_sketch_view(h, C.byref(v))
        if rc != _lib.FL_OK:
            raise FlError(rc, "fl_sketch_view")
        device = dg.row_ptr.device
        n, tot = int(v.n), int(v.total)
        off = torch.empty(n + 1, dtype=torch.int64, device=device)
        rank = torch.empty(tot, dtype=torch.int32, device=device)
        dist = torch.empty(tot, dtype=torch.int32, device=device)
        thr = torch.empty(tot, dtype=torch.int32, device=device)
        torch.cuda.synchronize(device)
        for dst, src, nbytes in ((off, v.off, (n + 1) * 8), (rank, v.rank, tot * 4),
                                 (dist, v.dist, tot * 4), (thr, v.thresh, tot * 4)):
            if nbytes:
                _memcpy_d2d(dst.data_ptr(), src, nbytes)
        torch.cuda.synchronize(device)
        return {"off": off, "rank": rank, "dist": dist, "thresh": thr, "total": tot}
    finally:
        lib().fl_sketch_free(h)


_hip = None


def _memcpy_d2d(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime (hipMemcpy)."""
    global _hip
    if _hip is None:
        # by soname: the runtime already loaded in this process (torch's or
        # the one libfl.so bound to), never a second copy
        lib()
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed: {rc}")


def rank_of(v: int, seed: int) -> int:
    return int(lib().fl_rank_of(v, seed))


def priority_of(v: int, seed: int) -> int:
    return int(lib().fl_priority_of(v, seed))
