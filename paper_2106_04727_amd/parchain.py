"""ctypes binding of libparchain.so (C ABI in include/parchain.h).

Names follow the C functions. Only argument marshalling happens here: torch
provides device memory and the stream, every step of the clustering runs in
the library's HIP kernels. There is no fallback: if the library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparchain.so")

LINKAGES = {"complete": 0, "average": 1, "ward": 2, "avgsq": 3}
# element type of the screening tiles (pc_precision)
PRECISIONS = {"fp16": 0, "bf16": 1, "fp32": 2}

PC_OK = 0
STATUS = {
    0: "PC_OK",
    -1: "PC_ERR_INVALID_ARG",
    -2: "PC_ERR_NONFINITE_INPUT",
    -3: "PC_ERR_OUT_OF_MEMORY",
    -4: "PC_ERR_DEVICE",
    -5: "PC_ERR_UNSUPPORTED",
    -6: "PC_ERR_BUSY",
    -7: "PC_ERR_CANCELLED",
}


class PCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class pc_merge(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int64), ("b", ctypes.c_int64), ("height", ctypes.c_double),
                ("size", ctypes.c_int64)]


class pc_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("prune", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("cache_slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pc_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("rounds", ctypes.c_int64), ("terminals", ctypes.c_int64),
                ("cluster_evals", ctypes.c_int64), ("point_pair_evals", ctypes.c_int64),
                ("overflow_queries", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("ms_init", ctypes.c_double), ("ms_rounds", ctypes.c_double),
                ("ms_finalize", ctypes.c_double), ("kernel_ms", ctypes.c_double * 4),
                ("kernel_launches", ctypes.c_int64 * 4), ("candidate_visits", ctypes.c_int64 * 4),
                ("cache_hits", ctypes.c_int64), ("cache_inserts", ctypes.c_int64),
                ("cache_fail", ctypes.c_int64), ("cache_derived", ctypes.c_int64),
                ("refined", ctypes.c_int64), ("fp64_fallbacks", ctypes.c_int64),
                ("ms_nn", ctypes.c_double), ("ms_merge", ctypes.c_double), ("ms_update", ctypes.c_double)]

    KERNELS = ("ring_search", "block_search", "pair_tiles", "ring_emit")

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("struct_size", "reserved", "kernel_ms", "kernel_launches", "candidate_visits")}
        d["kernels"] = {k: {"ms": self.kernel_ms[i], "launches": self.kernel_launches[i],
                            "visits": self.candidate_visits[i]}
                        for i, k in enumerate(self.KERNELS)}
        return d


_lib = None
_lock = threading.Lock()

class pc_server_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("slots", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("fake_us_per_kpoint", ctypes.c_double),
                ("fake_growth", ctypes.c_double)]


class pc_request_info(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("state", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("footprint_bytes", ctypes.c_uint64), ("t_submit_ms", ctypes.c_double),
                ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("stats", pc_stats), ("error", ctypes.c_char * 120)]

    STATES = ("waiting", "running", "done", "cancelled")

    def as_dict(self):
        return {"status": self.status, "state": self.STATES[self.state], "slot": self.slot,
                "footprint_bytes": self.footprint_bytes, "t_submit_ms": self.t_submit_ms,
                "t_start_ms": self.t_start_ms, "t_done_ms": self.t_done_ms,
                "stats": self.stats.as_dict(), "error": self.error.decode(errors="replace")}


class pc_server_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("slots", ctypes.c_int32),
                ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("running", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("budget_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes_in_use", ctypes.c_uint64), ("requeued", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("struct_size", "reserved")}


EXPORTS = ["pc_context_create", "pc_context_destroy", "pc_hac_workspace_bytes", "pc_hac", "pc_hac_noalloc",
           "pc_last_error", "pc_version", "pc_server_create", "pc_server_submit", "pc_server_poll",
           "pc_server_query", "pc_server_wait", "pc_server_cancel", "pc_server_release",
           "pc_server_get_stats", "pc_server_destroy"]


def load_library(path: str | None = None):
    """Load libparchain.so (raises if it is missing: there is no fallback)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise OSError("libparchain.so not built (%s); run __graft_entry__.build()" % p)
        lib = ctypes.CDLL(p)
        vp = ctypes.c_void_p
        lib.pc_context_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
        lib.pc_context_create.restype = ctypes.c_int
        lib.pc_context_destroy.argtypes = [vp]
        lib.pc_context_destroy.restype = None
        lib.pc_hac_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp]
        lib.pc_hac_workspace_bytes.restype = ctypes.c_size_t
        lib.pc_hac.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                               vp, vp, ctypes.c_int, vp, vp]
        lib.pc_hac.restype = ctypes.c_int
        lib.pc_hac_noalloc.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        lib.pc_hac_noalloc.restype = ctypes.c_int
        lib.pc_last_error.argtypes = []
        lib.pc_last_error.restype = ctypes.c_char_p
        lib.pc_version.argtypes = []
        lib.pc_version.restype = ctypes.c_char_p
        lib.pc_server_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
        lib.pc_server_create.restype = ctypes.c_int
        lib.pc_server_submit.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                         ctypes.POINTER(ctypes.c_uint64)]
        lib.pc_server_submit.restype = ctypes.c_int
        lib.pc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), vp]
        lib.pc_server_poll.restype = ctypes.c_int
        lib.pc_server_query.argtypes = [vp, ctypes.c_uint64, vp]
        lib.pc_server_query.restype = ctypes.c_int
        lib.pc_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, vp]
        lib.pc_server_wait.restype = ctypes.c_int
        lib.pc_server_cancel.argtypes = [vp, ctypes.c_uint64]
        lib.pc_server_cancel.restype = ctypes.c_int
        lib.pc_server_release.argtypes = [vp, ctypes.c_uint64]
        lib.pc_server_release.restype = ctypes.c_int
        lib.pc_server_get_stats.argtypes = [vp, vp]
        lib.pc_server_get_stats.restype = ctypes.c_int
        lib.pc_server_destroy.argtypes = [vp]
        lib.pc_server_destroy.restype = None
        if path is None:
            _lib = lib
        return lib


def version() -> str:
    return load_library().pc_version().decode()


def _check(lib, st: int):
    if st != PC_OK:
        raise PCError(st, lib.pc_last_error().decode())


def _link(linkage) -> int:
    return LINKAGES[linkage] if isinstance(linkage, str) else int(linkage)


def _prec(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


TIME_KERNELS, TIME_PHASES = 1, 2  # pc_options.timing bits


def _timing(timing) -> int:
    """True: kernels and round phases; "kernels": the kernel events only."""
    if timing == "kernels":
        return TIME_KERNELS
    return TIME_KERNELS | TIME_PHASES if timing else 0


def _options(prune=True, timing=False, cache_slots=-1, precision="fp16") -> pc_options:
    return pc_options(ctypes.sizeof(pc_options), _prec(precision), 1 if prune else 0, _timing(timing),
                      int(cache_slots), 0)


def workspace_bytes(n: int, d: int, linkage, precision="fp16") -> int:
    opt = _options(precision=precision)
    return int(load_library().pc_hac_workspace_bytes(n, d, _link(linkage), ctypes.byref(opt)))


class Context:
    """A pc_context on one HIP device (owns the device workspace; at most
    ``hbm_budget_bytes`` of it when that is > 0)."""

    def __init__(self, device: int = -1, hbm_budget_bytes: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.pc_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pc_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hac(self, points, n: int, d: int, linkage, out, *, points_on_device: bool,
            out_on_device: bool, stream=None, prune: bool = True, stats: bool = True,
            timing: bool = False, cache_slots: int = -1, precision="fp16"):
        """Raw call: ``points``/``out`` are integer addresses."""
        opt = _options(prune, timing, cache_slots, precision)
        st = pc_stats()
        st.struct_size = ctypes.sizeof(pc_stats)
        rc = self.lib.pc_hac(self.handle, ctypes.c_void_p(points), int(n), int(d),
                             1 if points_on_device else 0, _link(linkage), ctypes.byref(opt),
                             ctypes.c_void_p(out), 1 if out_on_device else 0,
                             ctypes.c_void_p(stream or 0), ctypes.byref(st) if stats else None)
        _check(self.lib, rc)
        return st.as_dict()

    def hac_noalloc(self, points, n: int, d: int, linkage, out, *, stream=None, prune: bool = True,
                    timing: bool = False, cache_slots: int = -1, precision="fp16"):
        """pc_hac_noalloc: ``points``/``out`` are device addresses; the call
        allocates no device memory (the library's static scratch array)."""
        opt = _options(prune, timing, cache_slots, precision)
        st = pc_stats()
        st.struct_size = ctypes.sizeof(pc_stats)
        rc = self.lib.pc_hac_noalloc(self.handle, ctypes.c_void_p(points), int(n), int(d), _link(linkage),
                                     ctypes.byref(opt), ctypes.c_void_p(out), ctypes.c_void_p(stream or 0),
                                     ctypes.byref(st))
        _check(self.lib, rc)
        return st.as_dict()


_default_ctx = {}


def _ctx(device: int) -> Context:
    c = _default_ctx.get(device)
    if c is None:
        c = _default_ctx[device] = Context(device)
    return c


def hac_device(x, linkage, *, prune: bool = True, ctx: Context | None = None, stream=None,
               timing: bool = False, cache_slots: int = -1, precision="fp16"):
    """Cluster a CUDA (HIP) float32 tensor of shape (n, d) that lives on the GPU.

    Returns ``(rows, stats)``: ``rows`` is an int64 device tensor (n-1, 4)
    holding pc_merge records (a, b, height bits, size); ``rows[:, 2]``
    viewed as float64 gives the heights.
    """
    import torch

    assert x.is_cuda and x.dtype == torch.float32 and x.dim() == 2
    x = x.contiguous()
    n, d = x.shape
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    ctx = ctx or _ctx(dev)
    rows = torch.empty((max(n - 1, 1), 4), dtype=torch.int64, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream(x.device).cuda_stream
    st = ctx.hac(x.data_ptr(), n, d, linkage, rows.data_ptr(), points_on_device=True,
                 out_on_device=True, stream=stream, prune=prune, timing=timing,
                 cache_slots=cache_slots, precision=precision)
    return rows[: n - 1], st


def rows_to_Z(rows) -> np.ndarray:
    """pc_merge records (int64 (m, 4), on host or device) -> scipy Z (float64)."""
    import torch

    r = rows.cpu() if isinstance(rows, torch.Tensor) else rows
    r = np.ascontiguousarray(np.asarray(r, dtype=np.int64))
    Z = np.empty((r.shape[0], 4), np.float64)
    Z[:, 0] = r[:, 0]
    Z[:, 1] = r[:, 1]
    Z[:, 2] = r[:, 2].view(np.float64)
    Z[:, 3] = r[:, 3]
    return Z


def hac(x, linkage, *, prune: bool = True, device: int = 0, return_stats: bool = False,
        cache_slots: int = -1, precision="fp16", timing: bool = False):
    """Cluster points (numpy array or tensor, (n, d) float32) on the GPU.

    Returns the scipy-convention linkage matrix Z (float64, (n-1, 4)).
    """
    import torch

    if isinstance(x, torch.Tensor) and x.is_cuda:
        xt = x.to(torch.float32)
    else:
        xt = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:%d" % device)
    rows, st = hac_device(xt, linkage, prune=prune, cache_slots=cache_slots, precision=precision,
                          timing=timing)
    torch.cuda.synchronize(xt.device)
    Z = rows_to_Z(rows)
    return (Z, st) if return_stats else Z


class Server:
    """A pc_server: many clustering requests on one device (see parchain.h).

    ``submit`` copies nothing: the point array and the output rows are kept
    alive here until the request is released.
    """

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget_bytes: int = 0,
                 fake_us_per_kpoint: float = 0.0, fake_growth: float = 1.0):
        self.lib = load_library()
        opt = pc_server_options(ctypes.sizeof(pc_server_options), int(slots), int(hbm_budget_bytes),
                                float(fake_us_per_kpoint), float(fake_growth))
        h = ctypes.c_void_p()
        # the server runs on this context's device (none in the no-device test mode)
        self.ctx = Context(device) if fake_us_per_kpoint <= 0.0 else None
        _check(self.lib, self.lib.pc_server_create(self.ctx.handle if self.ctx else None, ctypes.byref(opt),
                                                   ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, x, linkage, *, cache_slots: int = -1, prune: bool = True, precision="fp16") -> int:
        x = np.ascontiguousarray(x, dtype=np.float32)
        n, d = x.shape
        out = np.zeros((max(n - 1, 1), 4), np.int64)
        opt = _options(prune, False, cache_slots, precision)
        t = ctypes.c_uint64()
        _check(self.lib, self.lib.pc_server_submit(self.handle, x.ctypes.data, n, d, _link(linkage),
                                                   ctypes.byref(opt), out.ctypes.data, ctypes.byref(t)))
        self._keep[t.value] = (x, out, n)
        return t.value

    def _info(self):
        info = pc_request_info()
        info.struct_size = ctypes.sizeof(pc_request_info)
        return info

    def poll(self, ticket: int) -> dict:
        """The request's full record (pc_server_query)."""
        info = self._info()
        _check(self.lib, self.lib.pc_server_query(self.handle, ticket, ctypes.byref(info)))
        return info.as_dict()

    def done(self, ticket: int):
        """(finished, status) of a request (pc_server_poll)."""
        d, r = ctypes.c_int(), ctypes.c_int()
        _check(self.lib, self.lib.pc_server_poll(self.handle, ticket, ctypes.byref(d), ctypes.byref(r), None))
        return bool(d.value), r.value

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> dict:
        info = self._info()
        _check(self.lib, self.lib.pc_server_wait(self.handle, ticket, float(timeout_ms), ctypes.byref(info)))
        return info.as_dict()

    def result(self, ticket: int, release: bool = True):
        """Wait for the request; return (Z, info); raise PCError if it failed."""
        info = self.wait(ticket)
        if info["status"] != PC_OK:
            raise PCError(info["status"], info["error"])
        _, out, n = self._keep[ticket]
        Z = rows_to_Z(out[: n - 1])
        if release:
            self.release(ticket)
        return Z, info

    def cancel(self, ticket: int):
        _check(self.lib, self.lib.pc_server_cancel(self.handle, ticket))

    def release(self, ticket: int):
        _check(self.lib, self.lib.pc_server_release(self.handle, ticket))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        st = pc_server_stats()
        st.struct_size = ctypes.sizeof(pc_server_stats)
        _check(self.lib, self.lib.pc_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pc_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()
        if getattr(self, "ctx", None):
            self.ctx.close()
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
