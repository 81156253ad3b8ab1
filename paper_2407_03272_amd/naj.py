"""Python binding of the C-ABI library libnaj.so (ctypes; argument marshalling only).

Every step of the solver runs in the library's HIP kernels.  PyTorch provides
device memory and streams: tensors are passed to the library as raw device
pointers, the current torch stream as the hipStream_t.  Names follow
include/naj.h.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import sys
import weakref
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnaj.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "naj.h")

NAJ_OK = 0
NAJ_NOT_CONVERGED = 1
NAJ_EINVAL = -1
NAJ_ENOMEM = -2
NAJ_EDEVICE = -3
NAJ_EBREAKDOWN = -4
NAJ_ECANCELLED = -5
NAJ_EBUSY = -6
NAJ_FP64 = 0
NAJ_MIXED = 1
NAJ_STOP_RELRES = 0
NAJ_STOP_OBJECTIVE = 1


class NajError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"naj status {status}: {msg}")
        self.status = status


class NajOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("k0", ctypes.c_int32), ("confirm_gap", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32), ("inner_stall", ctypes.c_int32),
                ("stop", ctypes.c_int32), ("pad_", ctypes.c_int32), ("fstar", ctypes.c_double)]


class NajResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("confirmations", ctypes.c_int32), ("relres", ctypes.c_double), ("hist_len", ctypes.c_int32),
                ("nrestart_log", ctypes.c_int32), ("kernel_ms", ctypes.c_double), ("passes", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("objgap", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

_SIGS = {
    "naj_opts_default": (None, [ctypes.POINTER(NajOpts)]),
    "naj_last_error": (ctypes.c_char_p, []),
    "naj_version": (ctypes.c_char_p, []),
    "naj_create_system": (ctypes.c_int, [_I64, _I64, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "naj_create_system_blockj": (ctypes.c_int, [_I64, _I64, _P, _P, _P, _I32, _P, ctypes.POINTER(_P)]),
    "naj_block_inverse": (ctypes.c_int, [_P, _P, _P]),
    "naj_destroy_system": (None, [_P]),
    "naj_system_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                       ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "naj_system_value_bytes": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "naj_system_offset_slices": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                                ctypes.POINTER(_I64)]),
    "naj_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(NajOpts), _P, ctypes.POINTER(NajResult), _P, _I32,
                                 _P, _I32, _P, _I32, _P]),
    "naj_solve_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(NajOpts), _P, ctypes.POINTER(NajResult), _P,
                                         _I32, _P]),
    "naj_cancel": (ctypes.c_int, [_P]),
    "naj_bandwidth_probe": (ctypes.c_int, [_I32, _P, _P, _I64, _I32, ctypes.POINTER(_D), _P]),
    "naj_step": (ctypes.c_int, [_P, _P, _P, _D, _P, _P, _P, _P]),
    "naj_residual": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "naj_diagonal": (ctypes.c_int, [_P, _P, _P]),
    "naj_batch_create": (ctypes.c_int, [_I32, _P, _P, ctypes.POINTER(NajOpts), _P, ctypes.POINTER(_P)]),
    "naj_batch_solve": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "naj_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "naj_batch_destroy": (None, [_P]),
    "naj_autotune_tiles": (ctypes.c_int, [_P, _I32, ctypes.POINTER(NajOpts), _I32, _P, ctypes.POINTER(_I32)]),
    "naj_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "naj_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "naj_server_create": (ctypes.c_int, [_I64, _I32, _I32, ctypes.POINTER(NajOpts), _P, ctypes.POINTER(_P)]),
    "naj_server_admit": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _P, _I32, _P, _P, _D, _P, ctypes.POINTER(_I64)]),
    "naj_server_step": (ctypes.c_int, [_P, _I32, _P, _I32, ctypes.POINTER(_I32)]),
    "naj_server_result": (ctypes.c_int, [_P, _I64, ctypes.POINTER(NajResult)]),
    "naj_server_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                       ctypes.POINTER(_I32)]),
    "naj_server_destroy": (None, [_P]),
}
NAJ_MAX_RHS = 8


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions declared in include/naj.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(naj_[a-z0-9_]+)\s*\(", text)))


# Live handles, closed by an exit hook before the interpreter and the HIP runtime shut down.  Freeing
# device memory from __del__ during interpreter finalization would run after the runtime (and a
# profiler attached to it) has already been torn down, which can crash the process in exit().
_live = {"server": weakref.WeakSet(), "batch": weakref.WeakSet(), "system": weakref.WeakSet()}


def _close_all():
    """Release every live server, batch and system (in that order: a batch or server refers to systems)."""
    for kind in ("server", "batch", "system"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _finalizing() -> bool:
    return sys.is_finalizing()


def load(path: str = LIB_PATH):
    """Load libnaj.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (python -m paper_2407_03272_amd.build "
                           "or __graft_entry__.build())")
    _torch()   # torch's HIP runtime is set up first: the library shares it (device memory, streams)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    atexit.register(_close_all)
    return lib


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(st: int):
    if st < 0:
        raise NajError(st, load().naj_last_error().decode())
    return st


def default_opts(**kw) -> NajOpts:
    o = NajOpts()
    load().naj_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    confirmations: int
    relres: float
    hist: np.ndarray = field(default_factory=lambda: np.zeros(0))
    restart_log: list = field(default_factory=list)
    trace: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    kernel_ms: float = 0.0
    passes: int = 0
    grid: int = 0
    objgap: float = float("nan")


class System:
    """A system Q x = b resident on the GPU (naj_create_system).

    rowptr, colidx: int32 CSR arrays; vals: float64; D: optional float64
    diagonal replacing J; jblock: block size of the block-diagonal J of
    eq. (J-blkdiag) (naj_create_system_blockj) instead of the diagonal J.
    Accepts numpy arrays or torch tensors; host arrays are copied to ``device``.
    """

    def __init__(self, rowptr, colidx, vals, D=None, device="cuda:0", stream=None, jblock=None):
        torch = _torch()
        lib = load()
        self.device = torch.device(device)
        self._rowptr = self._dev(rowptr, torch.int32)
        self._colidx = self._dev(colidx, torch.int32)
        self._vals = self._dev(vals, torch.float64)
        self._D = None if D is None else self._dev(D, torch.float64)
        self.n = int(self._rowptr.numel() - 1)
        self.nnz = int(self._colidx.numel())
        h = ctypes.c_void_p()
        self.jblock = jblock
        with torch.cuda.device(self.device):
            if jblock is not None:
                if D is not None:
                    raise ValueError("a block J and a caller diagonal D exclude each other")
                st = lib.naj_create_system_blockj(self.n, self.nnz, _ptr(self._rowptr), _ptr(self._colidx),
                                                  _ptr(self._vals), int(jblock), _stream_ptr(stream), ctypes.byref(h))
            else:
                st = lib.naj_create_system(self.n, self.nnz, _ptr(self._rowptr), _ptr(self._colidx), _ptr(self._vals),
                                           _ptr(self._D), _stream_ptr(stream), ctypes.byref(h))
        _check(st)
        self._h = h
        _live["system"].add(self)
        # inputs are copied by the library; drop our references
        self._rowptr = self._colidx = self._vals = self._D = None

    def _dev(self, a, dtype):
        torch = _torch()
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=self.device, dtype=dtype).contiguous()

    def vec(self, a):
        return self._dev(a, _torch().float64)

    def close(self):
        if getattr(self, "_h", None):
            load().naj_destroy_system(self._h)
            self._h = None

    def __del__(self):
        try:
            if _finalizing():   # the exit hook has released every handle; the runtime may be gone now
                return
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        n, nnz, by, st = _I64(), _I64(), _I64(), _I64()
        lay = _I32()
        _check(load().naj_system_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(by),
                                      ctypes.byref(lay), ctypes.byref(st)))
        of, ns, onz = _I64(), _I64(), _I64()
        _check(load().naj_system_offset_slices(self._h, ctypes.byref(of), ctypes.byref(ns), ctypes.byref(onz)))
        vb = _I32()
        _check(load().naj_system_value_bytes(self._h, ctypes.byref(vb)))
        return dict(n=n.value, nnz=nnz.value, device_bytes=by.value, layout=lay.value, stored_entries=st.value,
                    offset_slices=of.value, nslices=ns.value, offset_nnz=onz.value, value_bytes=vb.value)

    def solve(self, b, x0=None, *, out=None, hist_cap: int | None = None, trace: bool = False, stream=None,
              **opts) -> tuple:
        """naj_solve: returns (x, SolveInfo).  Options as in naj_opts (tol, max_iter, restart, k0, ...)."""
        torch = _torch()
        lib = load()
        o = default_opts(**opts)
        b = self.vec(b)
        x0 = None if x0 is None else self.vec(x0)
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        cap = o.max_iter if hist_cap is None else hist_cap
        hist = np.zeros(max(cap, 1), dtype=np.float64)
        rlog = np.zeros(64, dtype=np.int32)
        tr = np.zeros((max(cap, 1), 2), dtype=np.float64) if trace else None
        res = NajResult()
        with torch.cuda.device(self.device):
            st = lib.naj_solve(self._h, _ptr(b), _ptr(x0), ctypes.byref(o), _ptr(x), ctypes.byref(res),
                               hist.ctypes.data_as(_P) if cap > 0 else None, cap,
                               rlog.ctypes.data_as(_P), 64,
                               tr.ctypes.data_as(_P) if trace else None, cap if trace else 0,
                               _stream_ptr(stream))
        if st < 0 and st not in (NAJ_EBREAKDOWN, NAJ_ECANCELLED):
            _check(st)
        info = SolveInfo(res.status, res.iterations, res.restarts, res.confirmations, res.relres,
                         hist[:res.hist_len].copy(), rlog[:res.nrestart_log].tolist(),
                         tr[:res.hist_len].copy() if trace else np.zeros((0, 2)),
                         res.kernel_ms, res.passes, res.grid, res.objgap)
        return x, info

    def cancel(self):
        """naj_cancel: ask the solve running on this system (in another thread) to stop."""
        _check(load().naj_cancel(self._h))

    def solve_noalloc(self, b, x0=None, *, out=None, stream=None, **opts) -> tuple:
        """naj_solve_noalloc: the same solve with its scratch in the library's static device array
        (allocates no device memory; ``out`` should be given so this call allocates nothing either)."""
        torch = _torch()
        lib = load()
        o = default_opts(**opts)
        b = self.vec(b)
        x0 = None if x0 is None else self.vec(x0)
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        rlog = np.zeros(64, dtype=np.int32)
        res = NajResult()
        with torch.cuda.device(self.device):
            st = lib.naj_solve_noalloc(self._h, _ptr(b), _ptr(x0), ctypes.byref(o), _ptr(x), ctypes.byref(res),
                                       rlog.ctypes.data_as(_P), 64, _stream_ptr(stream))
        if st < 0 and st not in (NAJ_EBREAKDOWN, NAJ_ECANCELLED):
            _check(st)
        info = SolveInfo(res.status, res.iterations, res.restarts, res.confirmations, res.relres,
                         np.zeros(0), rlog[:res.nrestart_log].tolist(), np.zeros((0, 2)),
                         res.kernel_ms, res.passes, res.grid, res.objgap)
        return x, info

    def step(self, p, r, beta: float, b, stream=None):
        """naj_step: one fused pass; returns (x, (s, gg, sabs))."""
        torch = _torch()
        p = self.vec(p)
        r = None if r is None else self.vec(r)
        b = self.vec(b)
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        red = np.zeros(3, dtype=np.float64)
        with torch.cuda.device(self.device):
            _check(load().naj_step(self._h, _ptr(p), _ptr(r), float(beta), _ptr(b), _ptr(x),
                                   red.ctypes.data_as(_P), _stream_ptr(stream)))
        return x, tuple(red)

    def residual(self, x, b, want_vector: bool = False, stream=None):
        """naj_residual: (b - Q x or None, ||b - Q x||^2)."""
        torch = _torch()
        x = self.vec(x)
        b = self.vec(b)
        out = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_vector else None
        rr = ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(load().naj_residual(self._h, _ptr(x), _ptr(b), _ptr(out), ctypes.byref(rr), _stream_ptr(stream)))
        return out, rr.value

    def diagonal(self, stream=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(load().naj_diagonal(self._h, _ptr(out), _stream_ptr(stream)))
        return out


    def block_inverse(self, stream=None):
        """The inverse blocks of a block-J system as an (n, jblock) float64 tensor: row r holds row
        r - i*jblock of (J^{i,i})^{-1} for the block i that contains r."""
        torch = _torch()
        out = torch.empty(self.n * int(self.jblock or 1), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(load().naj_block_inverse(self._h, _ptr(out), _stream_ptr(stream)))
        return out.view(self.n, -1)


class Batch:
    """Many systems with several right-hand sides each, solved together (naj_batch_*).

    systems: list of System; nrhs: list of ints (1..NAJ_MAX_RHS); options as in naj_opts.
    solve(bs, x0s=None) takes per-system right-hand sides of shape (n_i, nrhs_i) (or (n_i,) when
    nrhs_i == 1) and returns (list of x, list of per-instance SolveInfo, kernel_ms).
    """

    def __init__(self, systems, nrhs, stream=None, **opts):
        torch = _torch()
        self.systems = list(systems)
        self.nrhs = [int(k) for k in nrhs]
        self.device = self.systems[0].device
        o = default_opts(**opts)
        self.opts = o
        arr = (_P * len(self.systems))(*[s._h for s in self.systems])
        ks = (_I32 * len(self.systems))(*self.nrhs)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(load().naj_batch_create(len(self.systems), arr, ks, ctypes.byref(o), _stream_ptr(stream),
                                           ctypes.byref(h)))
        self._h = h
        _live["batch"].add(self)

    def info(self) -> dict:
        nt, g, by = _I32(), _I32(), _I64()
        _check(load().naj_batch_info(self._h, ctypes.byref(nt), ctypes.byref(g), ctypes.byref(by)))
        return dict(ntiles=nt.value, grid=g.value, device_bytes=by.value)

    def close(self):
        if getattr(self, "_h", None):
            load().naj_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            if _finalizing():   # the exit hook has released every handle; the runtime may be gone now
                return
            self.close()
        except Exception:
            pass

    def solve(self, bs, x0s=None, outs=None, stream=None):
        torch = _torch()
        nsys = len(self.systems)
        bt = [self.systems[i]._dev(bs[i], torch.float64) for i in range(nsys)]
        x0t = None if x0s is None else [None if x0s[i] is None else self.systems[i]._dev(x0s[i], torch.float64)
                                        for i in range(nsys)]
        xs = outs if outs is not None else [torch.empty_like(bt[i]) for i in range(nsys)]
        bp = (_P * nsys)(*[t.data_ptr() for t in bt])
        xp = (_P * nsys)(*[t.data_ptr() for t in xs])
        x0p = None if x0t is None else (_P * nsys)(*[0 if t is None else t.data_ptr() for t in x0t])
        ninst = sum(self.nrhs)
        res = (NajResult * ninst)()
        with torch.cuda.device(self.device):
            st = load().naj_batch_solve(self._h, bp, x0p, xp, res, _stream_ptr(stream))
        if st < 0 and st != NAJ_EBREAKDOWN:
            _check(st)
        infos = [SolveInfo(r.status, r.iterations, r.restarts, r.confirmations, r.relres, kernel_ms=r.kernel_ms,
                           passes=r.passes, grid=r.grid) for r in res]
        return xs, infos, (res[0].kernel_ms if ninst else 0.0)


def autotune_tiles(system: System, nrhs: int, passes: int = 20, stream=None, **opts) -> int:
    """naj_autotune_tiles: time tile sizes on `system` alone and record the fastest; returns it."""
    torch = _torch()
    o = default_opts(**opts)
    best = _I32()
    with torch.cuda.device(system.device):
        _check(load().naj_autotune_tiles(system._h, int(nrhs), ctypes.byref(o), int(passes), _stream_ptr(stream),
                                         ctypes.byref(best)))
    return best.value


def bandwidth_probe(mode: int, nbytes: int = 1 << 30, reps: int = 20, device="cuda:0", stream=None) -> dict:
    """naj_bandwidth_probe on fresh buffers of `nbytes`: mode 0 read, 1 copy, 2 write.  Returns the mean
    milliseconds per launch and the rate in GB/s (bytes moved per launch / time)."""
    torch = _torch()
    dev = torch.device(device)
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev) if mode != 2 else None
    dst = torch.empty(nbytes // 8 if mode != 0 else 2, dtype=torch.float64, device=dev)
    ms = _D()
    with torch.cuda.device(dev):
        _check(load().naj_bandwidth_probe(int(mode), _ptr(src), _ptr(dst), int(nbytes), int(reps), ctypes.byref(ms),
                                          _stream_ptr(stream)))
    moved = nbytes * (2 if mode == 1 else 1)
    out = {"mode": ("read", "copy", "write")[mode], "bytes_per_launch": moved, "ms": ms.value,
           "gbps": moved / (ms.value / 1e3) / 1e9}
    if mode == 1:
        out["copy_exact"] = bool(torch.equal(src, dst))
    return out


def tune_save(path: str):
    _check(load().naj_tune_save(path.encode()))


def tune_load(path: str):
    _check(load().naj_tune_load(path.encode()))


class Server:
    """Serving loop over the naj_server_* entry points (continuous batching).

    Requests (one system, 1..NAJ_MAX_RHS right-hand sides, their own tolerance) are
    admitted while others run; ``step`` advances every admitted request and returns the
    tickets that finished; ``result`` hands back the answer and frees the request's
    slot and memory.  The passes run on ``stream`` (a torch stream of its own by default,
    so that uploads on other streams do not wait for them).
    """

    def __init__(self, mem_budget: int, max_slots: int = 64, max_rhs: int = NAJ_MAX_RHS, device="cuda:0",
                 stream=None, **opts):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.upload = torch.cuda.Stream(device=self.device)
        o = default_opts(**opts)
        h = _P()
        with torch.cuda.device(self.device):
            _check(load().naj_server_create(int(mem_budget), int(max_slots), int(max_rhs), ctypes.byref(o),
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        _live["server"].add(self)
        self._req = {}     # ticket -> (x tensor, nrhs, inputs kept alive until admitted)
        self._done = (_I64 * 4096)()

    def _dev(self, a, dtype):
        torch = _torch()
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=self.device, dtype=dtype).contiguous()

    def stage(self, rowptr, colidx, vals, b, x0=None, D=None):
        """Device copies of a request's inputs (made on the upload stream), for admit; a request
        that finds the server busy can be retried with them without uploading again."""
        torch = _torch()
        with torch.cuda.device(self.device), torch.cuda.stream(self.upload):
            out = (self._dev(rowptr, torch.int32), self._dev(colidx, torch.int32), self._dev(vals, torch.float64),
                   self._dev(b, torch.float64), None if x0 is None else self._dev(x0, torch.float64),
                   None if D is None else self._dev(D, torch.float64))
        self.upload.synchronize()
        return out

    def admit(self, rowptr, colidx, vals, b, x0=None, D=None, tol: float = 0.0):
        """Returns a ticket, or None when the server is busy (no slot or budget free now)."""
        torch = _torch()
        rp, ci, va, bb, x0t, Dt = self.stage(rowptr, colidx, vals, b, x0, D)
        with torch.cuda.device(self.device):
            x = torch.empty_like(bb)
        n = rp.numel() - 1
        nrhs = 1 if bb.dim() == 1 else int(bb.shape[1])
        t = _I64()
        with torch.cuda.device(self.device):
            st = load().naj_server_admit(self._h, n, ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr(),
                                         None if Dt is None else Dt.data_ptr(), nrhs, bb.data_ptr(),
                                         None if x0t is None else x0t.data_ptr(), float(tol), x.data_ptr(),
                                         ctypes.byref(t))
        if st == NAJ_EBUSY:
            return None
        _check(st)
        self._req[t.value] = (x, nrhs)
        return t.value

    def step(self, chunks: int = 1) -> list:
        """Run `chunks` chunks of passes (0: none); returns the tickets found finished."""
        torch = _torch()
        nd = _I32()
        with torch.cuda.device(self.device):
            _check(load().naj_server_step(self._h, int(chunks), self._done, len(self._done), ctypes.byref(nd)))
        return [self._done[i] for i in range(nd.value)]

    def result(self, ticket: int):
        """(x on the device, list of SolveInfo) of a finished request; frees its slot."""
        torch = _torch()
        x, nrhs = self._req[ticket]
        res = (NajResult * nrhs)()
        with torch.cuda.device(self.device):
            st = load().naj_server_result(self._h, int(ticket), res)
        if st < 0 and st != NAJ_EBREAKDOWN:
            _check(st)
        del self._req[ticket]
        return x, [SolveInfo(r.status, r.iterations, r.restarts, r.confirmations, r.relres, passes=r.passes,
                             grid=r.grid) for r in res]

    def info(self) -> dict:
        bu, bt, su, stt = _I64(), _I64(), _I32(), _I32()
        _check(load().naj_server_info(self._h, ctypes.byref(bu), ctypes.byref(bt), ctypes.byref(su), ctypes.byref(stt)))
        return dict(bytes_used=bu.value, bytes_total=bt.value, slots_used=su.value, slots_total=stt.value)

    def close(self):
        if getattr(self, "_h", None):
            load().naj_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            if _finalizing():   # the exit hook has released every handle; the runtime may be gone now
                return
            self.close()
        except Exception:
            pass

