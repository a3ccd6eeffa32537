"""Thin Python binding of the C ABI in ``include/caqr.h`` (``libcaqr.so``).

Argument marshalling only: every step of the factorization runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current
stream.  Matrices are column-major: an m-by-n matrix is a CUDA float64 tensor
of shape (m, n) with strides (1, ldx), ldx >= m (see :func:`fortran`).

There is no CPU fallback: if the library is not built this module raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcaqr.so")

OP_N, OP_T = 0, 1
F64, F32 = 0, 1

_STATUS = {
    0: "CAQR_SUCCESS",
    1: "CAQR_ERR_INVALID_VALUE",
    2: "CAQR_ERR_ALLOC",
    3: "CAQR_ERR_DEVICE",
    4: "CAQR_ERR_NOT_SUPPORTED",
    5: "CAQR_ERR_SINGULAR",
    6: "CAQR_ERR_NONFINITE",
    7: "CAQR_ERR_NOT_CONVERGED",
}


class CaqrError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {_STATUS.get(code, code)} ({_lib().caqr_status_string(code).decode()})")


class TreeOpts(ctypes.Structure):
    _fields_ = [("leaf_rows", ctypes.c_int32), ("leaves_per_wg", ctypes.c_int32),
                ("inner_block", ctypes.c_int32), ("arity", ctypes.c_int32)]


class FactorsInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nb", ctypes.c_int64), ("panels", ctypes.c_int64),
                ("leaf_rows", ctypes.c_int32), ("leaves_per_wg", ctypes.c_int32),
                ("leaves_panel0", ctypes.c_int64), ("depth_panel0", ctypes.c_int32), ("t_formed", ctypes.c_int32),
                ("inner_block", ctypes.c_int32), ("arity", ctypes.c_int32)]


class TraceEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("panel", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("width", ctypes.c_int32), ("leaves", ctypes.c_int32),
                ("ms", ctypes.c_double)]


TRACE_KINDS = {0: "panel", 1: "update_t", 2: "update_n", 3: "form_t", 4: "other", 5: "update_t_levels"}


LS_F64, LS_MIXED_F32 = 0, 1


class LsOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("no_fallback", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("index", ctypes.c_int64), ("iters", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("eta", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("workers", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64),
                ("reserved", ctypes.c_int64)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64), ("end_ns", ctypes.c_int64)]


_lib_obj = None
_lib_lock = threading.Lock()

EXPORTS = [
    "caqr_create", "caqr_destroy", "caqr_set_stream", "caqr_get_stream", "caqr_set_workspace_limit", "caqr_sync",
    "caqr_status_string", "caqr_device_count", "tsqr_factor", "caqr_factor", "apply_q", "caqr_factors_destroy",
    "caqr_factors_get_info", "caqr_factors_get_signs", "ls_solve", "caqr_set_trace", "caqr_set_trace_kinds", "caqr_trace_read",
    "tsqr_factor_batched", "caqr_batch_destroy", "caqr_batch_get_plan", "caqr_batch_get_signs", "caqr_tune_batched",
    "caqr_batch_plan_for", "ls_solve_batched", "caqr_server_create", "caqr_server_submit", "caqr_server_wait", "caqr_server_destroy",
    "caqr_debug_fail_at", "ls_solve_noalloc",
]


def _lib():
    global _lib_obj
    with _lib_lock:
        if _lib_obj is not None:
            return _lib_obj
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.caqr_create.argtypes = [ctypes.POINTER(vp), i32]
        L.caqr_destroy.argtypes = [vp]
        L.caqr_set_stream.argtypes = [vp, vp]
        L.caqr_get_stream.argtypes = [vp, ctypes.POINTER(vp)]
        L.caqr_set_workspace_limit.argtypes = [vp, ctypes.c_size_t]
        L.caqr_debug_fail_at.argtypes = [vp, i64]
        L.caqr_sync.argtypes = [vp]
        L.caqr_status_string.argtypes = [i32]
        L.caqr_status_string.restype = ctypes.c_char_p
        L.caqr_device_count.argtypes = []
        L.tsqr_factor.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(TreeOpts), ctypes.POINTER(vp)]
        L.caqr_factor.argtypes = [vp, i64, i64, i64, vp, i64, ctypes.POINTER(TreeOpts), ctypes.POINTER(vp)]
        L.apply_q.argtypes = [vp, vp, i32, i64, vp, i64]
        L.caqr_factors_destroy.argtypes = [vp]
        L.caqr_factors_get_info.argtypes = [vp, ctypes.POINTER(FactorsInfo)]
        L.caqr_factors_get_signs.argtypes = [vp, vp, dp]
        L.ls_solve.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, ctypes.POINTER(LsOpts), ctypes.POINTER(LsInfo)]
        L.ls_solve_noalloc.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, ctypes.POINTER(LsInfo)]
        L.caqr_set_trace.argtypes = [vp, i32]
        L.caqr_set_trace_kinds.argtypes = [vp, ctypes.c_uint32]
        L.caqr_trace_read.argtypes = [vp, ctypes.POINTER(TraceEntry), i64, ctypes.POINTER(i64)]
        pi64 = ctypes.POINTER(i64)
        L.tsqr_factor_batched.argtypes = [vp, i64, pi64, pi64, ctypes.POINTER(vp), pi64, i32,
                                          ctypes.POINTER(TreeOpts), ctypes.POINTER(vp)]
        L.caqr_batch_destroy.argtypes = [vp]
        L.caqr_batch_get_plan.argtypes = [vp, i64, ctypes.POINTER(TreeOpts)]
        L.caqr_batch_get_signs.argtypes = [vp, i64, dp]
        L.caqr_tune_batched.argtypes = [vp, i32]
        L.caqr_batch_plan_for.argtypes = [vp, i64, i64, i32, ctypes.POINTER(TreeOpts)]
        L.ls_solve_batched.argtypes = [vp, i64, pi64, pi64, pi64, ctypes.POINTER(vp), pi64, ctypes.POINTER(vp), pi64,
                                       ctypes.POINTER(TreeOpts), ctypes.POINTER(LsInfo)]
        L.caqr_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.caqr_server_submit.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, ctypes.POINTER(i64)]
        L.caqr_server_wait.argtypes = [vp, i64, ctypes.POINTER(LsInfo), ctypes.POINTER(RequestTimes)]
        L.caqr_server_destroy.argtypes = [vp]
        for name in EXPORTS:
            if name not in ("caqr_status_string",):
                getattr(L, name).restype = ctypes.c_int
        _lib_obj = L
        return L


def library() -> ctypes.CDLL:
    """The loaded ``libcaqr.so`` (raises if it is not built)."""
    return _lib()


def _check(code: int, where: str):
    if code != 0:
        raise CaqrError(code, where)


def device_count() -> int:
    return int(_lib().caqr_device_count())


class Handle:
    """A library handle on one GPU; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        self.device = device
        _check(_lib().caqr_create(ctypes.byref(self._h), device), "caqr_create")

    @property
    def ptr(self):
        return self._h

    def use_current_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(_lib().caqr_set_stream(self._h, ctypes.c_void_p(s)), "caqr_set_stream")

    def set_workspace_limit(self, nbytes: int):
        _check(_lib().caqr_set_workspace_limit(self._h, nbytes), "caqr_set_workspace_limit")

    def fail_at(self, k: int):
        """Test hook: the k-th library launch site from now on reports a device
        error instead of enqueuing (0 switches it off)."""
        _check(_lib().caqr_debug_fail_at(self._h, k), "caqr_debug_fail_at")

    def sync(self):
        _check(_lib().caqr_sync(self._h), "caqr_sync")

    def set_trace(self, enable: bool):
        _check(_lib().caqr_set_trace(self._h, 1 if enable else 0), "caqr_set_trace")

    def set_trace_kinds(self, kinds):
        """Trace only the named kinds ("panel", "update_t", "update_n", "form_t", "other")."""
        mask = 0
        codes = {v: k for k, v in TRACE_KINDS.items()}
        for k in kinds:
            mask |= 1 << codes[k]
        _check(_lib().caqr_set_trace_kinds(self._h, mask), "caqr_set_trace_kinds")

    def take_trace(self, max_entries: int = 1 << 16):
        """Recorded launches (launch order) with their device time in ms; clears the record."""
        buf = (TraceEntry * max_entries)()
        count = ctypes.c_int64()
        _check(_lib().caqr_trace_read(self._h, buf, max_entries, ctypes.byref(count)), "caqr_trace_read")
        out = []
        for e in buf[: min(count.value, max_entries)]:
            out.append({"kind": TRACE_KINDS.get(e.kind, e.kind), "panel": e.panel, "rows": e.rows, "cols": e.cols,
                        "width": e.width, "leaves": e.leaves, "ms": e.ms})
        return out

    def close(self):
        if self._h:
            _lib().caqr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict = {}


def handle(device: int = 0) -> Handle:
    """A cached handle per (thread, device)."""
    key = (threading.get_ident(), device)
    h = _handles.get(key)
    if h is None:
        h = _handles[key] = Handle(device)
    h.use_current_stream()
    return h


def fortran(x, device="cuda", dtype=torch.float64) -> torch.Tensor:
    """Copy a 2-D array into a column-major CUDA tensor (float64 by default)."""
    t = torch.as_tensor(x, dtype=dtype)
    if t.ndim == 1:
        t = t[:, None]
    out = torch.empty((t.shape[1], t.shape[0]), dtype=dtype, device=device).t()
    out.copy_(t)
    return out


def _ld(t: torch.Tensor, dtypes=(torch.float64,)) -> int:
    if t.dtype not in dtypes or not t.is_cuda or t.ndim != 2:
        raise ValueError("expected a 2-D " + "/".join(str(d).split(".")[-1] for d in dtypes) + " CUDA tensor")
    m, n = t.shape
    if t.stride(0) != 1 and not (n <= 1 and t.is_contiguous()):
        raise ValueError("matrix must be column-major (stride (1, ld))")
    return max(1, t.stride(1) if n > 1 else m)


def _opts(leaf_rows=0, leaves_per_wg=0, inner_block=0, arity=0):
    if not leaf_rows and not leaves_per_wg and not inner_block and not arity:
        return None
    return ctypes.byref(TreeOpts(leaf_rows, leaves_per_wg, inner_block, arity))


class Factors:
    """Owner of a ``caqr_factors_t``; keeps the factored tensor alive."""

    def __init__(self, h: Handle, ptr: ctypes.c_void_p, A: torch.Tensor):
        self.h, self._f, self.A = h, ptr, A

    def info(self) -> FactorsInfo:
        inf = FactorsInfo()
        _check(_lib().caqr_factors_get_info(self._f, ctypes.byref(inf)), "caqr_factors_get_info")
        return inf

    def signs(self):
        import numpy as np

        d = np.zeros(self.A.shape[1])
        _check(_lib().caqr_factors_get_signs(self.h.ptr, self._f, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "caqr_factors_get_signs")
        return d

    @property
    def R(self) -> torch.Tensor:
        n = self.A.shape[1]
        return torch.triu(self.A[:n, :n])

    def apply_q(self, C: torch.Tensor, op: int = OP_T) -> torch.Tensor:
        """In place: C <- Q^T C (op=OP_T) or Q C (op=OP_N)."""
        self.h.use_current_stream()
        if C.shape[0] != self.A.shape[0]:
            raise ValueError("C must have m rows")
        _check(_lib().apply_q(self.h.ptr, self._f, op, C.shape[1], ctypes.c_void_p(C.data_ptr()), _ld(C)), "apply_q")
        return C

    def q_thin(self) -> torch.Tensor:
        m, n = self.A.shape
        Q = torch.zeros((n, m), dtype=torch.float64, device=self.A.device).t()
        Q[:n, :n] = torch.eye(n, dtype=torch.float64, device=self.A.device)
        return self.apply_q(Q, OP_N)

    def close(self):
        if self._f:
            _lib().caqr_factors_destroy(self._f)
            self._f = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tsqr(A: torch.Tensor, leaf_rows: int = 0, leaves_per_wg: int = 0, device: int = 0,
         inner_block: int = 0, arity: int = 0) -> Factors:
    """In place TSQR of a column-major CUDA tensor; returns the factors (R = F.R)."""
    h = handle(device)
    m, n = A.shape
    f = ctypes.c_void_p()
    _check(_lib().tsqr_factor(h.ptr, m, n, ctypes.c_void_p(A.data_ptr()), _ld(A),
                              _opts(leaf_rows, leaves_per_wg, inner_block, arity), ctypes.byref(f)), "tsqr_factor")
    return Factors(h, f, A)


def caqr(A: torch.Tensor, nb: int = 64, leaf_rows: int = 0, leaves_per_wg: int = 0, device: int = 0,
         inner_block: int = 0, arity: int = 0) -> Factors:
    """In place CAQR (panel width nb) of a column-major CUDA tensor."""
    h = handle(device)
    m, n = A.shape
    f = ctypes.c_void_p()
    _check(_lib().caqr_factor(h.ptr, m, n, nb, ctypes.c_void_p(A.data_ptr()), _ld(A),
                              _opts(leaf_rows, leaves_per_wg, inner_block, arity), ctypes.byref(f)), "caqr_factor")
    return Factors(h, f, A)


def ls_solve(A: torch.Tensor, B: torch.Tensor, device: int = 0, precision: int = LS_F64, tol: float = 0.0,
             max_iter: int = 0, fallback: bool = True):
    """Least squares: returns (X = B[:n], info).  FP64 (default): A and B in
    place (A factored, B <- Q^T B).  precision=LS_MIXED_F32: A only read,
    trailing updates on FP32 MFMA and FP64 refinement to the backward-error
    bound tol (0: 1e-12), falling back to the FP64 solve when it stalls
    (fallback=False: CAQR_ERR_NOT_CONVERGED instead, status 7).  Raises
    CaqrError on argument or device errors only."""
    h = handle(device)
    m, n = A.shape
    info = LsInfo()
    opts = None
    if precision != LS_F64 or tol or max_iter or not fallback:
        opts = ctypes.byref(LsOpts(precision, max_iter, tol, 0 if fallback else 1, 0))
    code = _lib().ls_solve(h.ptr, m, n, B.shape[1], ctypes.c_void_p(A.data_ptr()), _ld(A),
                           ctypes.c_void_p(B.data_ptr()), _ld(B), opts, ctypes.byref(info))
    if code not in (0, 5, 6, 7):
        _check(code, "ls_solve")
    return B[:n], info


def ls_solve_noalloc(A: torch.Tensor, B: torch.Tensor, device: int = 0):
    """ls_solve through the entry point that allocates no device memory (its
    workspace is the library's static per-GPU scratch array): returns
    (X = B[:n], info); raises CaqrError(CAQR_ERR_NOT_SUPPORTED) when the
    problem's workspace does not fit that array."""
    h = handle(device)
    m, n = A.shape
    info = LsInfo()
    code = _lib().ls_solve_noalloc(h.ptr, m, n, B.shape[1], ctypes.c_void_p(A.data_ptr()), _ld(A),
                                   ctypes.c_void_p(B.data_ptr()), _ld(B), ctypes.byref(info))
    if code not in (0, 5, 6):
        _check(code, "ls_solve_noalloc")
    return B[:n], info


class Batch:
    """Owner of a ``caqr_batch_t``; keeps the factored tensors alive."""

    def __init__(self, h: Handle, ptr: ctypes.c_void_p, As):
        self.h, self._b, self.As = h, ptr, list(As)

    def plan(self, i: int):
        """(leaf_rows, leaves_per_wg, arity) of problem i."""
        o = TreeOpts()
        _check(_lib().caqr_batch_get_plan(self._b, i, ctypes.byref(o)), "caqr_batch_get_plan")
        return int(o.leaf_rows), int(o.leaves_per_wg), int(o.arity)

    def signs(self, i: int):
        import numpy as np

        d = np.zeros(self.As[i].shape[1])
        _check(_lib().caqr_batch_get_signs(self._b, i, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "caqr_batch_get_signs")
        return d

    def R(self, i: int) -> torch.Tensor:
        n = self.As[i].shape[1]
        return torch.triu(self.As[i][:n, :n])

    def close(self):
        if self._b:
            _lib().caqr_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_DT = {torch.float64: F64, torch.float32: F32}


def _dtype_code(dtype) -> int:
    if dtype not in _DT:
        raise ValueError("dtype must be torch.float64 or torch.float32")
    return _DT[dtype]


def tsqr_batched(As, leaf_rows: int = 0, leaves_per_wg: int = 0, device: int = 0, arity: int = 0) -> Batch:
    """In place TSQR of every column-major CUDA tensor in ``As`` (all float64 or
    all float32; one plan for all when leaf_rows/leaves_per_wg are given, else
    the tuned or default plans of that type)."""
    h = handle(device)
    k = len(As)
    dtype = As[0].dtype if k else torch.float64
    dt = _dtype_code(dtype)
    m = (ctypes.c_int64 * max(1, k))(*[int(a.shape[0]) for a in As])
    n = (ctypes.c_int64 * max(1, k))(*[int(a.shape[1]) for a in As])
    ld = (ctypes.c_int64 * max(1, k))(*[_ld(a, (dtype,)) for a in As])
    ptrs = (ctypes.c_void_p * max(1, k))(*[a.data_ptr() for a in As])
    b = ctypes.c_void_p()
    _check(_lib().tsqr_factor_batched(h.ptr, k, m, n, ptrs, ld, dt, _opts(leaf_rows, leaves_per_wg, 0, arity),
                                      ctypes.byref(b)), "tsqr_factor_batched")
    return Batch(h, b, As)


def ls_solve_batched(As, Bs, leaf_rows: int = 0, leaves_per_wg: int = 0, device: int = 0, arity: int = 0):
    """Batched least squares in place (n_i <= 64, float64, column-major CUDA
    tensors): returns ([X_i = B_i[:n_i]], [(status, index)]); raises only on
    argument or device errors."""
    h = handle(device)
    k = len(As)
    arr = lambda vals: (ctypes.c_int64 * max(1, k))(*vals)
    m = arr([int(a.shape[0]) for a in As])
    n = arr([int(a.shape[1]) for a in As])
    r = arr([int(b.shape[1]) for b in Bs])
    la = arr([_ld(a) for a in As])
    lb = arr([_ld(b) for b in Bs])
    pa = (ctypes.c_void_p * max(1, k))(*[a.data_ptr() for a in As])
    pb = (ctypes.c_void_p * max(1, k))(*[b.data_ptr() for b in Bs])
    info = (LsInfo * max(1, k))()
    code = _lib().ls_solve_batched(h.ptr, k, m, n, r, pa, la, pb, lb, _opts(leaf_rows, leaves_per_wg, 0, arity), info)
    if code not in (0, 5, 6):
        _check(code, "ls_solve_batched")
    return [b[: a.shape[1]] for a, b in zip(As, Bs)], [(int(info[i].status), int(info[i].index)) for i in range(k)]


def tune_batched(device: int = 0, dtype=torch.float64):
    """Measure the batched plans of one element type per size bucket (stored in the handle)."""
    h = handle(device)
    _check(_lib().caqr_tune_batched(h.ptr, _dtype_code(dtype)), "caqr_tune_batched")


def batch_plan_for(m: int, n: int, device: int = 0, dtype=torch.float64):
    """(leaf_rows, leaves_per_wg, arity) a batched call without a plan uses for an m-by-n problem."""
    h = handle(device)
    o = TreeOpts()
    _check(_lib().caqr_batch_plan_for(h.ptr, m, n, _dtype_code(dtype), ctypes.byref(o)), "caqr_batch_plan_for")
    return int(o.leaf_rows), int(o.leaves_per_wg), int(o.arity)


class Server:
    """Served least-squares stream (``caqr_server_*``): requests solved
    concurrently by ``workers`` streams within a device memory budget."""

    def __init__(self, workers: int = 8, budget_bytes: int = 8 << 30, device: int = 0):
        self._s = ctypes.c_void_p()
        o = ServerOpts(device, workers, budget_bytes, 0)
        _check(_lib().caqr_server_create(ctypes.byref(o), ctypes.byref(self._s)), "caqr_server_create")
        self._keep = {}

    def submit(self, A: torch.Tensor, B: torch.Tensor, X: torch.Tensor) -> int:
        """Queue min ||A X - B|| (A, B read only; X receives the n-by-nrhs
        solution).  The request's device work is ordered after what torch's
        current stream has enqueued so far (A, B and X as that stream sees
        them).  The tensors are kept alive until ``wait``."""
        m, n = A.shape
        t = ctypes.c_int64()
        stream = torch.cuda.current_stream(A.device).cuda_stream
        _check(_lib().caqr_server_submit(self._s, m, n, B.shape[1], ctypes.c_void_p(A.data_ptr()), _ld(A),
                                         ctypes.c_void_p(B.data_ptr()), _ld(B), ctypes.c_void_p(X.data_ptr()),
                                         _ld(X), ctypes.c_void_p(stream), ctypes.byref(t)), "caqr_server_submit")
        self._keep[t.value] = (A, B, X)
        return t.value

    def wait(self, ticket: int):
        """(status, index, submit_ns, start_ns, end_ns) of a finished request."""
        info, tm = LsInfo(), RequestTimes()
        code = _lib().caqr_server_wait(self._s, ticket, ctypes.byref(info), ctypes.byref(tm))
        self._keep.pop(ticket, None)
        if code not in (0, 5, 6):
            _check(code, "caqr_server_wait")
        return int(info.status), int(info.index), int(tm.submit_ns), int(tm.start_ns), int(tm.end_ns)

    def close(self):
        if self._s:
            _lib().caqr_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
