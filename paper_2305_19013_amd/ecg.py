"""Python binding of the C ABI in ``include/ecg.h`` (argument marshalling only).

Every numerical step runs in the HIP library ``libecg.so``; this module converts
arguments and owns nothing but handles.  PyTorch is used only for device memory
(tensors on ``cuda``) and the current HIP stream.  If the library is missing the
import fails: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecg.so")

ECG_OK = 0
ECG_ENOTCONV = 1
ECG_EINVAL = -1
ECG_ENOMEM = -2
ECG_EHIP = -3
ECG_EBREAKDOWN = -4
STATUS_NAMES = {0: "ok", 1: "not_converged", -1: "einval", -2: "enomem", -3: "ehip", -4: "breakdown"}

REDUCE_NONE, REDUCE_ONCE, REDUCE_REPEAT, REDUCE_SCHEDULE = 0, 1, 2, 3
FP64, FP32_REFINED = 0, 1
PRECOND_NONE, PRECOND_SPLIT = 0, 1
SRE_CG2, MSDO_CG, MODIFIED_MSDO = 0, 1, 2
RESTART_NONE, RESTART_EVERY, RESTART_TOL = 0, 1, 2
BJ_IC0, BJ_CHOL = 0, 1

EXPORTED = (
    "ecg_options_default", "ecg_operator_create_csr", "ecg_operator_destroy", "ecg_operator_info",
    "ecg_partition_create", "ecg_partition_destroy", "ecg_precond_create_bj_ic0", "ecg_precond_create_bj",
    "ecg_precond_create_factor", "ecg_precond_destroy", "ecg_workspace_size", "ecg_solve", "ecg_spmv",
    "ecg_last_error", "ecg_debug_spmm", "ecg_debug_spmm_kernel", "ecg_debug_split", "ecg_debug_gram", "ecg_debug_update", "ecg_debug_gram_f32", "ecg_debug_update_f32",
    "ecg_debug_precond_apply", "ecg_stats_enable", "ecg_stats_read", "ecg_progress",
)
STAT_NAMES = ("spmm", "cgs2_gram", "cgs2_gram_reduce", "cgs2_update", "small_gram", "factor",
              "times_small", "final_update", "split_precond", "vector")


class Options(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("kmax", C.c_int32),
        ("reduce", C.c_int32),
        ("switch_tol", C.c_double),
        ("t_min", C.c_int32),
        ("min_gap", C.c_int32),
        ("schedule", C.POINTER(C.c_int32)),
        ("n_schedule", C.c_int32),
        ("precision", C.c_int32),
        ("inner_tol", C.c_double),
        ("max_outer", C.c_int32),
        ("replace_every", C.c_int32),
        ("trunc", C.c_int32),
        ("q_budget_bytes", C.c_int64),
        ("deflate_tol", C.c_double),
        ("precond", C.c_int32),
        ("M", C.c_void_p),
        ("variant", C.c_int32),
        ("restart", C.c_int32),
        ("restart_every", C.c_int32),
        ("restart_tol", C.c_double),
        ("max_restarts", C.c_int32),
        ("restart_at_switch", C.c_int32),
        ("refine_keep_q", C.c_int32),
    ]


class Report(C.Structure):
    _fields_ = [
        ("iters", C.c_int32),
        ("n_switch", C.c_int32),
        ("switch_iters", C.c_int32 * 8),
        ("t_final", C.c_int32),
        ("outer_iters", C.c_int32),
        ("deflated_cols", C.c_int32),
        ("trunc_used", C.c_int32),
        ("blocks_dropped", C.c_int32),
        ("vectors_stored", C.c_int64),
        ("relres_recursive", C.c_double),
        ("relres_true", C.c_double),
        ("seconds", C.c_double),
        ("status", C.c_int32),
        ("n_restart", C.c_int32),
        ("restart_iters", C.c_int32 * 8),
        ("vectors_peak", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "iters": self.iters,
            "switch_iters": list(self.switch_iters[: self.n_switch]),
            "t_final": self.t_final,
            "outer_iters": self.outer_iters,
            "deflated_cols": self.deflated_cols,
            "trunc_used": self.trunc_used,
            "blocks_dropped": self.blocks_dropped,
            "vectors_stored": int(self.vectors_stored),
            "vectors_peak": int(self.vectors_peak),
            "n_restart": self.n_restart,
            "restart_iters": list(self.restart_iters[: min(self.n_restart, 8)]),
            "relres_recursive": self.relres_recursive,
            "relres_true": self.relres_true,
            "seconds": self.seconds,
            "status": STATUS_NAMES.get(self.status, str(self.status)),
        }


class KernelStats(C.Structure):
    _fields_ = [
        ("count", C.c_int64 * 10),
        ("ms", C.c_double * 10),
        ("bytes", C.c_double * 10),
        ("flops", C.c_double * 10),
    ]


_lib = None


def lib():
    """Load libecg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
        sig = {
            "ecg_options_default": (i32, [C.POINTER(Options)]),
            "ecg_operator_create_csr": (i32, [i64, i64, vp, vp, vp, C.c_int, vp, C.POINTER(vp)]),
            "ecg_operator_destroy": (None, [vp]),
            "ecg_operator_info": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
            "ecg_partition_create": (i32, [i64, i32, vp, C.c_int, vp, C.POINTER(vp)]),
            "ecg_partition_destroy": (None, [vp]),
            "ecg_precond_create_bj_ic0": (i32, [vp, vp, vp, C.POINTER(vp)]),
            "ecg_precond_create_bj": (i32, [vp, i32, vp, C.c_int, i32, vp, C.POINTER(vp)]),
            "ecg_precond_create_factor": (i32, [i64, i64, vp, vp, vp, C.c_int, vp, C.POINTER(vp)]),
            "ecg_precond_destroy": (None, [vp]),
            "ecg_workspace_size": (i32, [vp, vp, C.POINTER(Options), C.POINTER(C.c_size_t)]),
            "ecg_solve": (i32, [vp, vp, dp, dp, C.POINTER(Options), vp, C.c_size_t, vp, C.POINTER(Report), vp]),
            "ecg_solve_noalloc": (i32, [vp, vp, dp, dp, C.POINTER(Options), vp, C.POINTER(Report), vp]),
            "ecg_spmv": (i32, [vp, dp, dp, vp]),
            "ecg_last_error": (C.c_char_p, []),
            "ecg_debug_spmm": (i32, [vp, i32, dp, dp, vp]),
            "ecg_debug_spmm_kernel": (i32, [vp, i32, i32, i32, vp, vp, vp]),
            "ecg_debug_split": (i32, [vp, i32, dp, dp, vp]),
            "ecg_debug_gram": (i32, [i64, i32, i32, dp, i32, dp, dp, vp]),
            "ecg_debug_update": (i32, [i64, i32, i32, dp, i32, dp, dp, vp]),
            "ecg_debug_gram_f32": (i32, [i64, i32, i32, dp, i32, dp, dp, vp]),
            "ecg_debug_update_f32": (i32, [i64, i32, i32, dp, i32, dp, dp, vp]),
            "ecg_debug_precond_apply": (i32, [vp, i32, i32, dp, dp, vp]),
            "ecg_stats_enable": (i32, [C.c_int]),
            "ecg_progress": (i32, [i32]),
            "ecg_stats_read": (i32, [C.POINTER(KernelStats), C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class EcgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, allow=(ECG_OK,)) -> int:
    if status not in allow:
        raise EcgError(status, lib().ecg_last_error().decode())
    return status


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


class Operator:
    """Sparse SPD matrix on the device (CSR: int64 rowptr, int32 colind, float64 vals)."""

    def __init__(self, rowptr, colind, vals):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.n = int(rowptr.shape[0] - 1)
        self.nnz = int(colind.shape[0])
        h = C.c_void_p()
        check(lib().ecg_operator_create_csr(self.n, self.nnz, rowptr.ctypes.data, colind.ctypes.data,
                                            vals.ctypes.data, 0, _stream(), C.byref(h)))
        self.handle = h

    @classmethod
    def from_csr(cls, csr):
        return cls(csr.rowptr, csr.colind, csr.vals)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ecg_operator_destroy(self.handle)
            self.handle = None

    def spmv(self, x, y):
        check(lib().ecg_spmv(self.handle, _ptr(x), _ptr(y), _stream()))

    def info(self):
        """(n, nnz) as the library holds them."""
        n, nnz = C.c_int64(), C.c_int64()
        check(lib().ecg_operator_info(self.handle, C.byref(n), C.byref(nnz)))
        return n.value, nnz.value


class Partition:
    """Subdomain map part[n] in [0, t) (every subdomain non-empty)."""

    def __init__(self, part, t: int):
        part = np.ascontiguousarray(part, dtype=np.int32)
        self.n = int(part.shape[0])
        self.t = int(t)
        h = C.c_void_p()
        check(lib().ecg_partition_create(self.n, self.t, part.ctypes.data, 0, _stream(), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ecg_partition_destroy(self.handle)
            self.handle = None


class Precond:
    """Split preconditioner M = L L^T (block-Jacobi IC(0), or M^{-1} = G G^T)."""

    def __init__(self, handle):
        self.handle = handle

    @classmethod
    def bj_ic0(cls, op: Operator, part: Partition):
        h = C.c_void_p()
        check(lib().ecg_precond_create_bj_ic0(op.handle, part.handle, _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def bj(cls, op: Operator, blocks, kind: int = 1):
        """Block-Jacobi on blocks independent of the partition (kind BJ_IC0 or BJ_CHOL)."""
        blocks = np.ascontiguousarray(blocks, dtype=np.int32)
        h = C.c_void_p()
        check(lib().ecg_precond_create_bj(op.handle, int(blocks.max()) + 1, blocks.ctypes.data, 0, kind, _stream(),
                                          C.byref(h)))
        return cls(h)

    @classmethod
    def factor(cls, rowptr, colind, vals):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        n = rowptr.shape[0] - 1
        h = C.c_void_p()
        check(lib().ecg_precond_create_factor(n, colind.shape[0], rowptr.ctypes.data, colind.ctypes.data,
                                              vals.ctypes.data, 0, _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def factor_device(cls, n, nnz, rowptr_t, colind_t, vals_t):
        """G from device tensors (int64 rowptr, int32 colind, float64 vals)."""
        h = C.c_void_p()
        check(lib().ecg_precond_create_factor(n, nnz, _ptr(rowptr_t), _ptr(colind_t), _ptr(vals_t), 1,
                                              _stream(), C.byref(h)))
        return cls(h)

    def apply(self, which: int, t: int, X, Y):
        check(lib().ecg_debug_precond_apply(self.handle, which, t, _ptr(X), _ptr(Y), _stream()))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ecg_precond_destroy(self.handle)
            self.handle = None


def options(**kw) -> Options:
    """ecg_options with the library defaults, overridden by keyword arguments."""
    o = Options()
    check(lib().ecg_options_default(C.byref(o)))
    sched = kw.pop("schedule", None)
    M = kw.pop("M", None)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    if sched:
        arr = (C.c_int32 * len(sched))(*sched)
        o.schedule = C.cast(arr, C.POINTER(C.c_int32))
        o.n_schedule = len(sched)
        o._sched_keepalive = arr
    if M is not None:
        o.precond = PRECOND_SPLIT
        o.M = M.handle
        o._M_keepalive = M
    return o


def workspace_size(op: Operator, part: Partition, opts: Options) -> int:
    out = C.c_size_t()
    check(lib().ecg_workspace_size(op.handle, part.handle, C.byref(opts), C.byref(out)))
    return int(out.value)


def _check_vectors(op: Operator, b, x):
    import torch

    for name, v in (("b", b), ("x", x)):
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.dim() == 1
                and v.is_contiguous() and v.numel() == op.n):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of length n = {op.n}")


def solve(op: Operator, part: Partition, b, x, opts: Options, workspace=None, rho_hist: bool = False):
    """Run ecg_solve on device tensors b, x (float64, length n); x holds x0 on entry.

    Returns (report dict, rho history or None).  The workspace is a uint8 CUDA tensor
    of at least workspace_size bytes (allocated here when not given).
    """
    import torch

    _check_vectors(op, b, x)
    need = workspace_size(op, part, opts)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    if workspace.numel() < need:
        raise ValueError("workspace too small")
    rep = Report()
    hist = None
    hp = None
    if rho_hist:
        hist = np.zeros(opts.kmax + 1, dtype=np.float64)
        hp = hist.ctypes.data
    st = lib().ecg_solve(op.handle, part.handle, _ptr(b), _ptr(x), C.byref(opts), _ptr(workspace), need,
                         _stream(), C.byref(rep), hp)
    check(st, allow=(ECG_OK, ECG_ENOTCONV, ECG_EBREAKDOWN))
    d = rep.as_dict()
    if hist is not None:
        hist = hist[: d["iters"] + 1]
    return d, hist


def solve_noalloc(op: Operator, part: Partition, b, x, opts: Options, rho_hist: bool = False):
    """Run ecg_solve_noalloc (the solve in the library's static 64 MiB device workspace, no
    allocation) on device tensors b, x; returns what solve() returns."""
    _check_vectors(op, b, x)
    rep = Report()
    hist = np.zeros(opts.kmax + 1, dtype=np.float64) if rho_hist else None
    st = lib().ecg_solve_noalloc(op.handle, part.handle, _ptr(b), _ptr(x), C.byref(opts), _stream(), C.byref(rep),
                                 None if hist is None else hist.ctypes.data)
    check(st, allow=(ECG_OK, ECG_ENOTCONV, ECG_EBREAKDOWN))
    d = rep.as_dict()
    if hist is not None:
        hist = hist[: d["iters"] + 1]
    return d, hist


def debug_spmm(op: Operator, t: int, X, Y):
    check(lib().ecg_debug_spmm(op.handle, t, _ptr(X), _ptr(Y), _stream()))


SPMM_AUTO, SPMM_CSR, SPMM_DIA, SPMM_GRID, SPMM_GRID_LDS, SPMM_GRID_DMA, SPMM_SELL = -1, 0, 1, 2, 3, 4, 5


def debug_spmm_kernel(op: Operator, kernel: int, t: int, X, Y):
    """Y = A X with a chosen product kernel (SPMM_*); FP64 or FP32 tensors."""
    prec = 1 if str(X.dtype) == "torch.float32" else 0
    check(lib().ecg_debug_spmm_kernel(op.handle, kernel, prec, t, _ptr(X), _ptr(Y), _stream()))


def debug_split(part: Partition, level: int, v, out):
    check(lib().ecg_debug_split(part.handle, level, _ptr(v), _ptr(out), _stream()))


def debug_gram(n, nb, wq, Q, t, Y, G):
    """G = Q^T Y; FP64 or FP32 tensors (all of one type)."""
    fn = lib().ecg_debug_gram_f32 if str(Q.dtype) == "torch.float32" else lib().ecg_debug_gram
    check(fn(n, nb, wq, _ptr(Q), t, _ptr(Y), _ptr(G), _stream()))


def debug_update(n, nb, wq, Q, t, G, W):
    """W -= Q G; FP64 or FP32 tensors (all of one type)."""
    fn = lib().ecg_debug_update_f32 if str(Q.dtype) == "torch.float32" else lib().ecg_debug_update
    check(fn(n, nb, wq, _ptr(Q), t, _ptr(G), _ptr(W), _stream()))


def stats_enable(on: bool = True):
    check(lib().ecg_stats_enable(1 if on else 0))


def stats_read(reset: bool = True) -> dict:
    """Per kernel class: launches, summed event milliseconds, algorithmic bytes and flops."""
    st = KernelStats()
    check(lib().ecg_stats_read(C.byref(st), 1 if reset else 0))
    return {name: {"count": int(st.count[i]), "ms": st.ms[i], "bytes": st.bytes[i], "flops": st.flops[i]}
            for i, name in enumerate(STAT_NAMES)}


def progress(every: int):
    """Print a progress line to stderr every `every` iterations (0 = off)."""
    check(lib().ecg_progress(int(every)))
