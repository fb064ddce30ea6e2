"""ctypes binding of libracmb.so (the gfx950 RAC-MBADMM library, include/racmb.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device memory comes from torch tensors on ``cuda`` (ROCm) and the work
is enqueued on torch's current stream.  If the shared library has not been
built, importing works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libracmb.so")

RAC_OK, RAC_ERR_ARG, RAC_ERR_NOT_PD, RAC_ERR_DEVICE, RAC_ERR_NOMEM, RAC_ERR_UNSUPPORTED = range(6)
RUN_CONVERGED, RUN_MAX_ITER, RUN_DIVERGED = 0, 1, 2
PROX_NONE, PROX_EN, PROX_BOX = 0, 1, 2
DT_F64, DT_F32, DT_BF16 = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
BETA_FIXED, BETA_RESBAL, BETA_MLP, BETA_SCHEDULE = 0, 1, 2, 3
BSWEEP_AUTO, BSWEEP_LANE, BSWEEP_TEAM = 0, 1, 2
VARIANT_RAC, VARIANT_RP = 0, 1
MAX_BLOCK = 128
MAX_EQ = 16
MLP_IN, MLP_HIDDEN = 8, 64
MLP_NPARAM = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1

EXPORTED = ["rac_solver_create", "rac_solver_destroy", "rac_solver_run", "rac_solver_set_state",
            "rac_solver_get_state", "rac_solver_history", "rac_solver_set_timing", "rac_solver_timing",
            "rac_solver_set_timing_mask", "rac_solver_set_timing_stride",
            "rac_solver_info", "rac_solver_features", "rac_solver_scale_beta", "rac_state_export",
            "rac_state_import",
            "rac_permutation", "rac_kkt", "rac_objective", "rac_regression_c", "rac_block_matrices",
            "rac_mlp_forward", "rac_mlp_loss_grad", "rac_mlp_adam", "rac_batch_create",
            "rac_batch_destroy", "rac_batch_run", "rac_batch_lane", "rac_batch_info", "rac_batch_set_timing",
            "rac_batch_timing", "rac_status_str", "rac_solve", "rac_solve_batch", "rac_permutation_host",
            "rac_batch_state_export", "rac_batch_state_import", "rac_permutation_noalloc", "rac_kkt_mu",
            "rac_solver_get_multipliers", "rac_solver_set_multipliers", "rac_svm_kernel_matrix",
            "rac_svm_decision", "rac_batch_set_lane_state", "rac_regression_c_csc"]


class RacError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, status_str(code), code))


class Problem_(C.Structure):
    _fields_ = [("n", C.c_int64), ("rows", C.c_int64), ("F", C.c_void_p), ("ldF", C.c_int64),
                ("F_dtype", C.c_int32), ("prox", C.c_int32), ("Ns", C.c_double),
                ("h", C.c_void_p), ("c", C.c_void_p), ("a", C.c_void_p), ("b", C.c_double),
                ("lam", C.c_double), ("alpha", C.c_double), ("lo", C.c_double),
                ("hi", C.c_double), ("obj_const", C.c_double), ("Hd", C.c_void_p), ("ldH", C.c_int64),
                ("H_dtype", C.c_int32), ("meq", C.c_int32), ("A", C.c_void_p), ("beq", C.c_void_p),
                ("colptr", C.c_void_p), ("rowidx", C.c_void_p)]


class Opts_(C.Structure):
    _fields_ = [("num_blocks", C.c_int64), ("seed", C.c_uint64), ("instance", C.c_uint64),
                ("precision", C.c_int32), ("beta_mode", C.c_int32), ("beta0", C.c_double),
                ("rb_mu", C.c_double), ("rb_tau", C.c_double),
                ("beta_schedule", C.POINTER(C.c_double)), ("mlp_weights", C.c_void_p),
                ("mlp_ymax", C.c_double), ("check_every", C.c_int64), ("max_iter", C.c_int64),
                ("tol", C.c_double), ("sweep_groups", C.c_int32), ("row_chunks", C.c_int32),
                ("overlap", C.c_int32), ("packed", C.c_int32), ("variant", C.c_int32), ("pad0", C.c_int32)]


class Lane_(C.Structure):
    _fields_ = [("problem", C.c_int32), ("prox", C.c_int32), ("lam", C.c_double), ("alpha", C.c_double),
                ("beta0", C.c_double)]


class BatchOpts_(C.Structure):
    _fields_ = [("block_size", C.c_int64), ("seed", C.c_uint64), ("precision", C.c_int32),
                ("beta_mode", C.c_int32), ("rb_mu", C.c_double), ("rb_tau", C.c_double),
                ("mlp_weights", C.c_void_p), ("mlp_ymax", C.c_double), ("check_every", C.c_int64),
                ("max_iter", C.c_int64), ("tol", C.c_double), ("use_graph", C.c_int32), ("tune", C.c_int32),
                ("sweep", C.c_int32), ("pad0", C.c_int32)]


class Result_(C.Structure):
    _fields_ = [("iters", C.c_int64), ("status", C.c_int32), ("pad0", C.c_int32),
                ("kkt", C.c_double), ("beta", C.c_double), ("objective", C.c_double),
                ("fail_iter", C.c_int64), ("fail_block", C.c_int64)]


_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def load():
    """Load the in-tree libracmb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libracmb.so is not built: run `python -c 'import __graft_entry__ as g; "
                           "g.build()'` (hipcc, gfx950) first; there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, i64, u64, dp = C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(C.c_double)
    sig = {
        "rac_solver_create": [C.POINTER(Problem_), C.POINTER(Opts_), C.POINTER(vp)],
        "rac_solver_destroy": [vp],
        "rac_solver_run": [vp, vp, C.POINTER(Result_)],
        "rac_solver_set_state": [vp, vp, vp, vp, C.c_double, C.c_double, i64, vp],
        "rac_solver_get_state": [vp, vp, vp, vp, dp, dp, C.POINTER(i64), vp],
        "rac_solver_history": [vp, dp, i64, C.POINTER(i64)],
        "rac_solver_set_timing": [vp, C.c_int32],
        "rac_solver_set_timing_mask": [vp, C.c_uint32],
        "rac_solver_set_timing_stride": [vp, i64],
        "rac_solver_timing": [vp, dp, C.POINTER(i64)],
        "rac_solver_info": [vp, C.POINTER(i64)],
        "rac_solver_features": [vp, C.POINTER(C.c_float)],
        "rac_solver_scale_beta": [vp, C.c_double, vp],
        "rac_state_export": [vp, vp, C.POINTER(C.c_size_t)],
        "rac_state_import": [vp, vp, C.c_size_t],
        "rac_permutation": [u64, u64, i64, i64, vp, vp],
        "rac_kkt": [C.POINTER(Problem_), vp, vp, vp, C.c_double, vp, dp],
        "rac_objective": [C.POINTER(Problem_), vp, vp, dp],
        "rac_regression_c": [vp, C.c_int32, i64, i64, i64, C.c_double, vp, vp, vp],
        "rac_block_matrices": [C.POINTER(Problem_), i64, u64, u64, i64, C.c_double, C.c_int32, vp,
                               C.POINTER(i64), vp],
        "rac_mlp_forward": [vp, vp, i64, C.c_float, vp, vp],
        "rac_mlp_loss_grad": [vp, vp, vp, i64, C.c_float, vp, dp, vp],
        "rac_mlp_adam": [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float, C.c_float, vp],
        "rac_batch_create": [C.c_int32, C.POINTER(Problem_), C.c_int32, C.POINTER(Lane_),
                             C.POINTER(BatchOpts_), C.POINTER(vp)],
        "rac_batch_destroy": [vp],
        "rac_batch_run": [vp, vp, C.POINTER(i64), C.POINTER(C.c_int32)],
        "rac_batch_lane": [vp, C.c_int32, C.POINTER(Result_), vp, vp, vp],
        "rac_batch_info": [vp, C.POINTER(i64)],
        "rac_batch_set_timing": [vp, C.c_int32],
        "rac_batch_timing": [vp, dp, C.POINTER(i64)],
        "rac_solve": [C.POINTER(Problem_), C.POINTER(Opts_), vp, vp, vp, vp, dp, C.POINTER(Result_)],
        "rac_solve_batch": [C.c_int32, C.POINTER(Problem_), C.c_int32, C.POINTER(Lane_), C.POINTER(BatchOpts_),
                            vp, vp, vp, vp, C.POINTER(Result_)],
        "rac_permutation_host": [u64, u64, i64, i64, C.POINTER(C.c_int32)],
        "rac_batch_state_export": [vp, vp, C.POINTER(C.c_size_t)],
        "rac_batch_state_import": [vp, vp, C.c_size_t],
        "rac_permutation_noalloc": [u64, u64, i64, i64, vp, vp],
        "rac_kkt_mu": [C.POINTER(Problem_), vp, vp, vp, dp, i64, vp, dp],
        "rac_solver_get_multipliers": [vp, dp, i64],
        "rac_solver_set_multipliers": [vp, dp, i64],
        "rac_svm_kernel_matrix": [vp, C.c_int32, i64, i64, vp, C.c_double, vp, i64, vp],
        "rac_svm_decision": [vp, C.c_int32, i64, i64, vp, vp, C.c_double, C.c_double, vp, i64, vp, vp, dp, vp],
        "rac_batch_set_lane_state": [vp, C.c_int32, vp, vp, vp, C.c_double, C.c_double],
        "rac_regression_c_csc": [vp, vp, vp, C.c_int32, i64, i64, C.c_double, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.rac_status_str.argtypes = [C.c_int]
    lib.rac_status_str.restype = C.c_char_p
    _lib = lib
    return lib


def status_str(code) -> str:
    try:
        return load().rac_status_str(int(code)).decode()
    except RuntimeError:
        return "status %d" % int(code)


def _check(code, what):
    if code != RAC_OK:
        raise RacError(code, what)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


_DT = {"f64": DT_F64, "f32": DT_F32, "bf16": DT_BF16}


def _torch_dtype(storage):
    torch = _torch()
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[storage]


# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """Device-resident problem (torch tensors keep the memory alive)."""
    F: object            # torch tensor (n, rows) contiguous == column-major rows x n
    storage: str
    rows: int
    n: int
    Ns: float
    c: object
    h: object = None
    a: object = None
    b: float = 0.0
    prox: int = PROX_NONE
    lam: float = 0.0
    alpha: float = 1.0
    lo: float = 0.0
    hi: float = 0.0
    obj_const: float = 0.0
    Hd: object = None    # dense form: torch tensor (n, n) symmetric (column-major = row-major), f64 or f32
    A: object = None     # dense form: torch tensor (meq, n) float64, row-major
    beq: object = None   # dense form: torch tensor (meq,) float64
    colptr: object = None  # sparse form: torch int64 tensor (n + 1,); F then holds the values
    rowidx: object = None  # sparse form: torch int32 tensor (nnz,)

    @property
    def ldF(self) -> int:
        """Leading dimension of the column-major data: F is an (n, ldF)-strided tensor view."""
        if self.F is None or self.colptr is not None:
            return 0
        assert self.F.stride(1) == 1 and self.F.stride(0) >= self.rows
        return int(self.F.stride(0))

    @property
    def meq(self) -> int:
        return 0 if self.A is None else int(self.A.shape[0])

    def struct(self) -> Problem_:
        hd_dt, ldH = DT_F64, 0
        if self.Hd is not None:
            assert self.Hd.stride(1) == 1
            ldH = int(self.Hd.stride(0))
            hd_dt = DT_F32 if self.Hd.dtype == _torch().float32 else DT_F64
        return Problem_(self.n, self.rows, None if self.F is None else self.F.data_ptr(), self.ldF,
                        _DT[self.storage], self.prox, self.Ns, None if self.h is None else self.h.data_ptr(),
                        self.c.data_ptr(), None if self.a is None else self.a.data_ptr(), self.b, self.lam,
                        self.alpha, self.lo, self.hi, self.obj_const,
                        None if self.Hd is None else self.Hd.data_ptr(), ldH, hd_dt, self.meq,
                        None if self.A is None else self.A.data_ptr(),
                        None if self.beq is None else self.beq.data_ptr(),
                        None if self.colptr is None else self.colptr.data_ptr(),
                        None if self.rowidx is None else self.rowidx.data_ptr())


def upload_columns(D, storage, device="cuda", align=8):
    """Column-major rows x n data (numpy, values exact in `storage`) -> device tensor view
    (n, rows) whose columns start at multiples of `align` elements (leading dimension
    rows rounded up; the padding is zero), so that the kernels can use aligned vector loads."""
    torch = _torch()
    Dt = np.ascontiguousarray(np.asarray(D).T)
    if storage == "f64":
        t = torch.from_numpy(Dt.astype(np.float64))
    elif storage == "f32":
        t = torch.from_numpy(Dt.astype(np.float32))
    else:  # bf16: values are exactly representable, so the conversion is exact
        t = torch.from_numpy(Dt.astype(np.float32)).to(torch.bfloat16)
    n, rows = t.shape
    ld = -(-rows // align) * align
    buf = torch.zeros((n, ld), dtype=t.dtype, device=device)
    buf[:, :rows] = t.to(device)
    return buf[:, :rows]


def regression_problem(D, y, lam=0.0, alpha=1.0, storage="f64", h=None, device="cuda") -> Problem:
    """Elastic net (Sec.3.1): H = D'D/N, c = -D'y/N computed on the device."""
    torch = _torch()
    load()
    N, n = D.shape
    F = upload_columns(D, storage, device)
    yt = torch.as_tensor(np.asarray(y, dtype=np.float64), device=device)
    c = torch.empty(n, dtype=torch.float64, device=device)
    _check(load().rac_regression_c(C.c_void_p(F.data_ptr()), _DT[storage], N, n, int(F.stride(0)), float(N),
                                   _ptr(yt), _ptr(c), _stream()), "rac_regression_c")
    ht = None if h is None else torch.as_tensor(np.asarray(h, dtype=np.float64), device=device)
    yy = float(np.dot(np.asarray(y, dtype=np.float64), np.asarray(y, dtype=np.float64)))
    return Problem(F=F, storage=storage, rows=N, n=n, Ns=float(N), c=c, h=ht,
                   prox=PROX_EN if lam > 0 else PROX_NONE, lam=float(lam), alpha=float(alpha),
                   obj_const=yy / (2.0 * N))


def regression_problem_tensor(F, y, lam=0.0, alpha=1.0, storage="bf16", h=None) -> Problem:
    """Elastic net from a device tensor F of shape (n, N) (column-major N x n data; a
    row-strided view (n, ldF) with ldF >= N is allowed)."""
    torch = _torch()
    n, N = F.shape
    dev = F.device
    yt = torch.as_tensor(np.asarray(y, dtype=np.float64), device=dev)
    c = torch.empty(n, dtype=torch.float64, device=dev)
    assert F.stride(1) == 1 and F.stride(0) >= N
    _check(load().rac_regression_c(C.c_void_p(F.data_ptr()), _DT[storage], N, n, int(F.stride(0)), float(N),
                                   _ptr(yt), _ptr(c), _stream()), "rac_regression_c")
    ht = None if h is None else torch.as_tensor(np.asarray(h, dtype=np.float64), device=dev)
    yy = float(np.dot(np.asarray(y, dtype=np.float64), np.asarray(y, dtype=np.float64)))
    return Problem(F=F, storage=storage, rows=int(N), n=int(n), Ns=float(N), c=c, h=ht,
                   prox=PROX_EN if lam > 0 else PROX_NONE, lam=float(lam), alpha=float(alpha),
                   obj_const=yy / (2.0 * N))


def svm_problem(X, labels, Cbox, storage="f32", device="cuda") -> Problem:
    """C-SVC dual (Sec.3.2), linear kernel: F = G' with G = diag(y) X, c = -e, a = y, box [0, C]."""
    torch = _torch()
    X = np.asarray(X)
    yl = np.asarray(labels, dtype=np.float64)
    n, r = X.shape
    G = X * yl[:, None].astype(X.dtype)        # a sign flip: exact in any precision
    F = upload_columns(G.T, storage, device)   # column j of F is row j of G
    c = torch.full((n,), -1.0, dtype=torch.float64, device=device)
    a = torch.as_tensor(yl, device=device)
    return Problem(F=F, storage=storage, rows=r, n=n, Ns=1.0, c=c, a=a, b=0.0, prox=PROX_BOX,
                   lo=0.0, hi=float(Cbox))


def sparse_regression_problem(colptr, rowidx, values, y, rows, lam=0.0, alpha=1.0, storage="f64", h=None,
                              device="cuda") -> Problem:
    """Elastic net (Sec.3.1) with sparse data F (rows x n) in compressed sparse columns (numpy or device
    tensors: colptr int64 n + 1, rowidx int32, values exact in `storage`, "f64" or "f32"):
    H = F'F/N, c = -F'y/N computed on the device."""
    torch = _torch()
    load()

    def dev(a, dt):
        return a.to(device, dt).contiguous() if hasattr(a, "data_ptr") else \
            torch.as_tensor(np.asarray(a), dtype=dt, device=device).contiguous()

    cp = dev(colptr, torch.int64)
    ri = dev(rowidx, torch.int32)
    vals = dev(values, torch.float64 if storage == "f64" else torch.float32)
    n = int(cp.shape[0]) - 1
    yt = dev(y, torch.float64)
    c = torch.empty(n, dtype=torch.float64, device=device)
    _check(load().rac_regression_c_csc(_ptr(cp), _ptr(ri), _ptr(vals), _DT[storage], int(rows), n, float(rows),
                                       _ptr(yt), _ptr(c), _stream()), "rac_regression_c_csc")
    ht = None if h is None else dev(h, torch.float64)
    yy = float(torch.dot(yt, yt).item())
    return Problem(F=vals, storage=storage, rows=int(rows), n=n, Ns=float(rows), c=c, h=ht,
                   prox=PROX_EN if lam > 0 else PROX_NONE, lam=float(lam), alpha=float(alpha),
                   obj_const=yy / (2.0 * rows), colptr=cp, rowidx=ri)


def dense_problem(Hd, c, *, A=None, beq=None, h=None, prox=PROX_NONE, lam=0.0, alpha=1.0, lo=0.0, hi=0.0,
                  obj_const=0.0, storage="f64", device="cuda") -> Problem:
    """The general QP of Eq.(1): min 1/2 x'(Hd + diag h)x + c'x + P(z) s.t. A x = beq, x = z, with an
    explicit symmetric Hd (numpy or device tensor, n x n; "f64" or "f32" storage, values exact in it)."""
    torch = _torch()
    load()
    dt = torch.float64 if storage == "f64" else torch.float32
    Ht = Hd.to(device, dt).contiguous() if hasattr(Hd, "data_ptr") else \
        torch.as_tensor(np.ascontiguousarray(np.asarray(Hd).T), dtype=dt, device=device).contiguous()
    n = int(Ht.shape[0])

    def vec(v):
        if v is None:
            return None
        return v.to(device, torch.float64).contiguous() if hasattr(v, "data_ptr") else \
            torch.as_tensor(np.asarray(v, dtype=np.float64), device=device).contiguous()

    At = None
    bt = None
    if A is not None:
        At = vec(A).reshape(-1, n).contiguous()
        bt = vec(beq).reshape(-1).contiguous()
    return Problem(F=None, storage="f64", rows=0, n=n, Ns=1.0, c=vec(c), h=vec(h), prox=int(prox), lam=float(lam),
                   alpha=float(alpha), lo=float(lo), hi=float(hi), obj_const=float(obj_const), Hd=Ht, A=At, beq=bt)


def svm_kernel_matrix(X, labels, gamma, storage="f64", device="cuda"):
    """rac_svm_kernel_matrix: Q_ij = y_i y_j exp(-gamma |x_i - x_j|^2) on the device (n x n float64)."""
    torch = _torch()
    dt = torch.float64 if storage == "f64" else torch.float32
    Xt = torch.as_tensor(np.ascontiguousarray(X), dtype=dt, device=device).contiguous()
    yt = torch.as_tensor(np.asarray(labels, dtype=np.float64), device=device)
    n, r = Xt.shape
    Q = torch.empty((n, n), dtype=torch.float64, device=device)
    _check(load().rac_svm_kernel_matrix(_ptr(Xt), _DT[storage], n, r, _ptr(yt), float(gamma), _ptr(Q), n, _stream()),
           "rac_svm_kernel_matrix")
    return Q, Xt, yt


def svm_kernel_problem(X, labels, Cbox, gamma, storage="f64", device="cuda"):
    """Gaussian-kernel C-SVC dual (Sec.3.2, Eq.(9)) in the dense form: Hd = Q (built on the device),
    c = -e, one equality row y'alpha = 0, box [0, C].  Returns (problem, device points, device labels)."""
    torch = _torch()
    Q, Xt, yt = svm_kernel_matrix(X, labels, gamma, storage, device)
    n = Q.shape[0]
    c = torch.full((n,), -1.0, dtype=torch.float64, device=device)
    prob = Problem(F=None, storage="f64", rows=0, n=n, Ns=1.0, c=c, prox=PROX_BOX, lo=0.0, hi=float(Cbox), Hd=Q,
                   A=yt.reshape(1, n).contiguous(), beq=torch.zeros(1, dtype=torch.float64, device=device))
    return prob, Xt, yt


def svm_decision(Xt, yt, alpha, gamma, bias, V, labels=None, storage="f64"):
    """rac_svm_decision: decision values at query points V (numpy m x r) and, with labels, the accuracy."""
    torch = _torch()
    dt = torch.float64 if storage == "f64" else torch.float32
    dev = Xt.device
    at = torch.as_tensor(np.asarray(alpha, dtype=np.float64), device=dev)
    Vt = torch.as_tensor(np.ascontiguousarray(V), dtype=dt, device=dev).contiguous()
    m = Vt.shape[0]
    f = torch.empty(m, dtype=torch.float64, device=dev)
    lt = None if labels is None else torch.as_tensor(np.asarray(labels, dtype=np.float64), device=dev)
    acc = C.c_double(float("nan"))
    _check(load().rac_svm_decision(_ptr(Xt), _DT[storage], Xt.shape[0], Xt.shape[1], _ptr(yt), _ptr(at),
                                   float(gamma), float(bias), _ptr(Vt), m, _ptr(f), _ptr(lt),
                                   None if lt is None else C.byref(acc), _stream()), "rac_svm_decision")
    return f.cpu().numpy(), (acc.value if lt is not None else None)


def kkt_mu(prob: Problem, x, z, xi, mu):
    """rac_kkt_mu: KKT residual parts with one multiplier per equality row."""
    torch = _torch()
    dev = prob.c.device
    ts = [torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev) for v in (x, z, xi)]
    m = np.ascontiguousarray(np.atleast_1d(np.asarray(mu, dtype=np.float64)))
    out = np.zeros(4)
    ps = prob.struct()
    _check(load().rac_kkt_mu(C.byref(ps), _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2]),
                             m.ctypes.data_as(C.POINTER(C.c_double)), int(m.size), _stream(),
                             out.ctypes.data_as(C.POINTER(C.c_double))), "rac_kkt_mu")
    return out


@dataclass
class Result:
    iters: int
    status: int
    kkt: float
    beta: float
    objective: float
    fail_iter: int
    fail_block: int


class Solver:
    """Handle around rac_solver: create once, run many times."""

    def __init__(self, prob: Problem, *, p=None, s=None, seed=0, instance=0, precision=PREC_FP64,
                 beta0=1.0, beta_mode=BETA_FIXED, rb_mu=10.0, rb_tau=2.0, beta_schedule=None,
                 mlp_weights=None, mlp_ymax=float(np.log(10.0)), check_every=10, max_iter=100,
                 tol=0.0, sweep_groups=0, row_chunks=0, overlap=True, packed=True, variant=VARIANT_RAC):
        self.lib = load()
        self.prob = prob
        if p is None:
            p = -(-prob.n // int(s))
        self.p = int(p)
        self._sched = None
        sched_ptr = None
        if beta_schedule is not None:
            self._sched = np.ascontiguousarray(beta_schedule, dtype=np.float64)
            sched_ptr = self._sched.ctypes.data_as(C.POINTER(C.c_double))
        self._w = mlp_weights
        self.opts = Opts_(self.p, int(seed), int(instance), int(precision), int(beta_mode), float(beta0),
                          float(rb_mu), float(rb_tau), sched_ptr,
                          None if mlp_weights is None else mlp_weights.data_ptr(), float(mlp_ymax),
                          int(check_every), int(max_iter), float(tol), int(sweep_groups), int(row_chunks),
                          0 if overlap else -1, 0 if packed else -1, int(variant), 0)
        self._ps = prob.struct()
        h = C.c_void_p()
        _check(self.lib.rac_solver_create(C.byref(self._ps), C.byref(self.opts), C.byref(h)),
               "rac_solver_create")
        self.h = h
        self.max_iter = int(max_iter)

    def close(self):
        if self.h:
            self.lib.rac_solver_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be finalised (torch and
        # profiler tools register their own exit handlers), and rac_*_destroy
        # synchronises the device and frees memory: make no HIP call then, the
        # process exit releases the device memory.  Call close() for a prompt release.
        # (The check is bound at definition time: module globals may be gone by then.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self, allow_not_pd=False) -> Result:
        r = Result_()
        code = self.lib.rac_solver_run(self.h, _stream(), C.byref(r))
        if code != RAC_OK and not (allow_not_pd and code == RAC_ERR_NOT_PD):
            raise RacError(code, "rac_solver_run")
        self.last_code = code
        return Result(r.iters, r.status, r.kkt, r.beta, r.objective, r.fail_iter, r.fail_block)

    def set_state(self, x, z, xi, mu=0.0, beta=None, iteration=0):
        torch = _torch()
        dev = self.prob.c.device
        xs = [torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev) if not hasattr(v, "data_ptr")
              else v.to(dev, torch.float64).contiguous() for v in (x, z, xi)]
        b = self.opts.beta0 if beta is None else beta
        _check(self.lib.rac_solver_set_state(self.h, _ptr(xs[0]), _ptr(xs[1]), _ptr(xs[2]), float(mu),
                                             float(b), int(iteration), _stream()), "rac_solver_set_state")

    def state(self):
        """(x, z, xi, mu, beta, iteration) with vectors as numpy float64."""
        torch = _torch()
        dev = self.prob.c.device
        x, z, xi = (torch.empty(self.prob.n, dtype=torch.float64, device=dev) for _ in range(3))
        mu, beta, it = C.c_double(), C.c_double(), C.c_int64()
        _check(self.lib.rac_solver_get_state(self.h, _ptr(x), _ptr(z), _ptr(xi), C.byref(mu), C.byref(beta),
                                             C.byref(it), _stream()), "rac_solver_get_state")
        return x.cpu().numpy(), z.cpu().numpy(), xi.cpu().numpy(), mu.value, beta.value, it.value

    PHASES = ("partition", "gram", "factor", "sweep", "zdual", "check")

    def set_timing(self, enable=True, phases=None, stride=1):
        """Per-phase HIP-event timing; `phases` (names) restricts it to those phases, and
        `stride` times the per-iteration phases of every stride-th iteration only."""
        _check(self.lib.rac_solver_set_timing_stride(self.h, int(stride)), "rac_solver_set_timing_stride")
        if phases is None:
            _check(self.lib.rac_solver_set_timing(self.h, 1 if enable else 0), "rac_solver_set_timing")
            return
        mask = 0
        for ph in phases:
            mask |= 1 << self.PHASES.index(ph)
        _check(self.lib.rac_solver_set_timing_mask(self.h, mask if enable else 0), "rac_solver_set_timing_mask")

    def timing(self):
        """{phase: (total ms, launches)} accumulated since set_timing."""
        ms = np.zeros(len(self.PHASES))
        cnt = (C.c_int64 * len(self.PHASES))()
        _check(self.lib.rac_solver_timing(self.h, ms.ctypes.data_as(C.POINTER(C.c_double)), cnt),
               "rac_solver_timing")
        return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(self.PHASES)}


    def info(self):
        v = (C.c_int64 * 8)()
        _check(self.lib.rac_solver_info(self.h, v), "rac_solver_info")
        return dict(p=v[0], sp=v[1], K=v[2], R=v[3], T=v[4], tileA=v[5], tileB=v[6], overlap=v[7])

    def features(self):
        """Controller features formed at the last KKT check (float32[8])."""
        out = np.zeros(MLP_IN, dtype=np.float32)
        _check(self.lib.rac_solver_features(self.h, out.ctypes.data_as(C.POINTER(C.c_float))),
               "rac_solver_features")
        return out

    def scale_beta(self, mult):
        """beta *= mult, recorded as a controller decision."""
        _check(self.lib.rac_solver_scale_beta(self.h, float(mult), _stream()), "rac_solver_scale_beta")

    def reset(self, beta=None):
        """Zero state (cold start) at iteration 0."""
        z = np.zeros(self.prob.n)
        self.set_state(z, z, z, 0.0, beta, 0)

    def history(self):
        out = np.zeros((max(self.max_iter, 1), 4))
        cnt = C.c_int64()
        _check(self.lib.rac_solver_history(self.h, out.ctypes.data_as(C.POINTER(C.c_double)),
                                           out.shape[0], C.byref(cnt)), "rac_solver_history")
        return out[:cnt.value]

    def multipliers(self):
        """Multipliers of the equality rows (numpy float64, one per row)."""
        k = self.prob.meq if self.prob.Hd is not None else (1 if self.prob.a is not None else 0)
        out = np.zeros(max(k, 1))
        _check(self.lib.rac_solver_get_multipliers(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), k),
               "rac_solver_get_multipliers")
        return out[:k]

    def set_multipliers(self, mu):
        m = np.ascontiguousarray(np.atleast_1d(np.asarray(mu, dtype=np.float64)))
        _check(self.lib.rac_solver_set_multipliers(self.h, m.ctypes.data_as(C.POINTER(C.c_double)), int(m.size)),
               "rac_solver_set_multipliers")

    def export_state(self) -> bytes:
        nb = C.c_size_t()
        _check(self.lib.rac_state_export(self.h, None, C.byref(nb)), "rac_state_export")
        buf = C.create_string_buffer(nb.value)
        _check(self.lib.rac_state_export(self.h, buf, C.byref(nb)), "rac_state_export")
        return buf.raw[:nb.value]

    def import_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.lib.rac_state_import(self.h, buf, len(blob)), "rac_state_import")


# ---------------------------------------------------------------------------

def solve(prob: Problem, *, p=None, s=None, seed=0, instance=0, precision=PREC_FP64, beta0=1.0,
          beta_mode=BETA_FIXED, rb_mu=10.0, rb_tau=2.0, beta_schedule=None, mlp_weights=None,
          mlp_ymax=float(np.log(10.0)), check_every=10, max_iter=100, tol=0.0, variant=VARIANT_RAC,
          allow_not_pd=False):
    """rac_solve: one call from the cold start; returns (Result, x, z, xi, mu) with numpy vectors."""
    torch = _torch()
    if p is None:
        p = -(-prob.n // int(s))
    sched = None if beta_schedule is None else np.ascontiguousarray(beta_schedule, dtype=np.float64)
    o = Opts_(int(p), int(seed), int(instance), int(precision), int(beta_mode), float(beta0), float(rb_mu),
              float(rb_tau), None if sched is None else sched.ctypes.data_as(C.POINTER(C.c_double)),
              None if mlp_weights is None else mlp_weights.data_ptr(), float(mlp_ymax), int(check_every),
              int(max_iter), float(tol), 0, 0, 0, 0, int(variant), 0)
    dev = prob.c.device
    x, z, xi = (torch.empty(prob.n, dtype=torch.float64, device=dev) for _ in range(3))
    mu = C.c_double()
    r = Result_()
    ps = prob.struct()
    code = load().rac_solve(C.byref(ps), C.byref(o), _stream(), _ptr(x), _ptr(z), _ptr(xi), C.byref(mu), C.byref(r))
    if code != RAC_OK and not (allow_not_pd and code == RAC_ERR_NOT_PD):
        raise RacError(code, "rac_solve")
    res = Result(r.iters, r.status, r.kkt, r.beta, r.objective, r.fail_iter, r.fail_block)
    return res, x.cpu().numpy(), z.cpu().numpy(), xi.cpu().numpy(), mu.value


def permutation_host(seed, instance, it, n):
    """rac_permutation_host: the partition draw on the CPU (numpy int32), no GPU call."""
    out = np.empty(int(n), dtype=np.int32)
    _check(load().rac_permutation_host(int(seed), int(instance), int(it), int(n),
                                       out.ctypes.data_as(C.POINTER(C.c_int32))), "rac_permutation_host")
    return out


NOALLOC_MAX_N = 262144


def permutation_noalloc(seed, instance, it, n, out):
    """rac_permutation_noalloc into the caller's int32 device tensor `out` (at least n entries),
    enqueued on torch's current stream without allocating or synchronising."""
    _check(load().rac_permutation_noalloc(int(seed), int(instance), int(it), int(n), _ptr(out), _stream()),
           "rac_permutation_noalloc")
    return out


def permutation(seed, instance, it, n, device="cuda"):
    torch = _torch()
    out = torch.empty(n, dtype=torch.int32, device=device)
    _check(load().rac_permutation(int(seed), int(instance), int(it), int(n), _ptr(out), _stream()),
           "rac_permutation")
    return out


def kkt(prob: Problem, x, z, xi, mu=0.0):
    torch = _torch()
    dev = prob.c.device
    ts = [torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev) for v in (x, z, xi)]
    out = np.zeros(4)
    ps = prob.struct()
    _check(load().rac_kkt(C.byref(ps), _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2]), float(mu), _stream(),
                          out.ctypes.data_as(C.POINTER(C.c_double))), "rac_kkt")
    return out


def objective(prob: Problem, z):
    torch = _torch()
    zt = torch.as_tensor(np.asarray(z, dtype=np.float64), device=prob.c.device)
    out = C.c_double()
    ps = prob.struct()
    _check(load().rac_objective(C.byref(ps), _ptr(zt), _stream(), C.byref(out)), "rac_objective")
    return out.value


def block_matrices(prob: Problem, p, seed, instance, it, beta, precision=PREC_FP64):
    torch = _torch()
    smax = -(-prob.n // p)
    sp = 16
    while sp < smax:
        sp *= 2
    out = torch.zeros(p * sp * sp, dtype=torch.float64, device=prob.c.device)
    spo = C.c_int64()
    ps = prob.struct()
    _check(load().rac_block_matrices(C.byref(ps), int(p), int(seed), int(instance), int(it), float(beta),
                                     int(precision), _ptr(out), C.byref(spo), _stream()),
           "rac_block_matrices")
    assert spo.value == sp
    return out.cpu().numpy().reshape(p, sp, sp), sp


def mlp_forward(w, feats, ymax=float(np.log(10.0))):
    torch = _torch()
    y = torch.empty(feats.shape[0], dtype=torch.float32, device=w.device)
    _check(load().rac_mlp_forward(_ptr(w), _ptr(feats), feats.shape[0], float(ymax), _ptr(y), _stream()),
           "rac_mlp_forward")
    return y


def mlp_loss_grad(w, feats, target, ymax=float(np.log(10.0))):
    torch = _torch()
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=w.device)
    loss = C.c_double()
    _check(load().rac_mlp_loss_grad(_ptr(w), _ptr(feats), _ptr(target), feats.shape[0], float(ymax),
                                    _ptr(g), C.byref(loss), _stream()), "rac_mlp_loss_grad")
    return loss.value, g


def mlp_adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().rac_mlp_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), int(t), float(lr), float(b1),
                               float(b2), float(eps), _stream()), "rac_mlp_adam")


# ---------------------------------------------------------------------------

class Batch:
    """Handle around rac_batch: many instances x lanes advanced together.

    lanes: list of (problem index, prox, lambda, alpha, beta0)."""

    def __init__(self, probs, lanes, *, s=64, seed=0, precision=PREC_FP64, beta_mode=BETA_FIXED,
                 rb_mu=10.0, rb_tau=2.0, mlp_weights=None, mlp_ymax=float(np.log(10.0)), check_every=10,
                 max_iter=100, tol=0.0, use_graph=True, tune=False, sweep=BSWEEP_AUTO):
        self.lib = load()
        self.probs = list(probs)
        self._ps = (Problem_ * len(self.probs))(*[p.struct() for p in self.probs])
        self._ls = (Lane_ * len(lanes))(*[Lane_(int(a), int(b), float(c), float(d), float(e))
                                          for a, b, c, d, e in lanes])
        self.lanes = list(lanes)
        self._w = mlp_weights
        o = BatchOpts_(int(s), int(seed), int(precision), int(beta_mode), float(rb_mu), float(rb_tau),
                       None if mlp_weights is None else mlp_weights.data_ptr(), float(mlp_ymax),
                       int(check_every), int(max_iter), float(tol), 1 if use_graph else 0, 1 if tune else 0,
                       int(sweep), 0)
        self.opts = o
        h = C.c_void_p()
        _check(self.lib.rac_batch_create(len(self.probs), self._ps, len(lanes), self._ls, C.byref(o),
                                         C.byref(h)), "rac_batch_create")
        self.h = h

    def close(self):
        if self.h:
            self.lib.rac_batch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be finalised (torch and
        # profiler tools register their own exit handlers), and rac_*_destroy
        # synchronises the device and frees memory: make no HIP call then, the
        # process exit releases the device memory.  Call close() for a prompt release.
        # (The check is bound at definition time: module globals may be gone by then.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self):
        """(iterations run, lanes still active)."""
        it, act = C.c_int64(), C.c_int32()
        _check(self.lib.rac_batch_run(self.h, _stream(), C.byref(it), C.byref(act)), "rac_batch_run")
        return it.value, act.value

    def lane(self, u, allow_not_pd=False):
        """(Result, x, z, xi) of lane u, vectors as numpy float64."""
        torch = _torch()
        n = self.probs[self.lanes[u][0]].n
        dev = self.probs[0].c.device
        x, z, xi = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        r = Result_()
        code = self.lib.rac_batch_lane(self.h, int(u), C.byref(r), _ptr(x), _ptr(z), _ptr(xi))
        if code != RAC_OK and not (allow_not_pd and code == RAC_ERR_NOT_PD):
            raise RacError(code, "rac_batch_lane")
        res = Result(r.iters, r.status, r.kkt, r.beta, r.objective, r.fail_iter, r.fail_block)
        return res, x.cpu().numpy(), z.cpu().numpy(), xi.cpu().numpy()

    def set_timing(self, enable=True):
        _check(self.lib.rac_batch_set_timing(self.h, 1 if enable else 0), "rac_batch_set_timing")

    def timing(self):
        """{phase: (milliseconds, launches)} since set_timing."""
        ms, cnt = (C.c_double * len(Solver.PHASES))(), (C.c_int64 * len(Solver.PHASES))()
        _check(self.lib.rac_batch_timing(self.h, ms, cnt), "rac_batch_timing")
        return {name: (ms[q], cnt[q]) for q, name in enumerate(Solver.PHASES)}

    def set_lane_state(self, u, x, z, xi, mu=0.0, beta=None):
        """Warm start of lane u from (x, z, xi, mu) (numpy or device tensors) with penalty beta."""
        torch = _torch()
        dev = self.probs[0].c.device
        ts = [v.to(dev, torch.float64).contiguous() if hasattr(v, "data_ptr") else
              torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev) for v in (x, z, xi)]
        b = self.lanes[u][4] if beta is None else beta
        _check(self.lib.rac_batch_set_lane_state(self.h, int(u), _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2]), float(mu),
                                                 float(b)), "rac_batch_set_lane_state")

    def export_state(self) -> bytes:
        nb = C.c_size_t()
        _check(self.lib.rac_batch_state_export(self.h, None, C.byref(nb)), "rac_batch_state_export")
        buf = C.create_string_buffer(nb.value)
        _check(self.lib.rac_batch_state_export(self.h, buf, C.byref(nb)), "rac_batch_state_export")
        return buf.raw[:nb.value]

    def import_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.lib.rac_batch_state_import(self.h, buf, len(blob)), "rac_batch_state_import")

    def info(self):
        v = (C.c_int64 * 10)()
        _check(self.lib.rac_batch_info(self.h, v), "rac_batch_info")
        return dict(lanes=v[0], instances=v[1], gram_tasks=v[2], inverse_tasks=v[3], unroll=v[4], graph=v[5],
                    team_size=v[6], teams=v[7], solo_groups=v[8], assembly_slots=v[9])


def solve_batch(probs, lanes, *, s=64, seed=0, precision=PREC_FP64, beta_mode=BETA_FIXED, rb_mu=10.0, rb_tau=2.0,
                mlp_weights=None, mlp_ymax=float(np.log(10.0)), check_every=10, max_iter=100, tol=0.0,
                use_graph=True, tune=False, sweep=BSWEEP_AUTO, allow_not_pd=False):
    """rac_solve_batch: one call; returns a list of (Result, x, z, xi) per lane (numpy vectors)."""
    torch = _torch()
    lib = load()
    probs = list(probs)
    ps = (Problem_ * len(probs))(*[p.struct() for p in probs])
    ls = (Lane_ * len(lanes))(*[Lane_(int(a), int(b), float(c), float(d), float(e)) for a, b, c, d, e in lanes])
    o = BatchOpts_(int(s), int(seed), int(precision), int(beta_mode), float(rb_mu), float(rb_tau),
                   None if mlp_weights is None else mlp_weights.data_ptr(), float(mlp_ymax), int(check_every),
                   int(max_iter), float(tol), 1 if use_graph else 0, 1 if tune else 0, int(sweep), 0)
    ns = [probs[l[0]].n for l in lanes]
    tot = int(sum(ns))
    dev = probs[0].c.device
    x, z, xi = (torch.empty(tot, dtype=torch.float64, device=dev) for _ in range(3))
    res = (Result_ * len(lanes))()
    code = lib.rac_solve_batch(len(probs), ps, len(lanes), ls, C.byref(o), _stream(), _ptr(x), _ptr(z), _ptr(xi),
                               res)
    if code != RAC_OK and not (allow_not_pd and code == RAC_ERR_NOT_PD):
        raise RacError(code, "rac_solve_batch")
    xs, zs, xis = x.cpu().numpy(), z.cpu().numpy(), xi.cpu().numpy()
    out, off = [], 0
    for u, n in enumerate(ns):
        r = res[u]
        out.append((Result(r.iters, r.status, r.kkt, r.beta, r.objective, r.fail_iter, r.fail_block),
                    xs[off:off + n].copy(), zs[off:off + n].copy(), xis[off:off + n].copy()))
        off += n
    return out


def solve_path(probs, lams, *, alpha, s=64, seed=0, beta_frac=0.1, warm=True, **kw):
    """A regularisation path (Sec.3.1) of every instance, solved stage by stage: stage j is one
    batch with one lane per instance at lambda lams[i][j] (penalty beta_frac * lambda), each lane
    started from the same instance's stage j-1 solution (warm=True) or cold.  Returns per stage
    the (Result, x, z, xi) of every instance's lane, and the iterations each stage ran."""
    stages, iters = [], []
    prev = None
    npts = len(lams[0])
    for j in range(npts):
        lanes = [(i, PROX_EN, float(lams[i][j]), float(alpha), beta_frac * float(lams[i][j])) for i in range(len(probs))]
        b = Batch(probs, lanes, s=s, seed=seed, **kw)
        if warm and prev is not None:
            for i, (r, x, z, xi) in enumerate(prev):
                b.set_lane_state(i, x, z, xi, 0.0, lanes[i][4])
        it, _ = b.run()
        out = [b.lane(i) for i in range(len(probs))]
        b.close()
        stages.append(out)
        iters.append(it)
        prev = out
    return stages, iters
