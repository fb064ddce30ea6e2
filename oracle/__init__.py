"""FP64 CPU oracle of RAC-MBADMM (arXiv 1907.01995) -- TEST INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
bench.py import this package.  The product (``paper_1907_01995_amd``) never
imports it, and it imports nothing from the product: the two share only the
seeded input generators in ``paper_1907_01995_amd/workloads.py``, which hold
none of the method's arithmetic.

The arithmetic lives in ``racmb_oracle.c`` (plain loops, FP64, one thread,
built with ``-ffp-contract=off``); this module compiles it with gcc when needed
and wraps it with ctypes.  The problem mappings below follow the paper:

* elastic net (Sec.3.1, Eq.(5)-(8)): ``c = -X'y/N`` and ``H = X'X/N`` (the
  paper's ``A = X/sqrt(N)``), split ``beta - z = 0`` with z as one block;
* C-SVC dual (Sec.3.2, Eq.(9)) with a linear kernel: ``Q = G G'`` where
  ``G = diag(y) X``, ``c = -e``, equality ``y'z = 0`` and the box ``[0, C]``;
  with the Gaussian kernel of Sec.3.2, ``Q_ij = y_i y_j exp(-gamma |x_i - x_j|^2)``
  is passed as the explicit dense part ``Hd`` of H;
* the general QP of Eq.(1)/Eq.(4): ``H = F'F/Ns + Hd + diag h`` and several
  equality rows ``A x = beq``.

``solve(..., rp=True)`` runs RP-MBADMM (Sec.1): contiguous fixed blocks solved
in an order drawn at random every iteration.

Functions without a pin in tests/test_oracle_pins.py would be marked
"parity unpinned" here; at present every function below has one.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "racmb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libracmb_oracle.so")

PROX_NONE, PROX_EN, PROX_BOX = 0, 1, 2
BETA_FIXED, BETA_RESBAL, BETA_MLP, BETA_SCHEDULE = 0, 1, 2, 3
RUN_CONVERGED, RUN_MAX_ITER, RUN_DIVERGED = 0, 1, 2
ERR_ARG, ERR_NOT_PD = 1, 2
MLP_IN, MLP_H = 8, 64

_lib = None


def build(force: bool = False) -> str:
    """Compile racmb_oracle.c into a shared library next to it (gcc, plain -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    i64, u64 = C.c_int64, C.c_uint64
    lib.orc_perm_key.restype = u64
    lib.orc_perm_key.argtypes = [u64, u64, u64, u64]
    lib.orc_splitmix64_next.restype = u64
    lib.orc_splitmix64_next.argtypes = [C.POINTER(u64)]
    lib.orc_permutation.restype = None
    lib.orc_permutation.argtypes = [u64, u64, u64, i64, C.POINTER(C.c_int32)]
    lib.orc_block_start.restype = i64
    lib.orc_block_start.argtypes = [i64, i64, i64]
    lib.orc_soft.restype = C.c_double
    lib.orc_soft.argtypes = [C.c_double, C.c_double]
    lib.orc_paper_S.restype = C.c_double
    lib.orc_paper_S.argtypes = [C.c_double, C.c_double]
    lib.orc_kkt.restype = C.c_double
    lib.orc_kkt.argtypes = [i64, i64, dp, C.c_double, dp, dp, dp, i64, dp, dp, C.c_int,
                            C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp,
                            dp, dp]
    lib.orc_objective.restype = C.c_double
    lib.orc_objective.argtypes = [i64, i64, dp, C.c_double, dp, dp, dp, C.c_int, C.c_double,
                                  C.c_double, C.c_double, dp]
    lib.orc_mlp_nparam.restype = i64
    lib.orc_mlp_forward.restype = None
    lib.orc_mlp_forward.argtypes = [i64, dp, C.c_double, dp, dp]
    lib.orc_mlp_loss_grad.restype = C.c_double
    lib.orc_mlp_loss_grad.argtypes = [i64, dp, C.c_double, dp, dp, dp]
    lib.orc_adam_step.restype = None
    lib.orc_adam_step.argtypes = [i64, dp, dp, dp, dp, i64, C.c_double, C.c_double, C.c_double,
                                  C.c_double]
    lib.orc_controller_features.restype = None
    lib.orc_controller_features.argtypes = [C.c_double] * 7 + [i64, dp]
    lib.orc_solve.restype = C.c_int
    lib.orc_solve.argtypes = [
        i64, i64, dp, C.c_double, dp, dp, dp, i64, dp, dp, C.c_int, C.c_double, C.c_double,
        C.c_double, C.c_double,
        i64, C.c_int, u64, u64, i64,
        C.c_int, C.c_double, dp, C.c_double, C.c_double,
        dp, C.c_double,
        i64, i64, C.c_double,
        dp, dp, dp, dp,
        dp, C.POINTER(i64), C.POINTER(C.c_int), dp, C.POINTER(i64), C.POINTER(i64)]
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, order="C"):
    if a is None:
        return None
    return np.require(np.asarray(a, dtype=np.float64), requirements=[order, "A", "W"])


# ---------------------------------------------------------------------------
# Problem description (oracle-side; the product has its own).

@dataclass
class Problem:
    """min 1/2 x'(F'F/Ns + Hd + diag h)x + c'x + P(z) + obj_const s.t. A x = beq, x = z.

    One equality row can be given as ``a`` (n) and ``b``; several as ``A``
    (meq x n) and ``beq`` (meq).  ``F`` may have zero rows when ``Hd`` carries H."""
    F: np.ndarray                  # rowsF x n, float64, column-major
    Ns: float
    c: np.ndarray
    h: np.ndarray | None = None
    a: np.ndarray | None = None
    b: float = 0.0
    prox: int = PROX_NONE
    lam: float = 0.0
    alpha: float = 1.0
    lo: float = 0.0
    hi: float = 0.0
    obj_const: float = 0.0
    Hd: np.ndarray | None = None   # n x n dense symmetric addend of H
    A: np.ndarray | None = None    # meq x n equality rows
    beq: np.ndarray | None = None  # meq

    @property
    def n(self):
        return self.F.shape[1]

    @property
    def m(self):
        return self.F.shape[0]

    def eq(self):
        """(meq, A as a C-ordered meq x n float64 array or None, beq or None)."""
        if self.A is not None:
            A = _f64(np.atleast_2d(self.A))
            return A.shape[0], A, _f64(np.atleast_1d(self.beq))
        if self.a is not None:
            return 1, _f64(np.asarray(self.a)[None, :]), np.array([float(self.b)])
        return 0, None, None

    def Hd_f(self):
        return None if self.Hd is None else _f64(self.Hd, order="F")


def en_problem(D, y, lam=0.0, alpha=1.0, h=None) -> Problem:
    """Elastic net of Eq.(5)/(8) with the data mapping of Sec.3.1: c = -D'y/N, H = D'D/N.

    ``lam == 0`` is ordinary least squares (no penalty, prox NONE)."""
    D = np.asfortranarray(np.asarray(D, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    N = D.shape[0]
    c = -(D.T @ y) / N
    prox = PROX_EN if lam > 0 else PROX_NONE
    return Problem(F=D, Ns=float(N), c=c, h=None if h is None else _f64(h), prox=prox,
                   lam=float(lam), alpha=float(alpha), obj_const=float(y @ y) / (2.0 * N))


def svm_problem(X, labels, Cbox) -> Problem:
    """C-SVC dual of Eq.(9), linear kernel: Q = G G' with G = diag(y) X, so F = G'."""
    X = np.asarray(X, dtype=np.float64)
    yl = np.asarray(labels, dtype=np.float64)
    G = X * yl[:, None]                   # n x r
    F = np.asfortranarray(G.T)            # r x n
    n = X.shape[0]
    return Problem(F=F, Ns=1.0, c=-np.ones(n), a=yl.copy(), b=0.0, prox=PROX_BOX, lo=0.0,
                   hi=float(Cbox))


def gaussian_kernel(X, Y, gamma):
    """K_ij = exp(-gamma |x_i - y_j|^2), the kernel of the SVM experiments (Sec.3.2)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = np.empty((X.shape[0], Y.shape[0]))
    for i in range(X.shape[0]):
        diff = Y - X[i]
        d[i] = np.sum(diff * diff, axis=1)
    return np.exp(-gamma * d)


def svm_kernel_problem(X, labels, Cbox, gamma) -> Problem:
    """C-SVC dual of Eq.(9) with the Gaussian kernel: H = Q, Q_ij = y_i y_j K_ij, given
    explicitly (no factor F), c = -e, equality y'z = 0, box [0, C]."""
    yl = np.asarray(labels, dtype=np.float64)
    n = yl.shape[0]
    Q = yl[:, None] * gaussian_kernel(X, X, gamma) * yl[None, :]
    return Problem(F=np.zeros((0, n), order="F"), Ns=1.0, c=-np.ones(n), a=yl.copy(), b=0.0,
                   prox=PROX_BOX, lo=0.0, hi=float(Cbox), Hd=np.asfortranarray(Q))


def svm_bias(res) -> float:
    """Bias of the decision function: b = -mu, the multiplier of y'alpha = 0 (on a
    free support vector i, y_i f(x_i) = 1 gives b = y_i - sum_j alpha_j y_j K_ij)."""
    return -float(np.atleast_1d(res.mu)[0])


def svm_decision(X_train, labels, alpha, bias, gamma, X_test):
    """f(x) = sum_j alpha_j y_j K(x_j, x) + b (Gaussian kernel; gamma None: linear kernel)."""
    coef = np.asarray(alpha, dtype=np.float64) * np.asarray(labels, dtype=np.float64)
    if gamma is None:
        w = np.asarray(X_train, dtype=np.float64).T @ coef
        return np.asarray(X_test, dtype=np.float64) @ w + bias
    return gaussian_kernel(X_test, X_train, gamma) @ coef + bias


def svm_accuracy(f, labels) -> float:
    """Fraction of points whose label has the sign of the decision value (f = 0 counts as +1)."""
    pred = np.where(np.asarray(f) >= 0.0, 1.0, -1.0)
    return float(np.mean(pred == np.asarray(labels)))


# ---------------------------------------------------------------------------

def perm_key(seed, inst, it, j) -> int:
    return int(_load().orc_perm_key(seed, inst, it, j))


def splitmix64_sequence(seed: int, count: int):
    st = C.c_uint64(seed)
    return [int(_load().orc_splitmix64_next(C.byref(st))) for _ in range(count)]


def permutation(seed, inst, it, n) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().orc_permutation(seed, inst, it, n, out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


def block_starts(n, p) -> np.ndarray:
    lib = _load()
    return np.array([lib.orc_block_start(i, n, p) for i in range(p + 1)], dtype=np.int64)


def blocks(seed, inst, it, n, p):
    pm = permutation(seed, inst, it, n)
    st = block_starts(n, p)
    return [pm[st[i]:st[i + 1]].copy() for i in range(p)]


def soft(a, b) -> float:
    return float(_load().orc_soft(a, b))


def paper_S(a, b) -> float:
    return float(_load().orc_paper_S(a, b))


def _mu_vec(meq, mu):
    v = np.zeros(max(meq, 1))
    if meq:
        v[:meq] = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    return v


def kkt(P: Problem, x, z, xi, mu=0.0, parts=False):
    out = np.zeros(3)
    x, z, xi = _f64(x), _f64(z), _f64(xi)
    meq, A, beq = P.eq()
    muv = _mu_vec(meq, mu)
    Hd = P.Hd_f()
    v = _load().orc_kkt(P.n, P.m, _dp(P.F), P.Ns, _dp(Hd), _dp(P.h), _dp(P.c), meq, _dp(A), _dp(beq),
                        P.prox, P.lam, P.alpha, P.lo, P.hi, _dp(x), _dp(z), _dp(xi), _dp(muv), _dp(out))
    return (float(v), out) if parts else float(v)


def objective(P: Problem, z) -> float:
    z = _f64(z)
    Hd = P.Hd_f()
    return float(_load().orc_objective(P.n, P.m, _dp(P.F), P.Ns, _dp(Hd), _dp(P.h), _dp(P.c), P.prox,
                                       P.lam, P.alpha, P.obj_const, _dp(z)))


# ---------------------------------------------------------------------------
# Penalty controller network (project addition; FP64 here).

def mlp_nparam() -> int:
    return int(_load().orc_mlp_nparam())


def mlp_forward(w, feats, ymax=np.log(10.0)):
    feats = _f64(np.atleast_2d(feats))
    w = _f64(w)
    y = np.zeros(feats.shape[0])
    _load().orc_mlp_forward(feats.shape[0], _dp(w), ymax, _dp(feats), _dp(y))
    return y


def mlp_loss_grad(w, feats, target, ymax=np.log(10.0)):
    feats = _f64(np.atleast_2d(feats))
    w = _f64(w)
    t = _f64(target)
    g = np.zeros(mlp_nparam())
    loss = _load().orc_mlp_loss_grad(feats.shape[0], _dp(w), ymax, _dp(feats), _dp(t), _dp(g))
    return float(loss), g


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays w, m, v."""
    _load().orc_adam_step(w.size, _dp(w), _dp(_f64(g)), _dp(m), _dp(v), t, lr, b1, b2, eps)


def controller_features(rp_now, rd_now, rp_old, rd_old, kkt_now, kkt_prev, last_log10_mult,
                        decisions):
    f = np.zeros(MLP_IN)
    _load().orc_controller_features(rp_now, rd_now, rp_old, rd_old, kkt_now, kkt_prev,
                                    last_log10_mult, decisions, _dp(f))
    return f


# ---------------------------------------------------------------------------

@dataclass
class Result:
    x: np.ndarray
    z: np.ndarray
    xi: np.ndarray
    mu: object                     # float for at most one equality row, else an array
    iters: int
    status: int
    beta: float
    hist: np.ndarray = field(repr=False)
    rc: int = 0
    fail_iter: int = -1
    fail_block: int = -1

    @property
    def r_p(self):
        return self.hist[:self.iters, 0]

    @property
    def r_d(self):
        return self.hist[:self.iters, 1]

    @property
    def betas(self):
        return self.hist[:self.iters, 2]

    @property
    def kkts(self):
        return self.hist[:self.iters, 3]


def solve(P: Problem, *, p=None, s=None, seed=0, inst=0, iter0=0, beta0=1.0,
          beta_mode=BETA_FIXED, beta_sched=None, rb_mu=10.0, rb_tau=2.0, mlp_w=None,
          mlp_ymax=np.log(10.0), check_every=10, max_iter=100, tol=0.0, state=None,
          rp=False) -> Result:
    """Run RAC-MBADMM (or RP-MBADMM with ``rp=True``) from ``state`` (x, z, xi, mu)
    or from zeros.

    Give either p (number of blocks) or s (maximum block size, p = ceil(n/s))."""
    n = P.n
    if p is None:
        p = -(-n // int(s))
    meq, A, beq = P.eq()
    if state is None:
        x, z, xi, mu = np.zeros(n), np.zeros(n), np.zeros(n), 0.0
    else:
        x, z, xi, mu = (_f64(state[0]).copy(), _f64(state[1]).copy(), _f64(state[2]).copy(),
                        state[3])
    muv = _mu_vec(meq, mu)
    hist = np.full((max(max_iter, 1), 4), np.nan)
    iters, status, fi, fb = C.c_int64(0), C.c_int(0), C.c_int64(-1), C.c_int64(-1)
    beta_out = C.c_double(0.0)
    sched = _f64(beta_sched)
    w = _f64(mlp_w)
    Hd = P.Hd_f()
    rc = _load().orc_solve(
        n, P.m, _dp(P.F), P.Ns, _dp(Hd), _dp(P.h), _dp(P.c), meq, _dp(A), _dp(beq), P.prox, P.lam,
        P.alpha, P.lo, P.hi, int(p), 1 if rp else 0, int(seed), int(inst), int(iter0),
        int(beta_mode), float(beta0), _dp(sched), rb_mu, rb_tau, _dp(w), float(mlp_ymax),
        int(check_every), int(max_iter), float(tol),
        _dp(x), _dp(z), _dp(xi), _dp(muv),
        _dp(hist), C.byref(iters), C.byref(status), C.byref(beta_out), C.byref(fi), C.byref(fb))
    mu_out = float(muv[0]) if meq <= 1 and P.A is None else muv[:meq].copy()
    return Result(x=x, z=z, xi=xi, mu=mu_out, iters=int(iters.value), status=int(status.value),
                  beta=beta_out.value, hist=hist, rc=int(rc), fail_iter=int(fi.value),
                  fail_block=int(fb.value))
