"""The dense form on the GPU: the general QP of Eq.(1) with an explicit Hessian and
several equality rows (Eq.(4)), and the Gaussian-kernel C-SVC dual of Sec.3.2
(Eq.(9)), against the FP64 oracle given the same problem.

Bars: FP64 iterates within 1e-8 relative of the oracle's (RAC and RP), the
converged solution of an equality-constrained QP equal to the solution of its
KKT system (numpy), the kernel matrix and decision values equal to the oracle's
to rounding, and the bias b = -mu (the multiplier of y'alpha = 0)."""
import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import racmb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def random_qp(n, meq, seed, storage="f64", prox=racmb.PROX_NONE, lam=0.0, alpha=1.0, lo=0.0, hi=0.0):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n // 2, n))
    Hd = G.T @ G / n + 0.05 * np.eye(n)
    Hd = 0.5 * (Hd + Hd.T)
    if storage == "f32":
        Hd = Hd.astype(np.float32).astype(np.float64)   # values exact in FP32
    c = rng.standard_normal(n)
    A = rng.standard_normal((meq, n)) if meq else None
    beq = A @ rng.uniform(0.1, 0.9, n) if meq else None
    gp = racmb.dense_problem(Hd, c, A=A, beq=beq, prox=prox, lam=lam, alpha=alpha, lo=lo, hi=hi, storage=storage)
    op = O.Problem(F=np.zeros((0, n), order="F"), Ns=1.0, c=c, prox=prox, lam=lam, alpha=alpha, lo=lo, hi=hi,
                   Hd=Hd, A=A, beq=beq)
    return gp, op, Hd, c, A, beq


def run(gp, **kw):
    s = racmb.Solver(gp, **kw)
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    return s, r, x, z, xi


@pytest.mark.parametrize("variant", [racmb.VARIANT_RAC, racmb.VARIANT_RP])
@pytest.mark.parametrize("n,meq,s,prox", [(301, 3, 32, racmb.PROX_NONE), (256, 1, 64, racmb.PROX_BOX),
                                          (200, 0, 16, racmb.PROX_EN), (130, 5, 128, racmb.PROX_EN)])
def test_dense_qp_parity(variant, n, meq, s, prox):
    gp, op, *_ = random_qp(n, meq, n + meq, prox=prox, lam=0.05, alpha=0.7, lo=0.0, hi=1.0)
    say("dense qp", n, meq, s, prox, variant)
    kw = dict(s=s, beta0=0.7, beta_mode=racmb.BETA_RESBAL, max_iter=60, check_every=10, seed=3)
    sol, r, x, z, xi = run(gp, variant=variant, **kw)
    ref = O.solve(op, s=s, beta0=0.7, beta_mode=O.BETA_RESBAL, max_iter=60, check_every=10, seed=3,
                  rp=variant == racmb.VARIANT_RP)
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8, rel(a, b)
    if meq:
        assert rel(sol.multipliers(), np.atleast_1d(ref.mu)) < 1e-8
    h = sol.history()
    np.testing.assert_allclose(h[:, 0], ref.r_p, rtol=1e-6, atol=1e-14)
    np.testing.assert_array_equal(h[:, 2], ref.betas)
    np.testing.assert_allclose(h[9::10, 3], ref.kkts[9::10], rtol=1e-6, atol=1e-14)
    ob = O.objective(op, ref.z)
    assert abs(r.objective - ob) <= 1e-7 * max(1.0, abs(ob))


def test_dense_fp32_storage_parity():
    gp, op, *_ = random_qp(260, 0, 5, storage="f32", prox=racmb.PROX_EN, lam=0.02, alpha=0.5)
    assert gp.Hd.dtype == torch.float32
    sol, r, x, z, xi = run(gp, s=32, beta0=0.5, max_iter=40, check_every=10, seed=1)
    ref = O.solve(op, s=32, beta0=0.5, max_iter=40, check_every=10, seed=1)
    assert rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8


def test_dense_equality_qp_reaches_kkt_system_solution():
    """min 1/2 x'Hx + c'x s.t. A x = beq (no prox): the bordered KKT system
    [[H, A'], [A, 0]] [x; -mu] = [-c; beq] gives the solution and multipliers."""
    n, meq = 180, 4
    gp, op, Hd, c, A, beq = random_qp(n, meq, 77)
    K = np.block([[Hd, A.T], [A, np.zeros((meq, meq))]])
    sol_ = np.linalg.solve(K, np.concatenate([-c, beq]))
    xs, mus = sol_[:n], -sol_[n:]
    say("dense equality qp to KKT 1e-10")
    s, r, x, z, xi = run(gp, s=32, beta0=1.0, beta_mode=racmb.BETA_RESBAL, max_iter=3000, check_every=10,
                         tol=1e-11, seed=2)
    assert r.status == racmb.RUN_CONVERGED
    assert rel(z, xs) < 1e-8
    assert rel(s.multipliers(), mus) < 1e-7
    k = racmb.kkt_mu(gp, x, z, xi, s.multipliers())
    kk, _ = O.kkt(op, x, z, xi, s.multipliers(), parts=True)
    assert abs(k[0] - kk) <= 1e-10 + 1e-8 * kk


def test_dense_kkt_and_objective_match_oracle():
    rng = np.random.default_rng(9)
    for meq, prox in ((0, racmb.PROX_EN), (1, racmb.PROX_BOX), (3, racmb.PROX_NONE)):
        gp, op, *_ = random_qp(150, meq, 40 + meq, prox=prox, lam=0.1, alpha=0.4, lo=0.0, hi=2.0)
        for _ in range(2):
            x, z, xi = rng.standard_normal(150), rng.standard_normal(150), rng.standard_normal(150)
            if prox == racmb.PROX_BOX:
                z = np.clip(z, 0, 2)
            z[::4] = 0.0
            mu = rng.standard_normal(meq)
            got = racmb.kkt_mu(gp, x, z, xi, mu)
            k, parts = O.kkt(op, x, z, xi, mu, parts=True)
            assert abs(got[0] - k) <= 1e-12 * k
            np.testing.assert_allclose(got[1:], parts, rtol=1e-12)
            if meq <= 1:
                g1 = racmb.kkt(gp, x, z, xi, float(mu[0]) if meq else 0.0)
                np.testing.assert_allclose(g1, got, rtol=0, atol=0)
            ob = O.objective(op, z)
            assert abs(racmb.objective(gp, z) - ob) <= 1e-12 * abs(ob)


def test_dense_block_matrices_match_definition():
    gp, op, Hd, c, A, beq = random_qp(97, 1, 3)
    h = np.linspace(0.1, 0.5, 97)
    gp.h = torch.as_tensor(h, device="cuda")
    M, sp = racmb.block_matrices(gp, 4, 5, 1, 7, 0.37)
    for i, B in enumerate(O.blocks(5, 1, 7, 97, 4)):
        ref = Hd[np.ix_(B, B)] + np.diag(h[B]) + 0.37 * (np.eye(len(B)) + np.outer(A[0, B], A[0, B]))
        lo = np.tril_indices(len(B))
        assert rel(M[i, :len(B), :len(B)][lo], ref[lo]) < 1e-14


def test_dense_not_positive_definite_reported_like_oracle():
    n = 40
    rng = np.random.default_rng(2)
    Hd = np.eye(n)
    h = np.zeros(n)
    h[17] = -1e3
    c = rng.standard_normal(n)
    gp = racmb.dense_problem(Hd, c, h=h)
    op = O.Problem(F=np.zeros((0, n), order="F"), Ns=1.0, c=c, h=h, Hd=Hd)
    ref = O.solve(op, p=4, beta0=1.0, max_iter=3)
    s = racmb.Solver(gp, p=4, beta0=1.0, max_iter=3)
    r = s.run(allow_not_pd=True)
    assert s.last_code == racmb.RAC_ERR_NOT_PD
    assert (r.fail_iter, r.fail_block) == (ref.fail_iter, ref.fail_block)


def test_dense_rejected_where_unsupported():
    gp, *_ = random_qp(64, 2, 1)
    ps = gp.struct()
    ps.meq = racmb.MAX_EQ + 1
    import ctypes as C
    h = C.c_void_p()
    opts = racmb.Opts_(4, 0, 0, 0, 0, 1.0, 10.0, 2.0, None, None, 1.0, 10, 10, 0.0, 0, 0, 0, 0, 0, 0)
    assert racmb.load().rac_solver_create(C.byref(ps), C.byref(opts), C.byref(h)) == racmb.RAC_ERR_ARG
    with pytest.raises(racmb.RacError) as e:
        racmb.Batch([gp], [(0, racmb.PROX_NONE, 0.0, 1.0, 1.0)], s=16, max_iter=1)
    assert e.value.code == racmb.RAC_ERR_UNSUPPORTED


# ---------------------------------------------------------------------------
# Gaussian-kernel C-SVC (Sec.3.2)

def two_class(n, r, seed, shift=0.7):
    rng = np.random.default_rng(seed)
    y = rng.choice([-1.0, 1.0], size=n)
    X = shift * y[:, None] * np.ones((1, r)) / np.sqrt(r) + rng.standard_normal((n, r))
    return X, y


def test_gaussian_kernel_matrix_matches_oracle():
    X, y = two_class(333, 7, 1)
    Q, _, _ = racmb.svm_kernel_matrix(X, y, 0.4)
    ref = O.svm_kernel_problem(X, y, 1.0, 0.4).Hd
    Qh = Q.cpu().numpy().T        # (n, n) tensor rows = columns of the column-major matrix
    assert rel(Qh, ref) < 1e-14
    assert np.array_equal(Qh, Qh.T)


@pytest.mark.parametrize("variant", [racmb.VARIANT_RAC, racmb.VARIANT_RP])
def test_gaussian_svm_parity_bias_decision_and_accuracy(variant):
    X, y = two_class(600, 8, 3)
    Xt_, yt_ = two_class(400, 8, 4)
    gamma, Cbox = 0.5, 1.0
    gp, Xd, yd = racmb.svm_kernel_problem(X, y, Cbox, gamma)
    op = O.svm_kernel_problem(X, y, Cbox, gamma)
    beta0 = 0.1 * 10                   # beta = 0.1 p (Sec.3.2), p = 10 blocks of 60
    say("gaussian svm 600x8", variant)
    s, r, x, z, xi = run(gp, p=10, beta0=beta0, max_iter=80, check_every=10, seed=5, variant=variant)
    ref = O.solve(op, p=10, beta0=beta0, max_iter=80, check_every=10, seed=5, rp=variant == racmb.VARIANT_RP)
    assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8
    mu = float(s.multipliers()[0])
    assert abs(mu - ref.mu) <= 1e-8 * max(1.0, abs(ref.mu))
    bias = -mu
    assert abs(bias - O.svm_bias(ref)) <= 1e-8 * max(1.0, abs(bias))
    f, acc = racmb.svm_decision(Xd, yd, z, gamma, bias, Xt_, labels=yt_)
    fref = O.svm_decision(X, y, ref.z, O.svm_bias(ref), gamma, Xt_)
    assert rel(f, fref) < 1e-8
    assert acc == O.svm_accuracy(fref, yt_)
    assert acc > 0.6
