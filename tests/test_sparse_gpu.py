"""The sparse factor form on the GPU (data in compressed sparse columns, the
high-sparsity regressions of Sec.3.1) against the FP64 oracle given the same
data densified.

Bars: iterates within 1e-8 relative of the oracle's (RAC and RP, FP64 and FP32
stored values, with and without an equality row), the KKT residual, objective
and block matrices equal to the definitions to rounding.  The residual update
uses atomic additions, so runs agree to rounding rather than bitwise."""
import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import racmb, workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def pair(w, lam=None, alpha=None):
    lam = w.lam if lam is None else lam
    alpha = w.alpha if alpha is None else alpha
    gp = racmb.sparse_regression_problem(w.colptr, w.rowidx, w.values, w.y, w.N, lam=lam, alpha=alpha,
                                         storage=w.storage)
    op = O.en_problem(w.dense(), w.y, lam=lam, alpha=alpha)
    return gp, op


@pytest.mark.parametrize("variant", [racmb.VARIANT_RAC, racmb.VARIANT_RP])
@pytest.mark.parametrize("N,n,density,s,storage", [
    (1500, 601, 0.02, 64, "f64"), (800, 257, 0.05, 32, "f32"), (3000, 130, 0.01, 128, "f64"),
    (500, 90, 0.1, 16, "f64"),
    (3000, 260, 0.05, 128, "f64"),      # blocks of 19200 entries: u in LDS, chunks of 10240
    (20000, 200, 0.002, 64, "f32"),     # more rows than LDS holds: u in device memory
    (20000, 300, 0.005, 128, "f64")])   # ... with blocks of 12800 entries in chunks
def test_sparse_en_parity(variant, N, n, density, s, storage):
    w = W.sparse_regression(N, n, density, data_seed=N + n, storage=storage)
    gp, op = pair(w)
    say("sparse en", N, n, density, s, storage, variant)
    kw = dict(s=s, beta0=0.1 * w.lam, beta_mode=racmb.BETA_RESBAL, max_iter=50, check_every=10, seed=4)
    sol = racmb.Solver(gp, variant=variant, **kw)
    r = sol.run()
    x, z, xi, mu, beta, it = sol.state()
    ref = O.solve(op, s=s, beta0=0.1 * w.lam, beta_mode=O.BETA_RESBAL, max_iter=50, check_every=10, seed=4,
                  rp=variant == racmb.VARIANT_RP)
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8, rel(a, b)
    h = sol.history()
    np.testing.assert_allclose(h[:, 0], ref.r_p, rtol=1e-6, atol=1e-14)
    np.testing.assert_array_equal(h[:, 2], ref.betas)
    ob = O.objective(op, ref.z)
    assert abs(r.objective - ob) <= 1e-8 * (abs(ob) + op.obj_const)


def test_sparse_en_converges_to_oracle_solution():
    w = W.sparse_regression(2000, 400, 0.03, data_seed=5)
    gp, op = pair(w)
    r, x, z, xi, mu = racmb.solve(gp, s=32, beta0=0.1 * w.lam, beta_mode=racmb.BETA_RESBAL, max_iter=3000,
                                  check_every=10, tol=1e-10)
    ref = O.solve(op, s=32, beta0=0.1 * w.lam, beta_mode=O.BETA_RESBAL, max_iter=4000, check_every=10, tol=1e-11)
    assert r.status == racmb.RUN_CONVERGED and ref.status == O.RUN_CONVERGED
    assert rel(z, ref.z) < 1e-7
    assert O.kkt(op, x, z, xi) < 1e-9


def test_sparse_svm_with_equality_row_parity():
    rng = np.random.default_rng(3)
    n, r = 700, 300
    X = np.where(rng.random((n, r)) < 0.03, rng.standard_normal((n, r)), 0.0)
    yl = rng.choice([-1.0, 1.0], size=n)
    X[:, 0] = 0.5 * yl          # one informative feature
    G = X * yl[:, None]         # n x r; F = G' (r x n), column j = sample j
    colptr = [0]
    rowidx, vals = [], []
    for j in range(n):
        nz = np.nonzero(G[j])[0]
        rowidx.extend(nz.tolist())
        vals.extend(G[j, nz].tolist())
        colptr.append(len(rowidx))
    cp = torch.as_tensor(np.array(colptr, dtype=np.int64), device="cuda")
    ri = torch.as_tensor(np.array(rowidx, dtype=np.int32), device="cuda")
    vv = torch.as_tensor(np.array(vals, dtype=np.float64), device="cuda")
    gp = racmb.Problem(F=vv, storage="f64", rows=r, n=n, Ns=1.0, c=torch.full((n,), -1.0, dtype=torch.float64,
                       device="cuda"), a=torch.as_tensor(yl, device="cuda"), b=0.0, prox=racmb.PROX_BOX, lo=0.0,
                       hi=1.0, colptr=cp, rowidx=ri)
    op = O.svm_problem(X, yl, 1.0)
    say("sparse svm 700 x 300")
    sol = racmb.Solver(gp, s=64, beta0=1.1, max_iter=60, check_every=10, seed=2)
    sol.run()
    x, z, xi, mu, beta, it = sol.state()
    ref = O.solve(op, s=64, beta0=1.1, max_iter=60, check_every=10, seed=2)
    assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8
    assert abs(mu - ref.mu) <= 1e-8 * max(1.0, abs(ref.mu))


def test_sparse_kkt_objective_and_block_matrices():
    w = W.sparse_regression(900, 210, 0.04, data_seed=11)
    gp, op = pair(w)
    rng = np.random.default_rng(1)
    for _ in range(2):
        x, z, xi = rng.standard_normal(210), rng.standard_normal(210), rng.standard_normal(210)
        z[::3] = 0.0
        got = racmb.kkt(gp, x, z, xi, 0.0)
        k, parts = O.kkt(op, x, z, xi, 0.0, parts=True)
        assert abs(got[0] - k) <= 1e-12 * k
        np.testing.assert_allclose(got[1:], parts, rtol=1e-12)
        ob = O.objective(op, z)
        assert abs(racmb.objective(gp, z) - ob) <= 1e-12 * (abs(ob) + op.obj_const)
    D = w.dense()
    M, sp = racmb.block_matrices(gp, 7, 5, 1, 3, 0.3)
    for i, B in enumerate(O.blocks(5, 1, 3, 210, 7)):
        ref = D[:, B].T @ D[:, B] / w.N + 0.3 * np.eye(len(B))
        lo = np.tril_indices(len(B))
        assert rel(M[i, :len(B), :len(B)][lo], ref[lo]) < 1e-13


def test_sparse_not_positive_definite_reported_like_oracle():
    w = W.sparse_regression(200, 24, 0.1, data_seed=2)
    h = np.zeros(24)
    h[13] = -1e3
    gp = racmb.sparse_regression_problem(w.colptr, w.rowidx, w.values, w.y, w.N, h=h)
    op = O.en_problem(w.dense(), w.y, h=h)
    ref = O.solve(op, p=4, beta0=1.0, max_iter=3)
    s = racmb.Solver(gp, p=4, beta0=1.0, max_iter=3)
    r = s.run(allow_not_pd=True)
    assert s.last_code == racmb.RAC_ERR_NOT_PD
    assert (r.fail_iter, r.fail_block) == (ref.fail_iter, ref.fail_block)
