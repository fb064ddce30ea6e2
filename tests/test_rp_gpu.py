"""RP-MBADMM on the GPU (fixed contiguous blocks, a random solve order every
iteration; Sec.1) against the FP64 oracle run with ``rp=True``.

Bars as for the RAC path: FP64-mode iterates within 1e-8 relative of the
oracle's, the penalty history equal, mixed precision within 1e-5 of the FP64
fixed point, failures of Assumption 2.1 reported at the oracle's (iteration,
position).  The solver forms the block Grams once and refactors only when the
penalty changes, which the phase counters show.
"""
import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import racmb, workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

RP = racmb.VARIANT_RP


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def en_pair(w, lam=None, alpha=None, h=None):
    lam = w.lam if lam is None else lam
    alpha = w.alpha if alpha is None else alpha
    gp = racmb.regression_problem(w.D, w.y, lam=lam, alpha=alpha, storage=w.storage, h=h)
    op = O.en_problem(w.D.astype(np.float64), w.y, lam=lam, alpha=alpha, h=h)
    return gp, op


def run(gp, **kw):
    s = racmb.Solver(gp, variant=RP, **kw)
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    return s, r, x, z, xi, mu


def test_rp_order_is_the_permutation_of_the_block_indices():
    # the order of iteration k is rac_permutation(seed, instance, k, p), bit-exact
    for p in (1, 7, 32, 782):
        g = racmb.permutation(5, 2, 9, p).cpu().numpy()
        assert np.array_equal(g, O.permutation(5, 2, 9, p))


def test_rp_least_squares_parity():
    w = W.ols_2000x200()
    gp, op = en_pair(w)
    say("rp ols 2000x200, 200 iterations")
    s, r, x, z, xi, mu = run(gp, s=20, beta0=1.0, max_iter=200, check_every=10, seed=3)
    ref = O.solve(op, s=20, beta0=1.0, max_iter=200, check_every=10, seed=3, rp=True)
    assert rel(z, ref.z) < 1e-8 and rel(x, ref.x) < 1e-8 and rel(xi, ref.xi) < 1e-8
    np.testing.assert_allclose(s.history()[:, 0], ref.r_p, rtol=1e-6, atol=1e-14)
    xs = np.linalg.lstsq(w.D, w.y, rcond=None)[0]
    assert rel(z, xs) < 1e-9


def test_rp_differs_from_rac():
    # same problem and seed, other variant: a different iterate before convergence
    w = W.lasso(N=1500, n=200, data_seed=31, block_size=32, storage="f64")
    gp, _ = en_pair(w)
    outs = []
    for variant in (racmb.VARIANT_RAC, RP):
        s = racmb.Solver(gp, s=32, beta0=w.beta0, max_iter=5, check_every=5, seed=1, variant=variant)
        s.run()
        outs.append(s.state()[1])
        s.close()
    assert rel(outs[0], outs[1]) > 1e-6


@pytest.mark.parametrize("storage,n,s", [("f32", 301, 32), ("f64", 300, 30), ("bf16", 257, 64),
                                          ("bf16", 700, 128), ("f64", 400, 100)])
def test_rp_lasso_fixed_beta_parity_ragged(storage, n, s):
    """Blocks of 100 to 128 columns (ragged: 116 and 117 at n = 700) take the sweep's
    128-column tiles, whose block inverse is staged in LDS in the drawn order."""
    w = W.lasso(N=2500, n=n, data_seed=12, block_size=s, storage=storage)
    gp, op = en_pair(w)
    b0 = 1.0 / w.N
    say("rp lasso", storage, n, s)
    sol, r, x, z, xi, mu = run(gp, s=s, beta0=b0, max_iter=60, check_every=10, seed=4)
    ref = O.solve(op, s=s, beta0=b0, max_iter=60, check_every=10, seed=4, rp=True)
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8
    np.testing.assert_allclose(sol.history()[:, 3], ref.hist[:60, 3], rtol=1e-6, atol=1e-12)


def test_rp_residual_balancing_refactors_on_beta_changes():
    w = W.lasso(N=3000, n=300, data_seed=13, block_size=32, storage="f32")
    gp, op = en_pair(w)
    say("rp lasso residual balancing")
    s = racmb.Solver(gp, s=32, beta0=w.beta0, beta_mode=racmb.BETA_RESBAL, max_iter=400, check_every=10,
                     tol=1e-8, seed=2, variant=RP)
    s.set_timing(True)
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    ref = O.solve(op, s=32, beta0=w.beta0, beta_mode=O.BETA_RESBAL, max_iter=400, check_every=10,
                  tol=1e-8, seed=2, rp=True)
    assert r.iters == ref.iters and r.status == racmb.RUN_CONVERGED
    betas = s.history()[:, 2]
    np.testing.assert_array_equal(betas, ref.betas)
    assert rel(z, ref.z) < 1e-8
    tm = s.timing()
    changes = 1 + int(np.sum(betas[1:] != betas[:-1]))
    assert tm["gram"][1] == 1                     # the fixed blocks' Grams, once
    assert tm["factor"][1] == changes             # one factorisation per penalty value
    assert tm["sweep"][1] == r.iters


def test_rp_svm_dual_parity():
    w = W.svm(n=1500, r=24, block_size=64, data_seed=7)
    gp = racmb.svm_problem(w.X, w.labels, w.C, storage=w.storage)
    op = O.svm_problem(w.X.astype(np.float64), w.labels, w.C)
    say("rp svm 1500x24")
    s, r, x, z, xi, mu = run(gp, s=64, beta0=w.beta0, max_iter=80, check_every=10, seed=1)
    ref = O.solve(op, s=64, beta0=w.beta0, max_iter=80, check_every=10, seed=1, rp=True)
    assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8
    assert abs(mu - ref.mu) <= 1e-8 * max(1.0, abs(ref.mu))


def test_rp_beta_schedule_parity():
    w = W.lasso(N=800, n=120, data_seed=5, block_size=16, storage="f64")
    gp, op = en_pair(w)
    sched = (1.0 / w.N) * 1.3 ** np.sin(np.arange(30))
    say("rp schedule")
    s, r, x, z, xi, mu = run(gp, s=16, beta0=1.0, beta_mode=racmb.BETA_SCHEDULE, beta_schedule=sched,
                             max_iter=30, check_every=10)
    ref = O.solve(op, s=16, beta0=1.0, beta_mode=O.BETA_SCHEDULE, beta_sched=sched, max_iter=30,
                  check_every=10, rp=True)
    np.testing.assert_array_equal(s.history()[:, 2], sched)
    assert rel(z, ref.z) < 1e-8


@pytest.mark.parametrize("p,K", [(1, 1), (1, 3), (5, 2), (37, 4)])
def test_rp_edge_partitions(p, K):
    rng = np.random.default_rng(p * 10 + K)
    N, n = 131, 37
    D = np.asfortranarray(rng.standard_normal((N, n)))
    y = rng.standard_normal(N)
    gp = racmb.regression_problem(D, y, lam=0.05, alpha=0.6, storage="f64")
    op = O.en_problem(D, y, lam=0.05, alpha=0.6)
    say("rp edge", p, K)
    s, r, x, z, xi, mu = run(gp, p=p, beta0=0.8, max_iter=25, check_every=7, seed=11, sweep_groups=K)
    ref = O.solve(op, p=p, beta0=0.8, max_iter=25, check_every=7, seed=11, rp=True)
    assert rel(z, ref.z) < 1e-9 and rel(xi, ref.xi) < 1e-9


def test_rp_streaming_sweep_matches_oracle():
    w = W.lasso(N=3000, n=300, data_seed=15, block_size=32, storage="f64")
    gp, op = en_pair(w)
    say("rp streaming sweep 3000x300, K = 2")
    s, r, x, z, xi, mu = run(gp, s=32, beta0=w.beta0, max_iter=30, check_every=10, seed=5, sweep_groups=2)
    assert s.info()["tileA"] == 0
    ref = O.solve(op, s=32, beta0=w.beta0, max_iter=30, check_every=10, seed=5, rp=True)
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_rp_mixed_precision_reaches_fp64_solution(storage):
    w = W.lasso(N=4000, n=400, data_seed=21, block_size=64, storage=storage)
    gp, op = en_pair(w)
    say("rp mixed", storage)
    s, r, x, z, xi, mu = run(gp, s=64, beta0=w.beta0, beta_mode=racmb.BETA_RESBAL, precision=racmb.PREC_MIXED,
                             max_iter=3000, check_every=10, tol=1e-9)
    ref = O.solve(op, s=64, beta0=w.beta0, beta_mode=O.BETA_RESBAL, max_iter=4000, check_every=10,
                  tol=1e-11, rp=True)
    assert r.status == racmb.RUN_CONVERGED and ref.status == O.RUN_CONVERGED
    assert rel(z, ref.z) < 1e-5
    obj = O.objective(op, ref.z)
    assert abs(r.objective - obj) < 1e-6 * abs(obj)


def test_rp_not_positive_definite_reported_like_oracle():
    w = W.least_squares(N=60, n=12, data_seed=1)
    h = np.zeros(12)
    h[5] = -1e3                      # variable 5: fixed block 1 of p = 3
    gp = racmb.regression_problem(w.D, w.y, h=h)
    op = O.en_problem(w.D, w.y, h=h)
    for it0 in (0, 3):
        ref = O.solve(op, p=3, beta0=1.0, max_iter=4, seed=it0, rp=True)
        s = racmb.Solver(gp, p=3, beta0=1.0, max_iter=4, seed=it0, variant=RP)
        r = s.run(allow_not_pd=True)
        assert s.last_code == racmb.RAC_ERR_NOT_PD
        assert ref.rc == O.ERR_NOT_PD
        assert (r.fail_iter, r.fail_block) == (ref.fail_iter, ref.fail_block)
        s.close()


def test_rp_checkpoint_resume_is_bit_exact():
    w = W.svm(n=900, r=16, block_size=64, data_seed=9)
    gp = racmb.svm_problem(w.X, w.labels, w.C, storage=w.storage)
    kw = dict(s=64, beta0=w.beta0, beta_mode=racmb.BETA_RESBAL, check_every=5, seed=6, variant=RP)
    a = racmb.Solver(gp, max_iter=40, **kw)
    a.run()
    xa = a.state()
    b = racmb.Solver(gp, max_iter=20, **kw)
    b.run()
    blob = b.export_state()
    c = racmb.Solver(gp, max_iter=20, **kw)
    c.import_state(blob)
    c.run()
    b.run()
    for st in (b.state(), c.state()):
        for u, v in zip(st[:3], xa[:3]):
            assert np.array_equal(u, v)
        assert st[3] == xa[3] and st[4] == xa[4] and st[5] == 40
