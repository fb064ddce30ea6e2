"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

lasso_20000x2000 (FP32 data, blocks of 64, the default row groups, Gram row
chunks, packed tiles and stream overlap):
  * FP64 mode, three iterations compared element by element with the oracle
    (which runs about one iteration per second at this size);
  * the timed configuration (mixed precision, learned penalty) run to
    KKT <= 1e-6; the oracle then recomputes the KKT residual and the objective
    of the GPU's iterate, which must agree with what the GPU reported, and the
    objective and z are compared with the oracle's own optimum of the same
    values (stored by tests/golden/make_golden.py): 1e-6 relative objective,
    1e-5 relative z.
Batched elastic-net paths, 256 instances x 16 lambda lanes (BF16 data, team
sweep, hipGraph, autotuned layout):
  * FP64 mode, ten iterations; sampled lanes (small instances, the median one,
    one that needs a team of 32, one with many blocks) compared element by
    element with the oracle;
  * the timed configuration run until every lane reaches KKT <= 1e-6; the
    oracle recomputes the KKT residual of sampled lanes and their objective is
    compared with the oracle's stored optimum (1e-6); the same solver continued
    from those states to KKT <= 1e-10 then matches the stored z to 1e-5 (at
    1e-6 an ill-conditioned lane, n > N with the smallest lambda, is 5e-5 away).
svm_20000x256 (FP32 data, blocks of 128, the equality row):
  * FP64 mode, ten iterations against the oracle;
  * mixed precision, 500 iterations: z in the box, the KKT residual falling,
    and the KKT residual and objective recomputed by the oracle.
lasso_10000x100000 (BF16 data, blocks of 128, 782 blocks): one oracle
iteration costs about a minute at this size, so the check is the property one:
mixed precision with the learned penalty run to KKT <= 1e-6, then the oracle's
KKT residual and objective of the GPU's iterate.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import racmb, workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden  # noqa: E402  (reader of the stored oracle solutions)

GOLDEN = os.path.dirname(os.path.abspath(make_golden.__file__))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

WEIGHTS = os.path.join(os.path.dirname(racmb.__file__), "controller_weights.npy")


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def mlp_weights():
    return torch.as_tensor(np.load(WEIGHTS).astype(np.float32), device="cuda")


@pytest.fixture(scope="module")
def lasso_full():
    w = W.lasso_20000x2000("f32")
    gp = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f32")
    op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
    return w, gp, op


def test_lasso_20000x2000_fp64_iterates_match_oracle(lasso_full):
    w, gp, op = lasso_full
    say("lasso 20000x2000, FP64 mode, 3 iterations")
    s = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_FP64, beta0=w.beta0, max_iter=3,
                     check_every=10, tol=0.0)
    info = s.info()
    timed = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_MIXED, beta0=w.beta0, max_iter=1,
                         check_every=10, tol=0.0)
    ti = timed.info()
    timed.close()
    say("launch", info, "timed configuration", ti)
    assert (info["p"], info["K"], info["R"], info["overlap"]) == (ti["p"], ti["K"], ti["R"], ti["overlap"])
    assert info["K"] > 1 and info["p"] == 32
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    s.close()
    ref = O.solve(op, s=w.block_size, beta0=w.beta0, max_iter=3, check_every=10)
    assert r.iters == 3 == ref.iters
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8, rel(a, b)


def test_lasso_20000x2000_timed_configuration_reaches_tolerance(lasso_full):
    w, gp, op = lasso_full
    say("lasso 20000x2000, mixed precision, learned penalty, to KKT <= 1e-6")
    s = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_MIXED, beta0=w.beta0,
                     beta_mode=racmb.BETA_MLP, mlp_weights=mlp_weights(), check_every=10, max_iter=5000,
                     tol=1e-6)
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    s.close()
    say("iterations", r.iters, "kkt", r.kkt, "objective", r.objective)
    assert r.status == racmb.RUN_CONVERGED and r.kkt <= 1e-6
    k = O.kkt(op, x, z, xi, mu)
    ob = O.objective(op, z)
    say("oracle kkt", k, "objective", ob)
    assert k <= 1e-6 and abs(k - r.kkt) <= 1e-6 * r.kkt
    assert abs(r.objective - ob) <= 1e-10 * (abs(ob) + op.obj_const)
    check_golden(os.path.join(GOLDEN, "lasso_20000x2000_solution.txt"), ob, z)


def golden_is_optimal(path, D, y, lam, alpha):
    """The stored optimum checked against the elastic-net optimality conditions of Eq.(6),
    recomputed with numpy from the same stored values: g = D'(Dz - y)/N + lam (1 - alpha) z
    equals -lam alpha sign(z_j) on the support and lies in [-lam alpha, lam alpha] off it
    (to 1e-8 of |D'y/N|_inf)."""
    head, z = make_golden.read(path)
    N = D.shape[0]
    g = D.T @ (D @ z - y) / N + lam * (1 - alpha) * z
    on = z != 0
    tol = 1e-8 * np.max(np.abs(D.T @ y)) / N
    assert np.max(np.abs(g[on] + lam * alpha * np.sign(z[on])), initial=0.0) <= tol
    assert np.max(np.abs(g[~on]), initial=0.0) <= lam * alpha + tol


def check_golden(path, objective, z, z_tol=1e-5):
    """The oracle's own optimum of the same stored values (FP64, run to KKT <= 1e-9 by
    tests/golden/make_golden.py): relative objective within 1e-6 and relative z error
    within z_tol (1e-5, the mixed-precision bar; None: objective only) (Eq.(5)-(8))."""
    head, zg = make_golden.read(path)
    og = float(head["objective"])
    ro = abs(objective - og) / abs(og)
    zn = float(np.linalg.norm(zg))
    err = float(np.linalg.norm(np.asarray(z) - zg))
    say(os.path.basename(path), "rel objective", ro, "z error", err, "|z*|", zn)
    assert ro <= 1e-6, ro
    if z_tol is None:
        return
    if zn == 0.0:                 # lambda = lambda_max: the optimum is z = 0 (to rounding)
        assert err <= 1e-12, err
    else:
        assert err <= z_tol * zn, err / zn


@pytest.fixture(scope="module")
def en_paths():
    Ns, ns = W.en_batch_sizes(256)
    insts = [W.en_instance_device(int(N), int(n), 1000 + i, storage="bf16") for i, (N, n) in enumerate(zip(Ns, ns))]
    probs = [racmb.regression_problem_tensor(d.F, d.y, lam=0.1 * d.lam_max, alpha=0.5, storage="bf16")
             for d in insts]
    lanes = [(i, racmb.PROX_EN, float(l), 0.5, 0.1 * float(l))
             for i, d in enumerate(insts) for l in W.lambda_grid(d.lam_max, 16, 0.01)]
    torch.cuda.synchronize()
    size = Ns.astype(np.float64) * ns
    order = np.argsort(size, kind="stable")
    big_rows = [i for i in range(len(Ns)) if Ns[i] > 16 * 640]
    wide = min(big_rows, key=lambda i: size[i])               # its group runs on a team of 32
    deep = max((i for i in range(len(Ns)) if size[i] <= 4e6), key=lambda i: ns[i])   # many blocks
    sample = sorted({int(order[0]), int(order[1]), int(order[len(order) // 2]), int(wide), int(deep)})
    return insts, probs, lanes, sample


def oracle_lane(d, lane, **kw):
    i, prox, lam, alpha, beta0 = lane
    op = O.en_problem(d.host_D(), d.y, lam=lam, alpha=alpha)
    return op, O.solve(op, inst=i, beta0=beta0, **kw)


def test_en_paths_256x16_fp64_sampled_lanes_match_oracle(en_paths):
    insts, probs, lanes, sample = en_paths
    say("en paths 256x16, FP64 mode, 10 iterations; sampled instances", sample,
        [(insts[i].N, insts[i].n) for i in sample])
    b = racmb.Batch(probs, lanes, s=64, seed=11, precision=racmb.PREC_FP64, beta_mode=racmb.BETA_FIXED,
                    check_every=10, max_iter=10, tol=0.0, use_graph=True, tune=True)
    it, act = b.run()
    info = b.info()
    say(info)
    assert it == 10 and act == len(lanes) and info["team_size"] > 0 and info["graph"] == 1
    for i in sample:
        for j in (4, 9, 15):                                   # z is not identically zero on these lanes
            u = 16 * i + j
            res, x, z, xi = b.lane(u)
            op, ref = oracle_lane(insts[i], lanes[u], s=64, seed=11, max_iter=10, check_every=10)
            say("lane", u, "instance", i, "rel z", rel(z, ref.z))
            assert res.iters == 10
            for a, c in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
                assert rel(a, c) < 1e-8, (u, rel(a, c))
    b.close()


def test_en_paths_256x16_timed_configuration_reaches_tolerance(en_paths):
    insts, probs, lanes, sample = en_paths
    say("en paths 256x16, mixed precision, learned penalty, every lane to KKT <= 1e-6")
    b = racmb.Batch(probs, lanes, s=64, seed=11, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_MLP,
                    mlp_weights=mlp_weights(), check_every=10, max_iter=1500, tol=1e-6, use_graph=True,
                    tune=True)
    it, act = b.run()
    say("iterations", it, "active", act, b.info())
    assert act == 0
    picked, starts = [], []
    for i in sample:
        for j in (0, 7, 15):
            u = 16 * i + j
            res, x, z, xi = b.lane(u)
            op = O.en_problem(insts[i].host_D(), insts[i].y, lam=lanes[u][2], alpha=0.5)
            k = O.kkt(op, x, z, xi)
            say("lane", u, "iterations", res.iters, "kkt", res.kkt, "oracle kkt", k)
            assert res.status == racmb.RUN_CONVERGED
            assert k <= 1e-6 and abs(k - res.kkt) <= 1e-6 * max(res.kkt, 1e-300) + 1e-15
            path = os.path.join(GOLDEN, "en_paths_256x16_lane%d_solution.txt" % u)
            golden_is_optimal(path, insts[i].host_D(), insts[i].y, lanes[u][2], 0.5)
            check_golden(path, O.objective(op, z), z, z_tol=None)   # objective at the timed tolerance
            picked.append((i, u))
            starts.append((x, z, xi, res.beta))
    b.close()
    # A KKT residual of 1e-6 bounds z only through the problem's conditioning (the lane of the
    # instance with n > N and the smallest lambda is 5e-5 away).  The same candidate solver,
    # continued from these states to KKT <= 1e-10, reaches the FP64 optimum to 1e-5 in z.
    say("sampled lanes continued in mixed precision to KKT <= 1e-10")
    sub = sorted({i for i, _ in picked})
    c = racmb.Batch([probs[i] for i in sub], [(sub.index(i),) + tuple(lanes[u][1:]) for i, u in picked], s=64,
                    seed=11, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_MLP, mlp_weights=mlp_weights(),
                    check_every=10, max_iter=20000, tol=1e-10, use_graph=True)
    for v, (x, z, xi, beta) in enumerate(starts):
        c.set_lane_state(v, x, z, xi, 0.0, beta)
    it, act = c.run()
    say("iterations", it, "active", act)
    assert act == 0
    for v, (i, u) in enumerate(picked):
        res, x, z, xi = c.lane(v)
        op = O.en_problem(insts[i].host_D(), insts[i].y, lam=lanes[u][2], alpha=0.5)
        check_golden(os.path.join(GOLDEN, "en_paths_256x16_lane%d_solution.txt" % u), O.objective(op, z), z)
    c.close()


@pytest.fixture(scope="module")
def svm_full():
    w = W.svm_20000x256()
    gp = racmb.svm_problem(w.X, w.labels, w.C, storage=w.storage)
    op = O.svm_problem(w.X.astype(np.float64), w.labels, w.C)
    return w, gp, op


def test_svm_20000x256_fp64_iterates_match_oracle(svm_full):
    w, gp, op = svm_full
    say("svm 20000x256, FP64 mode, 10 iterations")
    s = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_FP64, beta0=w.beta0, max_iter=10,
                     check_every=10, tol=0.0)
    say(s.info())
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    s.close()
    ref = O.solve(op, s=w.block_size, beta0=w.beta0, max_iter=10, check_every=10)
    for a, b in ((x, ref.x), (z, ref.z), (xi, ref.xi)):
        assert rel(a, b) < 1e-8, rel(a, b)
    assert abs(mu - ref.mu) <= 1e-8 * max(1.0, abs(ref.mu))


def test_svm_20000x256_mixed_iterate_checked_by_oracle(svm_full):
    """The linear-kernel dual at this size converges slowly (its Q has rank 256
    for 20000 variables): the check is on a fixed number of iterations."""
    w, gp, op = svm_full
    say("svm 20000x256, mixed precision, residual balancing, 500 iterations")
    s = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_MIXED, beta0=w.beta0,
                     beta_mode=racmb.BETA_RESBAL, check_every=10, max_iter=500, tol=0.0)
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    kk = s.history()[:, 3]
    s.close()
    say("iterations", r.iters, "kkt", r.kkt, "objective", r.objective, "first check", kk[9])
    assert r.iters == 500 and np.all((z >= 0.0) & (z <= w.C))
    assert r.kkt < 0.5 * kk[9]
    k = O.kkt(op, x, z, xi, mu)
    ob = O.objective(op, z)
    say("oracle kkt", k, "objective", ob)
    assert abs(k - r.kkt) <= 1e-6 * r.kkt
    assert abs(r.objective - ob) <= 1e-10 * max(1.0, abs(ob))


def test_lasso_10000x100000_mixed_reaches_tolerance():
    w = W.lasso_10000x100000("bf16")
    say("lasso 10000x100000 generated; mixed precision, learned penalty, to KKT <= 1e-6")
    gp = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="bf16")
    s = racmb.Solver(gp, s=w.block_size, precision=racmb.PREC_MIXED, beta0=w.beta0,
                     beta_mode=racmb.BETA_MLP, mlp_weights=mlp_weights(), check_every=10, max_iter=5000,
                     tol=1e-6)
    say(s.info())
    r = s.run()
    x, z, xi, mu, beta, it = s.state()
    s.close()
    del gp
    say("iterations", r.iters, "kkt", r.kkt, "objective", r.objective)
    assert r.status == racmb.RUN_CONVERGED and r.kkt <= 1e-6
    op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
    k = O.kkt(op, x, z, xi, mu)
    ob = O.objective(op, z)
    say("oracle kkt", k, "objective", ob)
    assert k <= 1e-6 and abs(k - r.kkt) <= 1e-6 * r.kkt
    assert abs(r.objective - ob) <= 1e-10 * (abs(ob) + op.obj_const)
