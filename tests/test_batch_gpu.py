"""Batched engine (rac_batch_*) against the FP64 oracle, lane by lane.

Each lane is an independent solve on its instance's data; lanes of instance i
share its partitions, drawn with the batch seed and instance id i, so the
oracle reproduces a lane with solve(seed=batch seed, inst=i)."""
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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def en_batch(storage="f64", ninst=5, lanes_per=3, seed=0, s=32):
    rng = np.random.default_rng(seed)
    ws, gps, ops, lanes = [], [], [], []
    for i in range(ninst):
        N = int(rng.integers(150, 1200))
        n = int(rng.integers(20, 330))
        w = W.gaussian_en(N, n, 0.1, 0.05, 0.1, 0.5, 100 + i + seed, s, storage)
        ws.append(w)
        gps.append(racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage=storage))
        ops.append(O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=0.5))
        for j in range(lanes_per):
            lam = w.lam * 3.0 ** (1 - j)
            lanes.append((i, racmb.PROX_EN, lam, 0.5, float(10 ** rng.uniform(-1.5, 0.5))))
    return ws, gps, ops, lanes


def oracle_lane(op, lane, **kw):
    i, prox, lam, alpha, beta0 = lane
    P = O.Problem(F=op.F, Ns=op.Ns, c=op.c, h=op.h, a=op.a, b=op.b, prox=prox, lam=lam, alpha=alpha,
                  lo=op.lo, hi=op.hi, obj_const=op.obj_const)
    return O.solve(P, inst=i, beta0=beta0, **kw)


def test_batch_lanes_match_oracle_fp64():
    ws, gps, ops, lanes = en_batch()
    say("batch fp64", len(lanes), "lanes")
    b = racmb.Batch(gps, lanes, s=32, seed=7, max_iter=30, check_every=10, use_graph=True)
    it, act = b.run()
    assert it == 30 and act == len(lanes)
    assert b.info()["graph"] == 1
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=7, max_iter=30, check_every=10)
        assert res.iters == 30
        assert rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8 and rel(x, ref.x) < 1e-8, u


def test_batch_graph_and_tuning_do_not_change_results():
    ws, gps, ops, lanes = en_batch("f32", ninst=4, lanes_per=2, seed=3)
    outs = []
    for graph, tune in ((True, True), (False, False)):
        b = racmb.Batch(gps, lanes, s=32, seed=1, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_RESBAL,
                        max_iter=40, check_every=10, use_graph=graph, tune=tune)
        b.run()
        say("graph", graph, "tune", tune, b.info())
        outs.append([b.lane(u)[1:] for u in range(len(lanes))])
    for la, lb in zip(*outs):
        for u, v in zip(la, lb):
            assert np.array_equal(u, v)


def test_batch_lanes_retire_like_the_oracle():
    ws, gps, ops, lanes = en_batch(ninst=4, lanes_per=3, seed=5)
    b = racmb.Batch(gps, lanes, s=32, seed=2, beta_mode=racmb.BETA_RESBAL, max_iter=600, check_every=10,
                    tol=1e-7)
    it, act = b.run()
    assert act == 0
    iters = []
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=2, beta_mode=O.BETA_RESBAL, max_iter=600,
                          check_every=10, tol=1e-7)
        assert res.status == racmb.RUN_CONVERGED and ref.status == O.RUN_CONVERGED
        assert res.iters == ref.iters, (u, res.iters, ref.iters)
        assert rel(z, ref.z) < 1e-8
        iters.append(res.iters)
    assert len(set(iters)) > 1        # lanes really retired at different iterations


def test_batch_svm_lanes():
    wv = [W.svm(n=int(n), r=12, block_size=32, data_seed=40 + k) for k, n in enumerate((300, 517))]
    gps = [racmb.svm_problem(w.X, w.labels, w.C) for w in wv]
    ops = [O.svm_problem(w.X.astype(np.float64), w.labels, w.C) for w in wv]
    lanes = [(0, racmb.PROX_BOX, 0.0, 1.0, 0.5), (0, racmb.PROX_BOX, 0.0, 1.0, 3.0),
             (1, racmb.PROX_BOX, 0.0, 1.0, 1.7)]
    b = racmb.Batch(gps, lanes, s=32, seed=4, max_iter=50, check_every=10, use_graph=False)
    b.run()
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=4, max_iter=50, check_every=10)
        assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8


@pytest.mark.parametrize("storage", ["bf16", "f32"])
def test_batch_mixed_precision_reaches_fp64_solution(storage):
    ws, gps, ops, lanes = en_batch(storage, ninst=3, lanes_per=2, seed=9)
    b = racmb.Batch(gps, lanes, s=32, seed=5, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_RESBAL,
                    max_iter=3000, check_every=10, tol=1e-9)
    it, act = b.run()
    assert act == 0
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=5, beta_mode=O.BETA_RESBAL, max_iter=4000,
                          check_every=10, tol=1e-11)
        assert rel(z, ref.z) < 1e-5, u


def test_batch_reports_assumption_failure_per_lane():
    ws, gps, ops, lanes = en_batch(ninst=2, lanes_per=2, seed=11)
    h = np.zeros(ws[1].n)
    h[3] = -1e4
    gps[1] = racmb.regression_problem(ws[1].D, ws[1].y, lam=ws[1].lam, alpha=0.5, h=h)
    opbad = O.en_problem(ws[1].D, ws[1].y, lam=ws[1].lam, alpha=0.5, h=h)
    b = racmb.Batch(gps, lanes, s=32, seed=3, max_iter=20, check_every=10)
    it, act = b.run()
    assert act == 2
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u, allow_not_pd=True)
        if lane[0] == 1:
            ref = oracle_lane(opbad, lane, s=32, seed=3, max_iter=20, check_every=10)
            assert ref.rc == O.ERR_NOT_PD
            assert (res.fail_iter, res.fail_block) == (ref.fail_iter, ref.fail_block)
        else:
            ref = oracle_lane(ops[0], lane, s=32, seed=3, max_iter=20, check_every=10)
            assert res.fail_iter == -1 and rel(z, ref.z) < 1e-8
