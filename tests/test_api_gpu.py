"""One-call entry points and batch checkpoints through the C ABI.

rac_solve and rac_solve_batch are checked against the FP64 oracle (1e-8 in FP64
mode) and against the handle API they are built on (bit for bit); a batch that
imports another batch's exported state continues bit for bit as the exporter
does (the state of Eq.(3): x, z, xi, the lanes' multipliers and penalties)."""
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


def en_batch(storage="f64", ninst=4, lanes_per=3, seed=0, s=32):
    rng = np.random.default_rng(seed)
    gps, ops, lanes = [], [], []
    for i in range(ninst):
        N = int(rng.integers(150, 900))
        n = int(rng.integers(20, 260))
        w = W.gaussian_en(N, n, 0.1, 0.05, 0.1, 0.5, 300 + i + seed, s, storage)
        gps.append(racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage=storage))
        ops.append(O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=0.5))
        for j in range(lanes_per):
            lanes.append((i, racmb.PROX_EN, w.lam * 3.0 ** (1 - j), 0.5, float(10 ** rng.uniform(-1.5, 0.5))))
    return gps, ops, lanes


def test_rac_solve_matches_oracle_and_handle_api():
    w = W.svm(n=1200, r=20, block_size=64, data_seed=17)
    gp = racmb.svm_problem(w.X, w.labels, w.C, storage="f64")
    op = O.svm_problem(w.X, w.labels, w.C)
    say("rac_solve svm 1200x20")
    for variant in (racmb.VARIANT_RAC, racmb.VARIANT_RP):
        kw = dict(s=64, beta0=w.beta0, beta_mode=racmb.BETA_RESBAL, max_iter=60, check_every=10, seed=2)
        res, x, z, xi, mu = racmb.solve(gp, variant=variant, **kw)
        ref = O.solve(op, s=64, beta0=w.beta0, beta_mode=O.BETA_RESBAL, max_iter=60, check_every=10, seed=2,
                      rp=variant == racmb.VARIANT_RP)
        assert res.iters == 60
        assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8
        assert abs(mu - ref.mu) <= 1e-8 * max(1.0, abs(ref.mu))
        h = racmb.Solver(gp, variant=variant, **kw)
        rh = h.run()
        st = h.state()
        h.close()
        assert np.array_equal(st[0], x) and np.array_equal(st[1], z) and np.array_equal(st[2], xi)
        assert st[3] == mu and rh.kkt == res.kkt and rh.objective == res.objective


def test_rac_solve_reports_assumption_failure():
    wl = W.least_squares(N=60, n=12, data_seed=1)
    h = np.zeros(12)
    h[5] = -1e3
    gp = racmb.regression_problem(wl.D, wl.y, h=h)
    ref = O.solve(O.en_problem(wl.D, wl.y, h=h), p=3, beta0=1.0, max_iter=4)
    res, x, z, xi, mu = racmb.solve(gp, p=3, beta0=1.0, max_iter=4, allow_not_pd=True)
    assert (res.fail_iter, res.fail_block) == (ref.fail_iter, ref.fail_block)
    with pytest.raises(racmb.RacError) as e:
        racmb.solve(gp, p=3, beta0=1.0, max_iter=4)
    assert e.value.code == racmb.RAC_ERR_NOT_PD


def test_rac_solve_batch_matches_oracle_and_batch_handle():
    gps, ops, lanes = en_batch()
    say("rac_solve_batch", len(lanes), "lanes")
    kw = dict(s=32, seed=7, max_iter=40, check_every=10, tol=1e-7, beta_mode=racmb.BETA_RESBAL)
    out = racmb.solve_batch(gps, lanes, **kw)
    b = racmb.Batch(gps, lanes, **kw)
    b.run()
    for u, lane in enumerate(lanes):
        res, x, z, xi = out[u]
        i, prox, lam, alpha, beta0 = lane
        op = ops[i]
        P = O.Problem(F=op.F, Ns=op.Ns, c=op.c, prox=prox, lam=lam, alpha=alpha, obj_const=op.obj_const)
        ref = O.solve(P, inst=i, s=32, seed=7, beta0=beta0, beta_mode=O.BETA_RESBAL, max_iter=40,
                      check_every=10, tol=1e-7)
        assert res.iters == ref.iters and res.status == ref.status
        assert rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8 and rel(x, ref.x) < 1e-8, u
        rb, xb, zb, xib = b.lane(u)
        assert np.array_equal(xb, x) and np.array_equal(zb, z) and np.array_equal(xib, xi)
        assert rb.iters == res.iters and rb.kkt == res.kkt
    b.close()


@pytest.mark.parametrize("storage,prec,sweep", [("f64", racmb.PREC_FP64, racmb.BSWEEP_TEAM),
                                                ("bf16", racmb.PREC_MIXED, racmb.BSWEEP_TEAM),
                                                ("f32", racmb.PREC_MIXED, racmb.BSWEEP_LANE)])
def test_batch_checkpoint_resume_is_bit_exact(storage, prec, sweep):
    gps, ops, lanes = en_batch(storage, ninst=3, lanes_per=4, seed=5)
    say("batch checkpoint", storage, prec, sweep)
    kw = dict(s=32, seed=3, precision=prec, beta_mode=racmb.BETA_RESBAL, check_every=10, tol=1e-9, sweep=sweep)
    a = racmb.Batch(gps, lanes, max_iter=60, **kw)
    a.run()
    full = [a.lane(u) for u in range(len(lanes))]
    a.close()
    b = racmb.Batch(gps, lanes, max_iter=30, **kw)
    b.run()
    blob = b.export_state()
    c = racmb.Batch(gps, lanes, max_iter=30, **kw)
    c.import_state(blob)
    c.run()
    b.run()
    for other in (b, c):
        for u in range(len(lanes)):
            r, x, z, xi = other.lane(u)
            rf, xf, zf, xif = full[u]
            assert np.array_equal(x, xf) and np.array_equal(z, zf) and np.array_equal(xi, xif), u
            assert r.iters == rf.iters and r.beta == rf.beta and r.kkt == rf.kkt
    # a buffer from a batch of another shape is refused
    d = racmb.Batch(gps[:2], [l for l in lanes if l[0] < 2], max_iter=10, **kw)
    with pytest.raises(racmb.RacError) as e:
        d.import_state(blob)
    assert e.value.code == racmb.RAC_ERR_ARG
    for h in (b, c, d):
        h.close()


def test_warm_started_lambda_path_matches_oracle_path():
    """A decreasing lambda path (Sec.3.1) run stage by stage with each lane started from
    the previous stage's solution: every stage equals the oracle started from the same
    state (FP64, fixed iteration count), and the converged path equals cold solves."""
    from paper_1907_01995_amd import workloads as W
    rng = np.random.default_rng(4)
    ws = [W.gaussian_en(int(rng.integers(200, 600)), int(rng.integers(30, 120)), 0.1, 0.05, 0.1, 0.5, 500 + i, 16,
                        "f64") for i in range(3)]
    gps = [racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage="f64") for w in ws]
    lmax = [np.max(np.abs(w.D.T @ w.y)) / (w.N * 0.5) for w in ws]
    lams = [W.lambda_grid(lm, 5, 0.05) for lm in lmax]
    say("warm path, fixed iterations")
    stages, iters = racmb.solve_path(gps, lams, alpha=0.5, s=16, seed=9, max_iter=25, check_every=5, tol=0.0)
    for i, w in enumerate(ws):
        st = None
        for j in range(5):
            P = O.en_problem(w.D, w.y, lam=lams[i][j], alpha=0.5)
            ref = O.solve(P, s=16, seed=9, inst=i, beta0=0.1 * lams[i][j], max_iter=25, check_every=5, state=st)
            r, x, z, xi = stages[j][i]
            assert rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8 and rel(x, ref.x) < 1e-8, (i, j)
            st = (ref.x, ref.z, ref.xi, 0.0)
    say("warm path to tolerance against cold solves")
    kw = dict(alpha=0.5, s=16, seed=9, max_iter=3000, check_every=10, tol=1e-9, beta_mode=racmb.BETA_RESBAL)
    warm, it_w = racmb.solve_path(gps, lams, warm=True, **kw)
    cold, it_c = racmb.solve_path(gps, lams, warm=False, **kw)
    for j in range(5):
        for i in range(3):
            assert warm[j][i][0].status == racmb.RUN_CONVERGED and cold[j][i][0].status == racmb.RUN_CONVERGED
            np.testing.assert_allclose(warm[j][i][2], cold[j][i][2], rtol=1e-6, atol=1e-8)
    assert sum(it_w) <= sum(it_c)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_nonfinite_device_arrays_are_rejected(storage):
    """rac_solver_create and rac_batch_create read the problem's device arrays once and
    reject a NaN or an infinity in F, c or h (RAC_ERR_ARG); the unmodified problem is
    accepted."""
    w = W.gaussian_en(300, 40, 0.1, 0.05, 0.1, 0.5, 77, 16, storage)
    lane = [(0, racmb.PROX_EN, w.lam, 0.5, 1.0)]

    def fresh():
        return racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage=storage, h=np.zeros(w.n))

    gp = fresh()
    racmb.Solver(gp, s=16, max_iter=1).close()
    racmb.Batch([gp], lane, s=16, max_iter=1).close()
    for what in ("F", "c", "h"):
        for bad in (float("nan"), float("inf"), -float("inf")):
            gp = fresh()
            t = getattr(gp, what)
            if what == "F":
                t[3, 5] = bad          # column 3, row 5
            else:
                t[7] = bad
            torch.cuda.synchronize()
            say(storage, what, bad)
            with pytest.raises(racmb.RacError) as e:
                racmb.Solver(gp, s=16, max_iter=1)
            assert e.value.code == racmb.RAC_ERR_ARG
            with pytest.raises(racmb.RacError) as e:
                racmb.Batch([gp], lane, s=16, max_iter=1)
            assert e.value.code == racmb.RAC_ERR_ARG
