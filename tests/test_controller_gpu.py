"""Learned penalty controller on the GPU: training kernels against the oracle's
FP64 training, features against the oracle's definition, the residual-balancing
fallback, and the gain of the trained network over the rules it replaces."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import controller as CT
from paper_1907_01995_amd import racmb, workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


def test_gpu_training_follows_oracle_training():
    rng = np.random.default_rng(3)
    X = rng.uniform(-3, 3, (96, 8)).astype(np.float32)
    Y = np.tanh(X[:, 0] - 0.5 * X[:, 3]).astype(np.float32) * 1.5
    w0 = CT.init_weights(5)
    wd = torch.as_tensor(w0, device="cuda")
    m, v = torch.zeros_like(wd), torch.zeros_like(wd)
    Xd, Yd = torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda")
    wo, mo, vo = w0.astype(np.float64), np.zeros(w0.size), np.zeros(w0.size)
    gl, ol = [], []
    for t in range(1, 61):
        lg, g = racmb.mlp_loss_grad(wd, Xd, Yd, CT.YMAX)
        racmb.mlp_adam(wd, g, m, v, t, lr=3e-3)
        lo, go = O.mlp_loss_grad(wo, X.astype(np.float64), Y.astype(np.float64), CT.YMAX)
        O.adam_step(wo, go, mo, vo, t, lr=3e-3)
        gl.append(lg)
        ol.append(lo)
    np.testing.assert_allclose(gl, ol, rtol=2e-4)
    assert gl[-1] < 0.2 * gl[0]
    w1 = wd.cpu().numpy()
    assert np.max(np.abs(w1 - wo)) / np.max(np.abs(wo)) < 1e-3


def test_features_match_oracle_definition():
    w = W.lasso(N=1500, n=200, data_seed=17, block_size=32, storage="f64")
    gp = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f64")
    op = O.en_problem(w.D, w.y, lam=w.lam, alpha=1.0)
    s = racmb.Solver(gp, s=32, beta0=w.beta0, beta_mode=racmb.BETA_FIXED, max_iter=20, check_every=10)
    s.run()
    f = s.features()
    ref = O.solve(op, s=32, beta0=w.beta0, max_iter=20, check_every=10)
    rp, rd, kk = ref.r_p, ref.r_d, ref.kkts
    fo = O.controller_features(rp[19], rd[19], rp[10], rd[10], kk[19], kk[9], 0.0, 0)
    np.testing.assert_allclose(f, fo, rtol=1e-5, atol=1e-6)


def test_nonfinite_network_falls_back_to_residual_balancing():
    w = W.lasso(N=2000, n=256, data_seed=19, block_size=64, storage="f32")
    gp = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f32")
    bad = torch.full((racmb.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
    kw = dict(s=64, beta0=w.beta0, max_iter=80, check_every=10, precision=racmb.PREC_MIXED)
    a = racmb.Solver(gp, beta_mode=racmb.BETA_MLP, mlp_weights=bad, **kw)
    a.run()
    b = racmb.Solver(gp, beta_mode=racmb.BETA_RESBAL, **kw)
    b.run()
    np.testing.assert_array_equal(a.history()[:, 2], b.history()[:, 2])
    for u, v in zip(a.state()[:3], b.state()[:3]):
        assert np.array_equal(u, v)


@pytest.mark.skipif(not os.path.exists(CT.WEIGHTS_PATH), reason="no trained weights")
def test_trained_controller_reaches_tolerance_in_fewer_iterations():
    wts = np.load(CT.WEIGHTS_PATH)
    specs = CT.sample_specs(9, 424242)          # held out: not the training seed's problems
    res = CT.evaluate(wts, specs, log=say)
    mlp, rb, fix = res.mean(axis=0)
    say("mean iterations mlp %.1f rb %.1f fixed %.1f" % (mlp, rb, fix))
    assert np.all(res[:, 0] < 3000)             # the network converged everywhere
    assert mlp < rb and mlp < fix


@pytest.mark.skipif(not os.path.exists(CT.WEIGHTS_PATH), reason="no trained weights")
def test_controller_keeps_the_fixed_point():
    # beta only changes the path: the network-driven solve ends at the oracle's solution
    w = W.lasso(N=2500, n=300, data_seed=23, block_size=64, storage="f32")
    gp = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f32")
    op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
    wd = torch.as_tensor(np.load(CT.WEIGHTS_PATH), device="cuda")
    s = racmb.Solver(gp, s=64, beta0=w.beta0, beta_mode=racmb.BETA_MLP, mlp_weights=wd,
                     precision=racmb.PREC_MIXED, max_iter=2000, check_every=10, tol=1e-9)
    r = s.run()
    assert r.status == racmb.RUN_CONVERGED
    ref = O.solve(op, s=64, beta0=1.0 / w.N, beta_mode=O.BETA_RESBAL, max_iter=3000, check_every=10,
                  tol=1e-11)
    z = s.state()[1]
    assert np.max(np.abs(z - ref.z)) / np.max(np.abs(ref.z)) < 1e-5
