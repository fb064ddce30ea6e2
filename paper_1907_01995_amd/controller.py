"""Learned penalty controller: training data from the solver's own trajectories,
training on the GPU with the library's forward/backward/Adam kernels, and
evaluation against residual balancing and a fixed penalty.

The paper sets the penalty by hand-made rules (gamma = 0.1 lambda or lambda for
the elastic net, Sec.3.1; beta = 0.1 p for the SVM, Sec.3.2) and its theory
assumes a fixed penalty (Thm 2.2 / 2.5).  The controller is a project addition:
every T iterations it maps features of the residual history to a multiplier in
[1/10, 10] for beta.  Non-finite outputs fall back to residual balancing inside
the library.

Labels come from short rollouts: at each decision point of a trajectory the
solver state is exported, each candidate multiplier m is applied to a copy and
run for H iterations at fixed penalty, and the label is ln(m*) for the m* with
the smallest KKT residual at the end.  The trajectory then continues with a mix
of the labelled action, a random action and the residual-balancing action, so
the data cover states the learned policy and the fallback will visit.

Training problems are small instances shaped like the least-squares, LASSO and
batched elastic-net workloads (unnormalised Gaussian and unit-norm designs,
several lambda and alpha values, penalties started from the paper's rule
perturbed by up to a decade either way).
"""
from __future__ import annotations

import argparse
import math
import os
import time
from dataclasses import dataclass

import numpy as np

from . import racmb
from . import workloads as W

MULTS = np.array([0.1, 0.25, 0.5, 1.0, 2.0, 4.0, 10.0])
YMAX = math.log(10.0)
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "controller_weights.npy")


@dataclass
class Spec:
    kind: str           # "ols", "lasso", "en"
    N: int
    n: int
    seed: int
    lam_frac: float
    alpha: float
    beta_scale: float
    block: int
    storage: str = "f32"


def sample_specs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = ["ols", "lasso", "en"][i % 3]
        N = int(np.exp(rng.uniform(np.log(600), np.log(4000))))
        n = int(np.exp(rng.uniform(np.log(64), np.log(min(600, N // 2)))))
        out.append(Spec(kind, N, n, int(rng.integers(1 << 30)), float(rng.uniform(0.03, 0.4)),
                        0.5 if kind == "en" else 1.0, float(10 ** rng.uniform(-1.0, 1.0)),
                        int(rng.choice([32, 64])), str(rng.choice(["f32", "bf16"]))))
    return out


def build_problem(spec: Spec):
    """(device problem, beta0) for a spec."""
    if spec.kind == "ols":
        w = W.least_squares(spec.N, spec.n, 0.01, spec.seed, spec.block, 1.0, spec.storage)
        beta0 = 1.0 * spec.beta_scale
        lam, alpha = 0.0, 1.0
    elif spec.kind == "lasso":
        w = W.lasso(spec.N, spec.n, 0.05, 0.05, spec.lam_frac, 1.0, spec.seed, spec.block, spec.storage)
        beta0, lam, alpha = w.beta0 * spec.beta_scale, w.lam, 1.0
    else:
        w = W.gaussian_en(spec.N, spec.n, 0.1, 0.05, spec.lam_frac, spec.alpha, spec.seed, spec.block,
                          spec.storage)
        beta0, lam, alpha = w.beta0 * spec.beta_scale, w.lam, spec.alpha
    prob = racmb.regression_problem(w.D, w.y, lam=lam, alpha=alpha, storage=spec.storage)
    return prob, beta0


def rb_multiplier(f):
    """Residual balancing (mu = 10, tau = 2) read from feature 0 = 0.5 log10(r_p/r_d)."""
    if f[0] > 0.5:
        return 2.0
    if f[0] < -0.5:
        return 0.5
    return 1.0


def generate(specs, T=10, H=20, max_decisions=25, tol=1e-6, seed=0, log=print):
    """Features and rollout labels (ln of the best multiplier) from solver trajectories."""
    rng = np.random.default_rng(seed)
    X, Y = [], []
    for si, spec in enumerate(specs):
        prob, beta0 = build_problem(spec)
        p = -(-spec.n // spec.block)
        common = dict(p=p, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_FIXED, check_every=T,
                      seed=spec.seed % 1000)
        base = racmb.Solver(prob, beta0=beta0, max_iter=T, tol=tol, **common)
        roll = racmb.Solver(prob, beta0=beta0, max_iter=H, tol=0.0, **common)
        nd = 0
        for d in range(max_decisions):
            r = base.run()
            if r.status != racmb.RUN_MAX_ITER:
                break
            f = base.features()
            blob = base.export_state()
            scores = []
            for m in MULTS:
                roll.import_state(blob)
                roll.scale_beta(m)
                rr = roll.run()
                k = rr.kkt if np.isfinite(rr.kkt) else 1e300
                scores.append(math.log10(max(k, 1e-300)))
            scores = np.array(scores)
            best = int(np.argmin(scores))
            if scores[3] <= scores[best] + 1e-3:      # prefer leaving beta alone on near-ties
                best = 3
            X.append(f.copy())
            Y.append(math.log(MULTS[best]))
            nd += 1
            u = rng.uniform()
            act = MULTS[best] if u < 0.6 else (rng.choice(MULTS) if u < 0.8 else rb_multiplier(f))
            if act != 1.0:
                base.scale_beta(act)
        base.close()
        roll.close()
        log("spec %d %s N=%d n=%d: %d decisions" % (si, spec.kind, spec.N, spec.n, nd))
    return np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32)


def init_weights(seed=0):
    rng = np.random.default_rng(seed)
    H, I = racmb.MLP_HIDDEN, racmb.MLP_IN
    W1 = rng.standard_normal((H, I)) / math.sqrt(I)
    W2 = rng.standard_normal((H, H)) / math.sqrt(H)
    W3 = 0.01 * rng.standard_normal(H)
    w = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, [0.0]])
    assert w.size == racmb.MLP_NPARAM
    return w.astype(np.float32)


def train(X, Y, steps=3000, lr=3e-3, seed=0, log=print, every=500):
    """Full-batch Adam (cosine-decayed step size) on the GPU with the library's kernels;
    returns (weights, losses)."""
    import torch
    w = torch.as_tensor(init_weights(seed), device="cuda")
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda")
    Yd = torch.as_tensor(np.ascontiguousarray(Y, dtype=np.float32), device="cuda")
    losses = []
    for t in range(1, steps + 1):
        loss, g = racmb.mlp_loss_grad(w, Xd, Yd, YMAX)
        racmb.mlp_adam(w, g, m, v, t, lr=lr * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps)))
        losses.append(loss)
        if t % every == 0 or t == 1:
            log("step %d loss %.5f" % (t, loss))
    return w.cpu().numpy(), np.array(losses)


def iterations_to_tol(prob, beta0, p, mode, weights=None, tol=1e-6, max_iter=3000, T=10, seed=0):
    import torch
    wd = None if weights is None else torch.as_tensor(np.asarray(weights, np.float32), device="cuda")
    s = racmb.Solver(prob, p=p, precision=racmb.PREC_MIXED, beta0=beta0, beta_mode=mode,
                     mlp_weights=wd, check_every=T, max_iter=max_iter, tol=tol, seed=seed)
    r = s.run()
    s.close()
    return r.iters if r.status == racmb.RUN_CONVERGED else max_iter * 10


def evaluate(weights, specs, log=print):
    """Iterations to KKT <= 1e-6 for the network, residual balancing and the fixed penalty."""
    rows = []
    for spec in specs:
        prob, beta0 = build_problem(spec)
        p = -(-spec.n // spec.block)
        kw = dict(seed=spec.seed % 1000)
        it_mlp = iterations_to_tol(prob, beta0, p, racmb.BETA_MLP, weights, **kw)
        it_rb = iterations_to_tol(prob, beta0, p, racmb.BETA_RESBAL, **kw)
        it_fix = iterations_to_tol(prob, beta0, p, racmb.BETA_FIXED, **kw)
        rows.append((it_mlp, it_rb, it_fix))
        log("%s N=%d n=%d scale=%.2f: mlp %d rb %d fixed %d" % (spec.kind, spec.N, spec.n,
                                                               spec.beta_scale, it_mlp, it_rb, it_fix))
    return np.array(rows)


def main():
    ap = argparse.ArgumentParser(description="train the penalty controller on the GPU")
    ap.add_argument("--out", default=WEIGHTS_PATH)
    ap.add_argument("--train-problems", type=int, default=600)
    ap.add_argument("--eval-problems", type=int, default=30)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--data-out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t0 = time.time()
    log = lambda *a: print(*a, flush=True)
    X, Y = generate(sample_specs(args.train_problems, args.seed), seed=args.seed, log=log)
    log("dataset: %d samples, label histogram %s (%.1fs)" % (
        len(Y), np.unique(np.round(np.exp(Y), 2), return_counts=True), time.time() - t0))
    if args.data_out:
        np.savez(args.data_out, X=X, Y=Y)
    w, losses = train(X, Y, steps=args.steps, seed=args.seed, log=log)
    np.save(args.out, w)
    log("saved %s (%.1fs)" % (args.out, time.time() - t0))
    res = evaluate(w, sample_specs(args.eval_problems, args.seed + 1000), log=log)
    log("held-out mean iterations: mlp %.1f rb %.1f fixed %.1f" % tuple(res.mean(axis=0)))


if __name__ == "__main__":
    main()
