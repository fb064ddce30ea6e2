"""Pins of the oracle's general form, its RP variant, its residual history and
its penalty decisions.

Every test checks the oracle against something computed independently of it:
numpy recomputations of the residual norms and KKT residual from the iterates,
the residual-balancing rule of Boyd et al. (2011, Sec.3.4.1), a numpy forward
pass written from the parameter layout documented in include/racmb.h, Adam
written from Kingma & Ba (2015), the paper's linear-map form of one iteration
(Sec.2), closed-form KKT systems of equality-constrained QPs, and brute-force
enumeration of box-constrained QPs.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_1907_01995_amd import workloads as W


# --------------------------------------------------------------------------
# independent numpy pieces

def np_H(P):
    H = P.F.T @ P.F / P.Ns
    if P.Hd is not None:
        H = H + P.Hd
    if P.h is not None:
        H = H + np.diag(P.h)
    return H


def np_eq(P):
    if P.A is not None:
        return np.atleast_2d(P.A).astype(float), np.atleast_1d(P.beq).astype(float)
    if P.a is not None:
        return P.a[None, :].astype(float), np.array([float(P.b)])
    return np.zeros((0, P.n)), np.zeros(0)


def np_kkt(P, x, z, xi, mu):
    """The KKT residual as documented for rac_kkt (include/racmb.h), in numpy."""
    H = np_H(P)
    A, b = np_eq(P)
    mu = np.atleast_1d(np.asarray(mu, dtype=float))[:A.shape[0]]
    Hx = H @ x
    Amu = A.T @ mu if A.shape[0] else np.zeros_like(x)
    feas = np.max(np.abs(x - z)) / (1 + max(np.max(np.abs(x)), np.max(np.abs(z))))
    if A.shape[0]:
        feas = max(feas, np.max(np.abs(A @ x - b)) /
                   (1 + np.max(np.abs(b)) + np.max(np.abs(A)) * np.max(np.abs(x))))
    scale = max(np.max(np.abs(Hx)), np.max(np.abs(P.c)), np.max(np.abs(xi)),
                np.max(np.abs(Amu)) if A.shape[0] else 0.0, 1e-300)
    stat = np.max(np.abs(Hx + P.c - xi - Amu)) / scale
    if P.prox == O.PROX_NONE:
        d = np.abs(xi)
    elif P.prox == O.PROX_EN:
        la, l2 = P.lam * P.alpha, P.lam * (1 - P.alpha)
        d = np.where(z > 0, np.abs(-xi - (la + l2 * z)),
                     np.where(z < 0, np.abs(-xi - (-la + l2 * z)), np.maximum(np.abs(xi) - la, 0)))
    else:
        w = -xi
        at_lo, at_hi = z <= P.lo, z >= P.hi
        d = np.where(at_lo & at_hi, 0.0, np.where(at_lo, np.maximum(w, 0),
                                                   np.where(at_hi, np.maximum(-w, 0), np.abs(w))))
    return max(feas, stat, np.max(d) / scale)


def np_forward(w, f, ymax=np.log(10.0)):
    """8 -> 64 -> 64 -> 1 tanh network from the documented parameter layout
    W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major matrices)."""
    o = 0
    W1 = w[o:o + 512].reshape(64, 8); o += 512
    b1 = w[o:o + 64]; o += 64
    W2 = w[o:o + 4096].reshape(64, 64); o += 4096
    b2 = w[o:o + 64]; o += 64
    W3 = w[o:o + 64]; o += 64
    b3 = w[o]
    h1 = np.tanh(W1 @ f + b1)
    h2 = np.tanh(W2 @ h1 + b2)
    return ymax * np.tanh(W3 @ h2 + b3)


def np_features(rp, rd, rp_old, rd_old, kkt, kkt_prev, last_l10, decisions):
    """Controller features as documented for rac_solver_features (include/racmb.h)."""
    lg = lambda v: np.log10(max(v, 1e-300))
    f = np.array([0.5 * (lg(rp) - lg(rd)), 0.5 * (lg(rp_old) - lg(rd_old)), lg(rp) - lg(rp_old),
                  lg(rd) - lg(rd_old), lg(kkt) - lg(kkt_prev) if kkt_prev > 0 else 0.0, last_l10,
                  (lg(kkt) + 6.0) / 3.0, decisions / 10.0])
    return np.clip(f, -4.0, 4.0)


def resbal_rule(rp, rd, mu_rb=10.0, tau=2.0):
    """Residual balancing, Boyd et al. (2011) Sec.3.4.1."""
    if rp > mu_rb * rd:
        return tau
    if rd > mu_rb * rp:
        return 1.0 / tau
    return 1.0


def _small_svm(n=40, r=6, seed=3):
    rng = np.random.default_rng(seed)
    yl = rng.choice([-1.0, 1.0], n)
    X = 0.6 * yl[:, None] + rng.standard_normal((n, r))
    return O.svm_problem(X, yl, 1.0), X, yl


def _replay(P, full, beta_hist, K, p, seed, rp=False):
    """Replay a run one iteration at a time with its penalties as a schedule;
    returns the per-iteration states (x, z, xi, mu) and z before each iteration."""
    st, states, zprevs = None, [], []
    for k in range(K):
        zprevs.append(np.zeros(P.n) if st is None else st[1].copy())
        r = O.solve(P, p=p, seed=seed, iter0=k, beta_mode=O.BETA_SCHEDULE,
                    beta_sched=[beta_hist[k]], max_iter=1, state=st, rp=rp)
        st = (r.x, r.z, r.xi, r.mu)
        states.append(st)
    return states, zprevs


# --------------------------------------------------------------------------
# residual history r_p, r_d (stacked r_p reading) and the penalty decisions

@pytest.mark.parametrize("rp_variant", [False, True])
def test_residual_history_and_resbal_decisions(rp_variant):
    P, _, _ = _small_svm()
    K, T, p, seed = 60, 10, 5, 7
    full = O.solve(P, p=p, seed=seed, beta0=0.05, beta_mode=O.BETA_RESBAL, max_iter=K, check_every=T,
                   rp=rp_variant)
    assert full.iters == K
    betas = full.betas
    states, zprevs = _replay(P, full, betas, K, p, seed, rp=rp_variant)
    A, b = np_eq(P)
    decisions = 0
    for k in range(K):
        x, z, xi, mu = states[k]
        rp_np = math.sqrt(np.sum((x - z) ** 2) + np.sum((A @ x - b) ** 2))
        rd_np = betas[k] * np.linalg.norm(z - zprevs[k])
        assert abs(full.r_p[k] - rp_np) <= 1e-9 * rp_np
        assert abs(full.r_d[k] - rd_np) <= 1e-9 * max(rd_np, 1e-300)
        if (k + 1) % T == 0:
            assert abs(full.kkts[k] - np_kkt(P, x, z, xi, mu)) <= 1e-9 * full.kkts[k]
            if k + 1 < K:
                assert betas[k + 1] == betas[k] * resbal_rule(rp_np, rd_np)
                decisions += betas[k + 1] != betas[k]
        elif k + 1 < K:
            assert betas[k + 1] == betas[k]
    assert decisions >= 2          # the run exercised the rule
    np.testing.assert_allclose(states[-1][1], full.z, rtol=1e-9, atol=1e-12)


def test_mlp_decisions_follow_numpy_forward_of_numpy_features():
    P, _, _ = _small_svm(seed=5)
    rng = np.random.default_rng(4)
    w = 0.4 * rng.standard_normal(O.mlp_nparam())
    K, T, p = 50, 10, 4
    full = O.solve(P, p=p, seed=2, beta0=0.3, beta_mode=O.BETA_MLP, mlp_w=w, max_iter=K, check_every=T)
    h = full.hist
    kkt_prev, last, dec = -1.0, 0.0, 0
    changes = 0
    for k in range(T - 1, K - 1, T):
        k0 = k + 1 - T
        f = np_features(h[k, 0], h[k, 1], h[k0, 0], h[k0, 1], h[k, 3], kkt_prev, last, dec)
        mult = math.exp(np_forward(w, f))
        assert abs(h[k + 1, 2] / h[k, 2] - mult) <= 1e-12 * mult
        changes += abs(mult - 1.0) > 1e-3
        kkt_prev, last, dec = h[k, 3], math.log10(mult), dec + 1
    assert changes >= 2


def test_mlp_forward_layout_matches_numpy():
    rng = np.random.default_rng(8)
    w = 0.5 * rng.standard_normal(O.mlp_nparam())
    f = rng.uniform(-3, 3, (7, 8))
    got = O.mlp_forward(w, f)
    want = np.array([np_forward(w, fi) for fi in f])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
    # every parameter block is used where the layout says: perturbing b3 shifts o only
    w2 = w.copy()
    w2[-1] += 0.1
    np.testing.assert_allclose(O.mlp_forward(w2, f), [np_forward(w2, fi) for fi in f], rtol=1e-13)


def test_adam_steps_two_to_five_match_kingma_ba():
    rng = np.random.default_rng(9)
    npar = 37
    w = rng.standard_normal(npar)
    m, v = np.zeros(npar), np.zeros(npar)
    wr, mr, vr = w.copy(), np.zeros(npar), np.zeros(npar)
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    for t in range(1, 6):
        g = rng.standard_normal(npar) * (0.1 * t)
        O.adam_step(w, g, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mr = b1 * mr + (1 - b1) * g
        vr = b2 * vr + (1 - b2) * g * g
        wr = wr - lr * (mr / (1 - b1 ** t)) / (np.sqrt(vr / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(w, wr, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(m, mr, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(v, vr, rtol=1e-13, atol=1e-18)


# --------------------------------------------------------------------------
# RP-MBADMM (Sec.1): fixed contiguous blocks, random order

def _lcqp(P):
    """The split problem (prox NONE) as the LCQP of Eq.(4) over (x, z)."""
    n = P.n
    Ht = np.zeros((2 * n, 2 * n))
    Ht[:n, :n] = np_H(P)
    ct = np.concatenate([P.c, np.zeros(n)])
    A, b = np_eq(P)
    rows = [np.hstack([np.eye(n), -np.eye(n)])]
    if A.shape[0]:
        rows.append(np.hstack([A, np.zeros((A.shape[0], n))]))
    bt = np.concatenate([np.zeros(n), b])
    return Ht, ct, np.vstack(rows), bt


def _paper_map(H, c, A, b, beta, order_blocks):
    """L_sigma, R_sigma, Lbar, Rbar, bbar as defined in Sec.2 (one RAC/RP iteration)."""
    nv = H.shape[0]
    S = H + beta * A.T @ A
    pos = np.empty(nv, dtype=int)
    for i, blk in enumerate(order_blocks):
        pos[np.asarray(blk)] = i
    L = np.where(pos[:, None] >= pos[None, :], S, 0.0)
    R = L - S
    m = A.shape[0]
    Lbar = np.block([[L, np.zeros((nv, m))], [beta * A, np.eye(m)]])
    Rbar = np.block([[R, A.T], [np.zeros((m, nv)), np.eye(m)]])
    bbar = np.concatenate([-c + beta * A.T @ b, beta * b])
    return Lbar, Rbar, bbar


def _rand_general(rng, n=7, m=5, meq=2, dense=True):
    F = rng.standard_normal((m, n))
    G = rng.standard_normal((n, n))
    Hd = G @ G.T / n if dense else None
    return O.Problem(F=np.asfortranarray(F), Ns=2.0, c=rng.standard_normal(n), h=rng.uniform(0.1, 0.4, n),
                     Hd=Hd, A=rng.standard_normal((meq, n)) if meq else None,
                     beq=rng.standard_normal(meq) if meq else None)


@pytest.mark.parametrize("rp_variant,meq,dense", [(True, 0, False), (True, 2, True), (False, 3, True),
                                                  (False, 1, True)])
def test_one_iteration_equals_paper_linear_map_general(rp_variant, meq, dense):
    rng = np.random.default_rng(12 + meq)
    n, p, beta, seed, it = 7, 3, 0.6, 4, 9
    P = _rand_general(rng, n=n, meq=meq, dense=dense)
    x0, z0, xi0 = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    mu0 = rng.standard_normal(meq) if meq else 0.0
    r = O.solve(P, p=p, seed=seed, iter0=it, beta0=beta, max_iter=1, state=(x0, z0, xi0, mu0), rp=rp_variant)
    st = O.block_starts(n, p)
    if rp_variant:
        order = O.permutation(seed, 0, it, p)
        blocks = [np.arange(st[i], st[i + 1]) for i in order]
    else:
        blocks = O.blocks(seed, 0, it, n, p)
    H, c, A, b = _lcqp(P)
    Lbar, Rbar, bbar = _paper_map(H, c, A, b, beta, blocks + [np.arange(n, 2 * n)])
    y0 = np.concatenate([xi0, np.atleast_1d(mu0)]) if meq else xi0
    zeta1 = np.linalg.solve(Lbar, Rbar @ np.concatenate([x0, z0, y0]) + bbar)
    got = np.concatenate([r.x, r.z, r.xi] + ([np.atleast_1d(r.mu)] if meq else []))
    np.testing.assert_allclose(got, zeta1, rtol=1e-11, atol=1e-12)


def test_rp_block_order_is_uniform_over_orders():
    # RP draws the order of p = 4 fixed blocks: all 4! orders, uniformly.
    p, draws = 4, 12000
    seen = [tuple(O.permutation(3, 0, k, p).tolist()) for k in range(draws)]
    counts = np.array([seen.count(o) for o in itertools.permutations(range(p))])
    assert np.all(counts > 0)
    chi2 = ((counts - draws / 24) ** 2 / (draws / 24)).sum()
    assert chi2 < stats.chi2.ppf(0.999, 23)


def test_rp_iterations_equal_cyclic_admm_with_drawn_orders():
    # Several RP iterations equal cyclic multi-block ADMM (numpy, exact block
    # minimisation by a dense solve) over the contiguous blocks in the drawn orders.
    w = W.lasso(N=120, n=24, data_seed=4, storage="f64")
    P = O.en_problem(w.D, w.y, lam=0.05, alpha=0.7)
    n, p, beta, K = w.n, 4, 0.7, 6
    r = O.solve(P, p=p, seed=5, beta0=beta, max_iter=K, rp=True)
    H = np_H(P)
    st = O.block_starts(n, p)
    x, z, xi = np.zeros(n), np.zeros(n), np.zeros(n)
    la, l2 = P.lam * P.alpha, P.lam * (1 - P.alpha)
    for k in range(K):
        for i in O.permutation(5, 0, k, p):
            B = np.arange(st[i], st[i + 1])
            g = H[B] @ x + P.c[B] - xi[B] + beta * (x[B] - z[B])
            x[B] -= np.linalg.solve(H[np.ix_(B, B)] + beta * np.eye(len(B)), g)
        v = beta * x - xi
        z = np.sign(v) * np.maximum(np.abs(v) - la, 0) / (beta + l2)
        xi = xi - beta * (x - z)
    np.testing.assert_allclose(r.x, x, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(r.z, z, rtol=1e-11, atol=1e-13)


def test_rp_single_block_equals_textbook_admm():
    # p = 1: RP and RAC are both the two-block ADMM of Boyd et al. (2011) Sec.6.4.
    w = W.lasso(N=150, n=20, data_seed=6, storage="f64")
    lam, beta, K = 0.05, 0.8, 25
    P = O.en_problem(w.D, w.y, lam=lam, alpha=1.0)
    r = O.solve(P, p=1, beta0=beta, max_iter=K, rp=True)
    H = w.D.T @ w.D / w.N
    c = -w.D.T @ w.y / w.N
    x = z = u = np.zeros(w.n)
    for _ in range(K):
        x = np.linalg.solve(H + beta * np.eye(w.n), beta * (z - u) - c)
        v = x + u
        z = np.sign(v) * np.maximum(np.abs(v) - lam / beta, 0)
        u = u + x - z
    np.testing.assert_allclose(r.z, z, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("alpha", [1.0, 0.6])
def test_rp_converges_to_brute_force_elastic_net(alpha):
    rng = np.random.default_rng(21)
    N, n = 30, 7
    D = rng.standard_normal((N, n))
    y = D @ np.array([2.0, 0, -1.5, 0, 0, 0.7, 0]) + 0.3 * rng.standard_normal(N)
    lam = 0.25 * np.max(np.abs(D.T @ y)) / N
    H = D.T @ D / N + lam * (1 - alpha) * np.eye(n)
    q = D.T @ y / N
    best = None
    for signs in itertools.product((-1, 0, 1), repeat=n):
        s = np.array(signs, dtype=float)
        act = s != 0
        xs = np.zeros(n)
        if act.any():
            xs[act] = np.linalg.solve(H[np.ix_(act, act)], q[act] - lam * alpha * s[act])
            if np.any(np.sign(xs[act]) != s[act]):
                continue
        if np.all(np.abs((H @ xs - q)[~act]) <= lam * alpha + 1e-12):
            best = xs
    P = O.en_problem(D, y, lam=lam, alpha=alpha)
    r = O.solve(P, p=3, beta0=1.0, max_iter=800, rp=True)
    np.testing.assert_allclose(r.z, best, rtol=1e-9, atol=1e-11)


# --------------------------------------------------------------------------
# general form: several equality rows and an explicit dense H

def test_equality_constrained_qp_matches_kkt_system():
    # min 1/2 x'Hx + c'x s.t. A x = b  <=>  [H A'; A 0][x; -mu] = [-c; b]   (Eq.(1)/(4))
    rng = np.random.default_rng(31)
    n, meq = 30, 3
    P = _rand_general(rng, n=n, m=40, meq=meq, dense=True)
    H = np_H(P)
    A, b = np_eq(P)
    K = np.block([[H, A.T], [A, np.zeros((meq, meq))]])
    sol = np.linalg.solve(K, np.concatenate([-P.c, b]))
    r = O.solve(P, s=8, beta0=1.0, max_iter=3000, check_every=10, tol=1e-12)
    assert r.status == O.RUN_CONVERGED
    np.testing.assert_allclose(r.z, sol[:n], rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(r.mu, -sol[n:], rtol=1e-8, atol=1e-9)
    assert O.kkt(P, sol[:n], sol[:n], np.zeros(n), -sol[n:]) < 1e-12


def test_dense_h_ridge_closed_form_and_objective():
    rng = np.random.default_rng(32)
    n, lam = 25, 0.4
    G = rng.standard_normal((n, n))
    Hd = G @ G.T / n
    P = O.Problem(F=np.zeros((0, n), order="F"), Ns=1.0, c=rng.standard_normal(n), Hd=Hd, prox=O.PROX_EN,
                  lam=lam, alpha=0.0)
    r = O.solve(P, s=5, beta0=1.0, max_iter=600)
    np.testing.assert_allclose(r.z, np.linalg.solve(Hd + lam * np.eye(n), -P.c), rtol=1e-9, atol=1e-11)
    z = rng.standard_normal(n)
    direct = 0.5 * z @ Hd @ z + P.c @ z + lam / 2 * z @ z
    assert abs(O.objective(P, z) - direct) < 1e-12 * abs(direct)


def _gauss_kernel(X, Y, gamma):
    d = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    return np.exp(-gamma * d)


def test_gaussian_kernel_svm_brute_force_and_bias():
    # C-SVC dual of Eq.(9) with the Gaussian kernel of Sec.3.2, Q_ij = y_i y_j K_ij,
    # against enumeration of {0, C, free}^n with the equality row; the bias of the
    # decision function is b = -mu (the equality multiplier), which equals
    # y_i - sum_j alpha_j y_j K_ij on every free support vector.
    rng = np.random.default_rng(6)
    n, r_, Cb, gamma = 8, 2, 1.0, 0.5
    yl = np.array([1, -1, 1, -1, 1, 1, -1, -1], dtype=float)
    X = 0.7 * yl[:, None] + rng.standard_normal((n, r_))
    Kx = _gauss_kernel(X, X, gamma)
    Q = yl[:, None] * Kx * yl[None, :]
    best, best_obj = None, np.inf
    for st in itertools.product((0, 1, 2), repeat=n):
        st = np.array(st)
        al = np.where(st == 1, Cb, 0.0)
        Fr = st == 2
        if Fr.any():
            k = Fr.sum()
            Kk = np.zeros((k + 1, k + 1))
            Kk[:k, :k] = Q[np.ix_(Fr, Fr)]
            Kk[:k, k] = yl[Fr]
            Kk[k, :k] = yl[Fr]
            rhs = np.concatenate([1.0 - Q[np.ix_(Fr, ~Fr)] @ al[~Fr], [-yl[~Fr] @ al[~Fr]]])
            sol = np.linalg.solve(Kk, rhs)
            al[Fr] = sol[:k]
        if abs(yl @ al) > 1e-9 or np.any(al < -1e-12) or np.any(al > Cb + 1e-12):
            continue
        g = Q @ al - 1.0
        # optimality of the candidate: with nu = the free-SV multiplier, check the box conditions
        obj = 0.5 * al @ Q @ al - al.sum()
        if obj < best_obj - 1e-13:
            best, best_obj = al, obj
    P = O.svm_kernel_problem(X, yl, Cb, gamma)
    r = O.solve(P, p=3, beta0=1.0, max_iter=6000, check_every=10, tol=1e-12)
    assert r.status == O.RUN_CONVERGED
    assert abs(O.objective(P, r.z) - best_obj) < 1e-9 * abs(best_obj)
    np.testing.assert_allclose(r.z, best, atol=1e-7)   # Q is positive definite: alpha is unique
    free = (best > 1e-6) & (best < Cb - 1e-6)
    assert free.any()
    b_sv = yl[free] - Kx[free] @ (best * yl)
    np.testing.assert_allclose(-r.mu, b_sv, atol=1e-7)
    assert abs(O.svm_bias(r) - b_sv[0]) < 1e-7
    # decision function and accuracy on the training points
    f = O.svm_decision(X, yl, r.z, O.svm_bias(r), gamma, X)
    np.testing.assert_allclose(f, Kx @ (r.z * yl) - r.mu, rtol=1e-12, atol=1e-12)
    assert 0.0 <= O.svm_accuracy(f, yl) <= 1.0


def test_kkt_general_zero_at_solution_and_linear_in_perturbation():
    rng = np.random.default_rng(33)
    n, meq = 12, 2
    P = _rand_general(rng, n=n, m=9, meq=meq, dense=True)
    H = np_H(P)
    A, b = np_eq(P)
    sol = np.linalg.solve(np.block([[H, A.T], [A, np.zeros((meq, meq))]]), np.concatenate([-P.c, b]))
    xs, mus = sol[:n], -sol[n:]
    assert O.kkt(P, xs, xs, np.zeros(n), mus) < 1e-13
    d = np.zeros(n)
    d[3] = 1e-4
    k1 = O.kkt(P, xs + d, xs + d, np.zeros(n), mus)
    assert abs(k1 - np_kkt(P, xs + d, xs + d, np.zeros(n), mus)) < 1e-12 * k1
    assert abs(O.kkt(P, xs + 2 * d, xs + 2 * d, np.zeros(n), mus) / k1 - 2.0) < 1e-3
    # a large multiplier dominates the scale through |A'mu|_inf
    xi = rng.standard_normal(n)
    kb = O.kkt(P, xs + d, xs, xi, 300.0 * mus)
    assert abs(kb - np_kkt(P, xs + d, xs, xi, 300.0 * mus)) < 1e-12 * kb


def test_warm_started_lambda_path_ends_at_cold_solutions():
    # Sec.3.1: a decreasing lambda path, each point started from the previous
    # point's (x, z, xi), reaches the same solutions as cold starts.
    w = W.lasso(N=200, n=40, data_seed=12, storage="f64")
    lams = W.lambda_grid(np.max(np.abs(w.D.T @ w.y)) / (w.N * 0.5), 5, 0.05)
    st, total_warm, total_cold = None, 0, 0
    for lam in lams:
        P = O.en_problem(w.D, w.y, lam=lam, alpha=0.5)
        rw = O.solve(P, s=8, beta0=0.1 * lam, beta_mode=O.BETA_RESBAL, max_iter=4000, check_every=10,
                     tol=1e-10, state=st)
        rc = O.solve(P, s=8, beta0=0.1 * lam, beta_mode=O.BETA_RESBAL, max_iter=4000, check_every=10,
                     tol=1e-10)
        assert rw.status == O.RUN_CONVERGED and rc.status == O.RUN_CONVERGED
        np.testing.assert_allclose(rw.z, rc.z, rtol=1e-7, atol=1e-9)
        st = (rw.x, rw.z, rw.xi, rw.mu)
        total_warm += rw.iters
        total_cold += rc.iters
    assert total_warm <= total_cold


def test_stored_lasso_20000x2000_solution_is_optimal():
    """The stored oracle optimum of lasso_20000x2000 (tests/golden, written by make_golden.py)
    checked against the LASSO optimality conditions of Eq.(6) with alpha = 1, recomputed with
    numpy from the same stored values: g = D'(Dz - y)/N equals -lambda sign(z_j) on the support
    and lies in [-lambda, lambda] off it (to 1e-9 of |D'y/N|_inf, the oracle's stopping
    tolerance), and the stored objective is that of z."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_golden
    w = W.lasso_20000x2000("f32")
    head, z = make_golden.read(os.path.join(os.path.dirname(make_golden.__file__), "lasso_20000x2000_solution.txt"))
    D = w.D.astype(np.float64)
    N = D.shape[0]
    r = D @ z - w.y
    g = D.T @ r / N
    on = z != 0
    assert 0 < on.sum() < z.size
    scale = np.max(np.abs(D.T @ w.y)) / N           # |c|_inf, the scale of the KKT residual
    assert np.max(np.abs(g[on] + w.lam * np.sign(z[on]))) <= 1e-9 * scale
    assert np.max(np.abs(g[~on])) <= w.lam
    obj = 0.5 * (r @ r) / N + w.lam * np.abs(z).sum()
    assert abs(obj - float(head["objective"])) <= 1e-12 * obj
    assert abs(np.linalg.norm(z) - float(head["znorm"])) <= 1e-12 * np.linalg.norm(z)
