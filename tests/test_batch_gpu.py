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


@pytest.fixture(autouse=True, params=["solo", "teams"])
def group_mode(request, monkeypatch):
    """Every test runs twice: with the lane groups of every instance of up to 4000 rows solo
    (one workgroup each; kept solo at creation even where the batch is too small for that to
    pay) and with every group on a team of workgroups."""
    monkeypatch.delenv("RACMB_SOLO_ROWS", raising=False)
    if request.param == "teams":
        monkeypatch.setenv("RACMB_SOLO_ROWS", "0")
        monkeypatch.delenv("RACMB_SOLO_FORCE", raising=False)
    else:
        monkeypatch.setenv("RACMB_SOLO_FORCE", "1")
    return request.param


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


@pytest.mark.parametrize("s", [32, 64])
@pytest.mark.parametrize("sweep", [racmb.BSWEEP_TEAM, racmb.BSWEEP_LANE])
def test_batch_lanes_match_oracle_fp64(sweep, s):
    """Blocks of 64 take the matrix-core inverse (four pivots per step), blocks of 32 the
    one-pivot-per-step inverse; both against the oracle's sequential sweep."""
    ws, gps, ops, lanes = en_batch(s=s)
    say("batch fp64", len(lanes), "lanes, sweep", sweep, "s", s)
    b = racmb.Batch(gps, lanes, s=s, seed=7, max_iter=30, check_every=10, use_graph=True, sweep=sweep)
    it, act = b.run()
    assert it == 30 and act == len(lanes)
    info = b.info()
    say(info)
    assert info["graph"] == 1
    assert (info["team_size"] > 0) == (sweep == racmb.BSWEEP_TEAM)
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=s, seed=7, max_iter=30, check_every=10)
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


@pytest.mark.parametrize("s", [32, 64])
def test_batch_lanes_retire_like_the_oracle(s):
    ws, gps, ops, lanes = en_batch(ninst=4, lanes_per=3, seed=5, s=s)
    b = racmb.Batch(gps, lanes, s=s, seed=2, beta_mode=racmb.BETA_RESBAL, max_iter=600, check_every=10,
                    tol=1e-7)
    it, act = b.run()
    assert act == 0
    iters = []
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=s, seed=2, beta_mode=O.BETA_RESBAL, max_iter=600,
                          check_every=10, tol=1e-7)
        assert res.status == racmb.RUN_CONVERGED and ref.status == O.RUN_CONVERGED
        assert res.iters == ref.iters, (u, res.iters, ref.iters)
        assert rel(z, ref.z) < 1e-8
        iters.append(res.iters)
    assert len(set(iters)) > 1        # lanes really retired at different iterations


@pytest.mark.parametrize("s", [32, 64])
def test_batch_svm_lanes(s):
    wv = [W.svm(n=int(n), r=12, block_size=s, data_seed=40 + k) for k, n in enumerate((300, 517))]
    gps = [racmb.svm_problem(w.X, w.labels, w.C) for w in wv]
    ops = [O.svm_problem(w.X.astype(np.float64), w.labels, w.C) for w in wv]
    lanes = [(0, racmb.PROX_BOX, 0.0, 1.0, 0.5), (0, racmb.PROX_BOX, 0.0, 1.0, 3.0),
             (1, racmb.PROX_BOX, 0.0, 1.0, 1.7)]
    b = racmb.Batch(gps, lanes, s=s, seed=4, max_iter=50, check_every=10, use_graph=False)
    b.run()
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=s, seed=4, max_iter=50, check_every=10)
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


@pytest.mark.parametrize("s", [32, 64])
def test_batch_reports_assumption_failure_per_lane(s):
    ws, gps, ops, lanes = en_batch(ninst=2, lanes_per=2, seed=11, s=s)
    h = np.zeros(ws[1].n)
    h[3] = -1e4
    gps[1] = racmb.regression_problem(ws[1].D, ws[1].y, lam=ws[1].lam, alpha=0.5, h=h)
    opbad = O.en_problem(ws[1].D, ws[1].y, lam=ws[1].lam, alpha=0.5, h=h)
    b = racmb.Batch(gps, lanes, s=s, seed=3, max_iter=20, check_every=10)
    it, act = b.run()
    assert act == 2
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u, allow_not_pd=True)
        if lane[0] == 1:
            ref = oracle_lane(opbad, lane, s=s, seed=3, max_iter=20, check_every=10)
            assert ref.rc == O.ERR_NOT_PD
            assert (res.fail_iter, res.fail_block) == (ref.fail_iter, ref.fail_block)
        else:
            ref = oracle_lane(ops[0], lane, s=s, seed=3, max_iter=20, check_every=10)
            assert res.fail_iter == -1 and rel(z, ref.z) < 1e-8


def test_team_and_lane_sweeps_agree_on_uneven_groups():
    """More than 16 lanes of one instance (two groups), uneven instance sizes, an
    instance with rows just past a team's tile boundaries, BF16 data: the team
    sweep (FP64 matrix-core products) and the per-lane sweep agree to rounding,
    and the team sweep is deterministic."""
    rng = np.random.default_rng(21)
    shapes = [(1000, 150), (517, 64), (2051, 97), (33, 40)]
    gps, lanes = [], []
    for i, (N, n) in enumerate(shapes):
        w = W.gaussian_en(N, n, 0.1, 0.05, 0.1, 0.5, 200 + i, 32, "bf16")
        gps.append(racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage="bf16"))
        nl = 19 if i == 0 else 3
        for k in range(nl):
            lam = w.lam * 2.0 ** (2 - k * 0.5)
            lanes.append((i, racmb.PROX_EN, lam, 0.5, float(10 ** rng.uniform(-1.0, 0.5))))
    outs = []
    for sweep in (racmb.BSWEEP_TEAM, racmb.BSWEEP_TEAM, racmb.BSWEEP_LANE):
        b = racmb.Batch(gps, lanes, s=32, seed=3, precision=racmb.PREC_MIXED, beta_mode=racmb.BETA_RESBAL,
                        max_iter=60, check_every=10, use_graph=True, sweep=sweep)
        b.run()
        say("sweep", sweep, b.info())
        outs.append([b.lane(u)[1:] for u in range(len(lanes))])
        b.close()
    for u in range(len(lanes)):
        for a, c in zip(outs[0][u], outs[1][u]):
            assert np.array_equal(a, c)                        # deterministic
        for a, c in zip(outs[0][u], outs[2][u]):
            assert rel(a, c) < 1e-9, (u, rel(a, c))            # same iteration, other summation order


def test_team_sweep_svm_lanes_with_equality_row():
    wv = [W.svm(n=int(n), r=12, block_size=32, data_seed=60 + k) for k, n in enumerate((300, 517))]
    gps = [racmb.svm_problem(w.X, w.labels, w.C) for w in wv]
    ops = [O.svm_problem(w.X.astype(np.float64), w.labels, w.C) for w in wv]
    lanes = [(k % 2, racmb.PROX_BOX, 0.0, 1.0, 0.3 + 0.4 * k) for k in range(5)]
    b = racmb.Batch(gps, lanes, s=32, seed=6, max_iter=40, check_every=10, use_graph=True,
                    sweep=racmb.BSWEEP_TEAM)
    b.run()
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=6, max_iter=40, check_every=10)
        assert rel(x, ref.x) < 1e-8 and rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8, u


def test_batch_phase_timing_counts_every_launch():
    ws, gps, ops, lanes = en_batch(ninst=2, lanes_per=2, seed=13)
    b = racmb.Batch(gps, lanes, s=32, seed=1, max_iter=20, check_every=10, use_graph=True)
    b.set_timing(True)
    b.run()
    ph = b.timing()
    # the Grams and inverses of a chunk are one launch each when every iteration has its slot
    na = 2 if b.info()["assembly_slots"] == 10 else 20
    assert ph["sweep"][1] == 20 and ph["gram"][1] == na and ph["factor"][1] == na and ph["check"][1] == 2
    assert all(ms > 0 for ms, cnt in ph.values() if cnt)
    res, x, z, xi = b.lane(0)
    ref = oracle_lane(ops[lanes[0][0]], lanes[0], s=32, seed=1, max_iter=20, check_every=10)
    assert rel(z, ref.z) < 1e-8                       # timing does not change the iteration


@pytest.mark.parametrize("s", [32, 64])
def test_chunk_assembly_matches_per_iteration_assembly(s, monkeypatch):
    """The Grams and inverses of a whole chunk formed at its start in one launch each (a
    slot per iteration), and at each iteration into one slot: bit-identical iterates and
    the same Assumption 2.1 failure report (its iteration counted from the chunk's start)."""
    ws, gps, ops, lanes = en_batch(ninst=3, lanes_per=2, seed=17, s=s)
    h = np.zeros(ws[2].n)
    h[5] = -1e4
    gps[2] = racmb.regression_problem(ws[2].D, ws[2].y, lam=ws[2].lam, alpha=0.5, h=h)
    outs = []
    for slots in (10, 1):
        if slots == 1:
            monkeypatch.setenv("RACMB_ASSEMBLY_SLOTS", "1")
        else:
            monkeypatch.delenv("RACMB_ASSEMBLY_SLOTS", raising=False)
        b = racmb.Batch(gps, lanes, s=s, seed=3, beta_mode=racmb.BETA_RESBAL, max_iter=40, check_every=10,
                        use_graph=True)
        assert b.info()["assembly_slots"] == slots
        b.run()
        outs.append([b.lane(u, allow_not_pd=True) for u in range(len(lanes))])
        b.close()
    for u, ((ra, *va), (rb, *vb)) in enumerate(zip(*outs)):
        assert (ra.iters, ra.status, ra.fail_iter, ra.fail_block) == (rb.iters, rb.status, rb.fail_iter, rb.fail_block)
        for p, q in zip(va, vb):
            assert np.array_equal(p, q), u
    assert any(r.fail_iter >= 0 for r, *_ in outs[0]) and any(r.fail_iter < 0 for r, *_ in outs[0])


def test_solo_and_team_groups_in_one_launch():
    """Instances on both sides of the solo bound (4000 rows) in one batch: solo groups and
    teams run in the same launch; every lane matches the oracle (FP64)."""
    rng = np.random.default_rng(31)
    shapes = [(4100, 90), (800, 130), (4000, 64), (4001, 40), (150, 33)]
    gps, ops, lanes = [], [], []
    for i, (N, n) in enumerate(shapes):
        w = W.gaussian_en(N, n, 0.1, 0.05, 0.1, 0.5, 700 + i, 32, "f64")
        gps.append(racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=0.5, storage="f64"))
        ops.append(O.en_problem(w.D, w.y, lam=w.lam, alpha=0.5))
        for k in range(3 if i != 1 else 18):
            lanes.append((i, racmb.PROX_EN, w.lam * 2.0 ** (1 - 0.5 * k), 0.5, float(10 ** rng.uniform(-1.0, 0.5))))
    b = racmb.Batch(gps, lanes, s=32, seed=8, max_iter=30, check_every=10, use_graph=True,
                    sweep=racmb.BSWEEP_TEAM)
    b.run()
    say(b.info())
    for u, lane in enumerate(lanes):
        res, x, z, xi = b.lane(u)
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=8, max_iter=30, check_every=10)
        assert rel(z, ref.z) < 1e-8 and rel(xi, ref.xi) < 1e-8 and rel(x, ref.x) < 1e-8, u


def test_solo_groups_go_to_teams_as_lanes_retire(group_mode):
    """Solo groups at creation; once lanes converge and retire, the groups move to teams
    (the decision is taken from the lanes' status alone).  The lanes still retire at the
    oracle's iterations with its solution, graph replay and direct launches agree bit for
    bit across the move, and a batch that imports a state exported after the move
    continues bit for bit."""
    if group_mode != "solo":
        pytest.skip("teams only: no solo groups to move")
    ws, gps, ops, lanes = en_batch(ninst=4, lanes_per=3, seed=5)
    kw = dict(s=32, seed=2, beta_mode=racmb.BETA_RESBAL, check_every=10, tol=1e-7)
    outs, infos = [], []
    for graph in (True, False):
        b = racmb.Batch(gps, lanes, max_iter=600, use_graph=graph, **kw)
        infos.append(b.info()["solo_groups"])
        it, act = b.run()
        assert act == 0
        infos.append(b.info()["solo_groups"])
        outs.append([b.lane(u) for u in range(len(lanes))])
        b.close()
    say("solo groups before / after, graph and direct:", infos)
    assert infos[0] > 0 and infos[1] == 0 and infos[2] > 0 and infos[3] == 0
    for u, lane in enumerate(lanes):
        (ra, xa, za, xia), (rb, xb, zb, xib) = outs[0][u], outs[1][u]
        assert ra.iters == rb.iters and np.array_equal(za, zb) and np.array_equal(xa, xb), u
        ref = oracle_lane(ops[lane[0]], lane, s=32, seed=2, beta_mode=O.BETA_RESBAL, max_iter=600,
                          check_every=10, tol=1e-7)
        assert ra.status == racmb.RUN_CONVERGED and ra.iters == ref.iters, (u, ra.iters, ref.iters)
        assert rel(za, ref.z) < 1e-8
    # checkpoint after the move: find a chunk at which the groups have moved and lanes remain
    first = min(r.iters for r, *_ in outs[0])
    last = max(r.iters for r, *_ in outs[0])
    assert first < last
    k = first + 10 if first + 10 < last else first
    c = racmb.Batch(gps, lanes, max_iter=k, use_graph=True, **kw)
    c.run()
    moved = c.info()["solo_groups"] == 0
    blob = c.export_state()
    d = racmb.Batch(gps, lanes, max_iter=600, use_graph=True, **kw)
    d.import_state(blob)
    assert (d.info()["solo_groups"] == 0) == moved
    d.run()
    for u in range(len(lanes)):
        r, x, z, xi = d.lane(u)
        ra, xa, za, xia = outs[0][u]
        assert r.iters == ra.iters and np.array_equal(z, za) and np.array_equal(x, xa), u
    c.close()
    d.close()
