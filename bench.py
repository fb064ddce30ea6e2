"""Benchmark of the RAC-MBADMM hot path on one MI355X.

Headline workload: the batched elastic-net regularisation paths, 256 independent
instances of uneven size (N in [1000, 20000] and n in [100, 4000], log-uniform),
Gaussian data stored in BF16, each solved at 16 points of a log lambda grid
(alpha = 0.5, lambda_j = lambda_max 0.01^(j/15)): 4096 lanes, blocks of 64.
Synthetic data, generated on the device with seeded generators.

A "step" is one RAC-MBADMM iteration (Eq.(3)) of every lane of the batch: the
instances' partition draws, the shared block Grams, the lanes' block inverses,
the Gauss-Seidel sweeps, the z blocks and dual steps, and every T = 10
iterations the KKT check and the penalty decision.  The candidate is the mixed
precision solver (BF16 block Grams on the matrix cores, FP64 everything else)
with the learned penalty controller, chunks of T iterations replayed from a
hipGraph.  `value` is lane-iterations per second with every lane active and the
data already in HBM.  The line also reports:
  time_to_tol  -- wall time until every lane is at KKT <= 1e-6, for the
                  candidate and for the plain FP64 fixed-penalty batch on the
                  same stored values (beta = 0.1 lambda_j, Sec.3.1);
  roofline     -- the batched sweep k_tsweep (FP64 matrix cores): its
                  algorithmic flops over its average launch time, from HIP
                  events around every launch of a timing run of the same length;
  cpu_baseline -- the FP64 oracle on sampled lanes of the same workload, the
                  lanes run in parallel threads (one lane per thread);
  legs         -- the single-instance workloads: least squares 2000x200 (FP64),
                  LASSO 20000x2000 (FP32), the linear SVM dual 20000x256 (FP32)
                  and the high-dimensional LASSO 10000x100000 (BF16), each with
                  its own throughput, sweep roofline and time to tolerance; the
                  two LASSO legs also time RP-MBADMM (fixed blocks, random
                  order; Sec.1) to the same tolerance; the dense form: the
                  Gaussian-kernel SVM dual 20000x128 (kernel matrix, the
                  paper's 10-iteration budget, held-out accuracy) and a general
                  QP 8192x8192 with 8 equality rows; sparse elastic nets in
                  compressed sparse columns shaped like E2006-tfidf (16087 x
                  150360, 0.9% dense) and the paper's synthetic 40000 x
                  4000000 (0.2% dense), 10 iterations each as in the paper;
                  and the batched workload's paths solved stage by stage,
                  warm-started against cold.
A ratio between two solvers is "speedup" when both reached the tolerance,
"speedup_at_least" when only the candidate did (the other stopped at its
iteration cap), and absent when the candidate did not.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
MFMA_PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}
METRIC = "time-to-1e-6 KKT residual & ADMM iters/s: learned-β batched vs plain FP64"
TIMING_STRIDE = 8            # sweeps timed with HIP events in a throughput run: iterations k % 8 == 0
WEIGHTS = os.path.join(ROOT, "paper_1907_01995_amd", "controller_weights.npy")
T_CHECK = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ratio(cand, plain, key="seconds"):
    """Speedup of cand over plain under the convergence rule stated above."""
    if not cand.get("converged"):
        return {"speedup_note": "candidate did not reach the tolerance: no ratio"}
    r = plain[key] / cand[key]
    return {"speedup": r} if plain.get("converged") else {"speedup_at_least": r}


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_threads():
    """Worker threads for the oracle baseline: the host's share for one GPU (at most 16)."""
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(16, n, os.cpu_count() or 1))


def algorithmic(phase, N, n, p, bA):
    """Algorithmic bytes and flops of one launch of a phase (one read of the data)."""
    sizes = np.diff((np.arange(p + 1) * n) // p)
    if phase == "sweep":
        return N * n * bA + 6 * n * 8, 4.0 * N * n
    if phase == "gram":
        return N * n * bA, float(np.sum(N * sizes * (sizes + 1)))
    if phase == "factor":
        return float(np.sum(sizes * sizes * 8)), float(np.sum(sizes ** 3))
    if phase == "check":
        return N * n * bA + 8 * n * 8, 2.0 * N * n
    return 0.0, 0.0


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE counters of the
    kernel (scaled by a plain copy of known size), or None when the kernel's sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    from paper_1907_01995_amd import profsum
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != profsum.source_hash(kernel):
        return None
    return rec["traffic_bytes_per_launch"]


def calibration_copy(torch):
    """Plain 256 MiB device copies (counter calibration for rocprofv3 --pmc runs)."""
    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


# ---------------------------------------------------------------------------
# Headline: batched elastic-net paths

def batched_workload(racmb, W, torch):
    Ns, ns = W.en_batch_sizes(256)
    insts = [W.en_instance_device(int(N), int(n), 1000 + i, storage="bf16") for i, (N, n) in enumerate(zip(Ns, ns))]
    probs = [racmb.regression_problem_tensor(d.F, d.y, lam=0.1 * d.lam_max, alpha=0.5, storage="bf16")
             for d in insts]
    lanes = [(i, racmb.PROX_EN, float(l), 0.5, 0.1 * float(l))
             for i, d in enumerate(insts) for l in W.lambda_grid(d.lam_max, 16, 0.01)]
    torch.cuda.synchronize()
    return Ns, ns, insts, probs, lanes


def batched_headline(args, racmb, W, torch, weights):
    t0 = time.time()
    Ns, ns, insts, probs, lanes = batched_workload(racmb, W, torch)
    elems = float(np.sum(Ns.astype(np.float64) * ns))
    log("batched workload generated in %.1fs (%d lanes, %.3e stored values)" % (time.time() - t0, len(lanes), elems))
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    cand = dict(s=64, seed=11, precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights,
                check_every=T_CHECK)
    cfg = {"workload": "en_paths_256x16", "instances": 256, "lanes": len(lanes), "stored_values": elems,
           "N_range": [int(Ns.min()), int(Ns.max())], "n_range": [int(ns.min()), int(ns.max())],
           "data_storage": "bf16", "block_size": 64, "alpha": 0.5,
           "lambda_grid": "lam_max * 0.01^(j/15), j<16", "precision": "mixed (bf16 MFMA Gram, f64 rest)",
           "beta_mode": "mlp" if weights is not None else "residual_balancing", "check_every": T_CHECK}

    # ---- throughput: every lane active (tol 0).  One batch object runs chunks of T
    # iterations, each replayed from the hipGraph captured on its first run; the warm-up
    # chunks (at least one) capture the graph and fill the tuning cache, and the timed
    # region is the next ceil(K/T) chunks (K rounded up to whole chunks, reported as steps).
    warm_chunks = max(1, -(-args.warmup // T_CHECK))
    timed_chunks = max(1, -(-args.steps // T_CHECK))
    b = racmb.Batch(probs, lanes, max_iter=T_CHECK, tol=0.0, use_graph=True, tune=True, **cand)
    for _ in range(warm_chunks):
        b.run()
    torch.cuda.synchronize()
    a = time.perf_counter()
    k = 0
    for _ in range(timed_chunks):
        k += b.run()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    info = b.info()
    b.close()
    del b
    warm_iters = warm_chunks * T_CHECK
    log("batched throughput: %d iterations in %.3fs -> %.2f ms/iteration, %.3e lane-iterations/s %s"
        % (k, dt, 1e3 * dt / k, len(lanes) * k / dt, info))
    cfg.update({"team_size_max": info["team_size"], "teams": info["teams"], "graph": info["graph"]})

    # ---- per-launch device time (events around every launch) of a run of the same length
    bt = racmb.Batch(probs, lanes, max_iter=int(k), tol=0.0, use_graph=True, tune=True, **cand)
    bt.set_timing(True)
    bt.run()
    ph = bt.timing()
    bt.close()
    del bt
    # per launch, and per iteration (the Grams and inverses of a chunk may be one launch)
    rows = {name: {"avg_us": 1e3 * ms / cnt, "launches": cnt, "us_per_iteration": 1e3 * ms / k}
            for name, (ms, cnt) in ph.items() if cnt}
    sw = ph["sweep"]
    avg = sw[0] / sw[1] / 1e3
    flops = 4.0 * 16 * elems                       # F_B'u and F_B d, every lane, every block
    # one read of F (BF16), of every lane's block inverses (the ten stored lower 16 x 16
    # FP64 tiles of a 64 x 64 block) and of the lane vectors, and one write of u and x
    nblk = float(np.sum(-(-ns // 64)))
    nbytes = 2.0 * elems + 16 * nblk * 10 * 256 * 8.0 + 16 * 8.0 * (2 * float(np.sum(Ns)) + 6 * float(np.sum(ns)))
    kern = "k_tsweep" if info["team_size"] else "k_bsweep"
    roof = {"bound": "mfma", "achieved": flops / avg / 1e12, "peak": MFMA_PEAK["f64"] / 1e12,
            "unit": "TFLOP/s", "kernel": kern, "avg_launch_us": avg * 1e6, "flops_per_launch": flops,
            "hbm_bytes_per_launch": nbytes, "hbm_GBps": nbytes / avg / 1e9,
            "traffic": measured_traffic(kern, "en_paths_256x16")}
    roof["frac"] = roof["achieved"] / roof["peak"]
    rows["sweep"]["TFLOPs"] = roof["achieved"]
    log("batched phases %s" % rows)

    out = {"metric": METRIC, "value": len(lanes) * k / dt, "unit": "lane-iters/s", "n_gpus": 1,
           "steps": int(k), "warmup": warm_iters, "ms_per_step": 1e3 * dt / k, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic", "config": cfg,
           "roofline": roof, "phases": rows}

    # ---- time until every lane's KKT <= 1e-6: candidate vs plain FP64 fixed beta
    if not args.no_time_to_tol:
        tt = {}
        plain = dict(s=64, seed=11, precision=racmb.PREC_FP64, beta_mode=racmb.BETA_FIXED, check_every=T_CHECK)
        got = {}
        for name, kw, cap in (("candidate", cand, args.batched_cap),
                              ("plain_fp64_fixed_beta", plain, args.batched_plain_cap)):
            bb = racmb.Batch(probs, lanes, max_iter=cap, tol=1e-6, use_graph=True, tune=True, **kw)
            torch.cuda.synchronize()
            a = time.perf_counter()
            it, act = bb.run()
            torch.cuda.synchronize()
            tt[name] = {"seconds": time.perf_counter() - a, "iterations": it, "lanes_converged": len(lanes) - act,
                        "converged": act == 0, "iteration_cap": cap}
            got[name] = {u: bb.lane(u) for u in range(0, len(lanes), 97)}
            bb.close()
            del bb
            log("batched time-to-tol %s: %s" % (name, tt[name]))
        tt.update(ratio(tt["candidate"], tt["plain_fp64_fixed_beta"]))
        zc, zp = got["candidate"], got["plain_fp64_fixed_beta"]
        both = [u for u in zc if zc[u][0].status == racmb.RUN_CONVERGED and zp[u][0].status == racmb.RUN_CONVERGED]
        tt["sampled_lanes_converged_in_both"] = len(both)
        tt["candidate_vs_plain_rel_z_sampled"] = float(max(
            (np.max(np.abs(zc[u][2] - zp[u][2])) / max(np.max(np.abs(zp[u][2])), 1e-300) for u in both), default=0.0))
        out["time_to_tol"] = tt

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batched_cpu_baseline(args, Ns, ns, insts, lanes)
    del probs, insts
    torch.cuda.empty_cache()
    return out


def batched_cpu_baseline(args, Ns, ns, insts, lanes):
    """The FP64 oracle on a stratified sample of the batch's lanes, one lane per thread.

    The instances are ordered by stored values N_i n_i and every (256/S)-th is taken,
    one lane (the middle lambda of its grid) each; every sampled lane runs
    `cpu_iters` iterations from a cold start.  The rate is the sample's
    lane-iterations per wall second, scaled by the ratio of the sample's mean
    stored values per lane to the whole workload's (the oracle's cost per
    iteration is proportional to N_i n_i for a fixed block size)."""
    import oracle as O
    sizes = Ns.astype(np.float64) * ns
    order = np.argsort(sizes, kind="stable")
    S = args.cpu_lanes
    pick = [int(order[int((q + 0.5) * len(order) / S)]) for q in range(S)]
    jobs = []
    for i in pick:
        u = 16 * i + 8
        _, _, lam, alpha, beta0 = lanes[u]
        D = insts[i].host_D()
        jobs.append((O.en_problem(D, insts[i].y, lam=lam, alpha=alpha), beta0, i))
    threads = cpu_threads()

    def one(job):
        P, beta0, inst = job
        return O.solve(P, s=64, seed=11, inst=inst, beta0=beta0, beta_mode=O.BETA_FIXED, max_iter=args.cpu_iters,
                       check_every=T_CHECK).iters

    a = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        its = list(ex.map(one, jobs))
    wall = time.perf_counter() - a
    scale = float(np.mean(sizes[pick]) / np.mean(sizes))
    model, nproc = cpu_info()
    rate = sum(its) / wall * scale
    log("cpu baseline: %d lanes x %d iterations in %.1fs on %d threads (size scale %.3f) -> %.3g lane-iters/s"
        % (S, args.cpu_iters, wall, threads, scale, rate))
    return {"value": rate, "unit": "lane-iters/s", "cores": threads, "kind": "oracle",
            "sample": "%d lanes (one per instance, instances stratified by N_i n_i, middle lambda), %d iterations "
                      "each from a cold start, FP64 oracle, one lane per thread; %.1f s wall; rate scaled by the "
                      "sample's mean stored values per lane over the workload's (%.3f)"
                      % (S, args.cpu_iters, wall, scale),
            "host_nproc": nproc, "cpu_model": model}


# ---------------------------------------------------------------------------
# Single-instance legs

def sweep_roofline(phases, N, n, p, bA, kernel, workload):
    ms, cnt = phases["sweep"]
    avg = ms / cnt / 1e3
    by, _ = algorithmic("sweep", N, n, p, bA)
    roof = {"bound": "hbm", "achieved": by / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "kernel": kernel, "avg_launch_us": avg * 1e6, "bytes_per_launch": by,
            "traffic": measured_traffic(kernel, workload)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    return roof


def phase_rows(phases, N, n, p, bA):
    rows = {}
    for ph, (ms, cnt) in phases.items():
        if cnt == 0:
            continue
        avg = ms / cnt / 1e3
        by, fl = algorithmic(ph, N, n, p, bA)
        rows[ph] = dict(avg_us=avg * 1e6, launches=cnt, GBps=by / avg / 1e9, TFLOPs=fl / avg / 1e12)
    return rows


def throughput(racmb, torch, prob, iters, warmup, kw):
    """Iterations per second over `iters` iterations (sweeps of every 8th iteration
    timed with HIP events), and the phase table of a separate run of the same length."""
    if warmup > 0:
        w = racmb.Solver(prob, max_iter=warmup, tol=0.0, **kw)
        w.run()
        w.close()
    sol = racmb.Solver(prob, max_iter=iters, tol=0.0, **kw)
    sol.set_timing(True, phases=["sweep"], stride=TIMING_STRIDE)
    torch.cuda.synchronize()
    a = time.perf_counter()
    res = sol.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    sweep_t = sol.timing()["sweep"]
    info = sol.info()
    sol.close()
    tim = racmb.Solver(prob, max_iter=iters, tol=0.0, **kw)
    tim.set_timing(True)
    tim.run()
    phases = tim.timing()
    tim.close()
    phases["sweep"] = sweep_t
    return res.iters / dt, 1e3 * dt / max(res.iters, 1), phases, info


def time_to_tol(racmb, torch, prob, kw, reps=2):
    best, st = None, None
    for rep in range(reps):
        so = racmb.Solver(prob, tol=1e-6, **kw)
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = so.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        best = dt if best is None else min(best, dt)
        if rep == reps - 1:
            st = so.state()
            rec = {"seconds": best, "iters": r.iters, "kkt": r.kkt, "converged": r.status == racmb.RUN_CONVERGED,
                   "objective": r.objective, "iteration_cap": kw["max_iter"]}
        so.close()
    return rec, st


def lasso_leg(args, racmb, W, torch, weights):
    """LASSO 20000 x 2000 (FP32, blocks of 64): iterations/s, sweep roofline, time to KKT <= 1e-6."""
    import oracle as O
    w = W.lasso_20000x2000("f32")
    N, n, s = w.N, w.n, w.block_size
    p = -(-n // s)
    prob32 = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f32")
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    kw = dict(s=s, precision=racmb.PREC_MIXED, beta0=w.beta0, beta_mode=mode, mlp_weights=weights,
              check_every=T_CHECK)
    ips, ms, phases, info = throughput(racmb, torch, prob32, args.single_steps, 20, kw)
    if args.calibrate_copy:
        calibration_copy(torch)
    out = {"workload": "lasso_20000x2000", "N": N, "n": n, "block_size": s, "p": p, "data_storage": "f32",
           "precision": "mixed (f32 MFMA Gram, f64 rest)", "beta_mode": "mlp" if weights is not None else
           "residual_balancing", "iters_per_s": ips, "ms_per_iteration": ms, "sweep_groups": info["K"],
           "roofline": sweep_roofline(phases, N, n, p, 4, "k_sweep2", "lasso_20000x2000"),
           "phases": phase_rows(phases, N, n, p, 4)}
    log("lasso_20000x2000: %.1f it/s, sweep %.1f us" % (ips, out["roofline"]["avg_launch_us"]))
    if not args.no_time_to_tol:
        prob64 = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f64")
        cand, stc = time_to_tol(racmb, torch, prob32, dict(kw, max_iter=5000))
        plain, stp = time_to_tol(racmb, torch, prob64, dict(s=s, precision=racmb.PREC_FP64, beta0=w.beta0,
                                                            beta_mode=racmb.BETA_FIXED, check_every=T_CHECK,
                                                            max_iter=20000))
        rp, _ = time_to_tol(racmb, torch, prob32, dict(kw, max_iter=5000, variant=racmb.VARIANT_RP))
        tt = {"candidate": cand, "plain_fp64_fixed_beta": plain, "rp_candidate": rp}
        tt.update(ratio(cand, plain))
        tt["rac_over_rp"] = ratio(cand, rp)
        tt["candidate_vs_plain_rel_z"] = float(np.max(np.abs(stc[1] - stp[1])) / np.max(np.abs(stp[1])))
        op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
        tt["oracle_kkt_of_candidate_iterate"] = O.kkt(op, stc[0], stc[1], stc[2], stc[3])
        tt["oracle_objective_of_candidate_z_vs_reported_rel"] = abs(O.objective(op, stc[1]) - cand["objective"]) / \
            abs(O.objective(op, stc[1]))
        out["time_to_tol"] = tt
        log("lasso_20000x2000 time-to-tol %s" % tt)
        del prob64
    del prob32
    return out


def ols_leg(args, racmb, W, torch):
    """Least squares 2000 x 200 (FP64, p = 10, beta = 1, 300 iterations, seed 0), against the
    oracle's 300 iterations (one thread) and the normal equations."""
    import oracle as O
    w = W.ols_2000x200()
    prob = racmb.regression_problem(w.D, w.y, storage="f64")
    kw = dict(s=w.block_size, precision=racmb.PREC_FP64, beta0=1.0, beta_mode=racmb.BETA_FIXED,
              check_every=T_CHECK, seed=0)
    ips, ms, phases, info = throughput(racmb, torch, prob, 300, 10, kw)
    so = racmb.Solver(prob, max_iter=300, tol=0.0, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    r = so.run()
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - a
    z = so.state()[1]
    so.close()
    op = O.en_problem(w.D, w.y)
    a = time.perf_counter()
    ro = O.solve(op, s=w.block_size, seed=0, beta0=1.0, max_iter=300, check_every=T_CHECK)
    cpu_s = time.perf_counter() - a
    ls = np.linalg.lstsq(w.D, w.y, rcond=None)[0]
    out = {"workload": "ols_2000x200", "N": 2000, "n": 200, "p": 10, "data_storage": "f64", "precision": "fp64",
           "iters_per_s": ips, "ms_per_iteration": ms, "seconds_300_iterations": gpu_s, "kkt": r.kkt,
           "roofline": sweep_roofline(phases, 2000, 200, 10, 8, "k_sweep2", "ols_2000x200"),
           "oracle_seconds_300_iterations": cpu_s, "oracle_threads": 1,
           "rel_z_vs_oracle": float(np.max(np.abs(z - ro.z)) / np.max(np.abs(ro.z))),
           "rel_z_vs_normal_equations": float(np.max(np.abs(z - ls)) / np.max(np.abs(ls)))}
    log("ols_2000x200: %s" % out)
    return out


def svm_leg(args, racmb, W, torch):
    """Linear SVM dual 20000 x 256 (FP32, blocks of 128, beta = 0.1 p): iterations/s, sweep
    roofline, and the KKT residual reached within a fixed iteration budget."""
    import oracle as O
    w = W.svm_20000x256()
    n, r, s = w.n, w.r, w.block_size
    p = -(-n // s)
    prob = racmb.svm_problem(w.X, w.labels, w.C, storage="f32")
    kw = dict(s=s, precision=racmb.PREC_MIXED, beta0=w.beta0, beta_mode=racmb.BETA_FIXED, check_every=T_CHECK)
    ips, ms, phases, info = throughput(racmb, torch, prob, args.single_steps, 10, kw)
    so = racmb.Solver(prob, max_iter=args.svm_budget, tol=1e-6, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    res = so.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    x, z, xi, mu, _, _ = so.state()
    so.close()
    op = O.svm_problem(w.X.astype(np.float64), w.labels, w.C)
    out = {"workload": "svm_20000x256", "n": n, "r": r, "block_size": s, "p": p, "data_storage": "f32",
           "precision": "mixed (f32 MFMA Gram, f64 rest)", "beta": w.beta0, "beta_mode": "fixed (0.1 p)",
           "iters_per_s": ips, "ms_per_iteration": ms,
           "roofline": sweep_roofline(phases, r, n, p, 4, "k_sweep2", "svm_20000x256"),
           "phases": phase_rows(phases, r, n, p, 4),
           "budget": {"iterations": res.iters, "seconds": dt, "kkt": res.kkt,
                      "converged": res.status == racmb.RUN_CONVERGED, "objective": res.objective,
                      "oracle_kkt_of_iterate": O.kkt(op, x, z, xi, mu),
                      "oracle_objective_of_z": O.objective(op, z)}}
    log("svm_20000x256: %s" % out)
    return out


def hidim_leg(args, racmb, W, torch, weights):
    """High-dimensional LASSO 10000 x 100000: time to KKT <= 1e-6, candidate vs plain FP64, and the
    candidate's iteration rate with the sweep's roofline (every 8th sweep timed) over 20 iterations."""
    t0 = time.time()
    w = W.lasso_10000x100000("bf16")
    log("hidim workload generated in %.1fs" % (time.time() - t0))
    s = w.block_size
    out = {"workload": "lasso_10000x100000", "N": w.N, "n": w.n, "block_size": s, "p": -(-w.n // s),
           "data_storage": "bf16", "lambda": "0.05 lam_max"}
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    runs = (("candidate", "bf16", dict(precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights,
                                        max_iter=5000)),
            ("rp_candidate", "bf16", dict(precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights,
                                          max_iter=5000, variant=racmb.VARIANT_RP)),
            ("plain_fp64_fixed_beta", "f64", dict(precision=racmb.PREC_FP64, beta_mode=racmb.BETA_FIXED,
                                                  max_iter=args.hidim_cap)))
    for name, storage, kw in runs:
        D = w.D if storage == "bf16" else w.D.astype(np.float64)
        gp = racmb.regression_problem(D, w.y, lam=w.lam, alpha=1.0, storage=storage)
        del D
        so = racmb.Solver(gp, s=s, beta0=w.beta0, check_every=T_CHECK, tol=1e-6, **kw)
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = so.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        out[name] = {"seconds": dt, "iters": r.iters, "kkt": r.kkt, "converged": r.status == racmb.RUN_CONVERGED,
                     "objective": r.objective, "ms_per_iteration": 1e3 * dt / max(r.iters, 1),
                     "iteration_cap": kw["max_iter"]}
        so.close()
        if name == "candidate":
            # the candidate's iteration rate and sweep roofline from a short fixed-length run
            tkw = {k: v for k, v in kw.items() if k != "max_iter"}
            tkw.update(s=s, beta0=w.beta0, check_every=T_CHECK)
            ips, msit, phases, _ = throughput(racmb, torch, gp, 20, 2, tkw)
            out.update(iters_per_s=ips, ms_per_iteration=msit,
                       roofline=sweep_roofline(phases, w.N, w.n, out["p"], 2, "k_sweep2", "lasso_10000x100000"),
                       phases=phase_rows(phases, w.N, w.n, out["p"], 2))
            log("hidim throughput: %.1f it/s, sweep %.1f us" % (ips, out["roofline"]["avg_launch_us"]))
        del so, gp
        torch.cuda.empty_cache()
        log("hidim time-to-tol %s: %s" % (name, out[name]))
    out.update(ratio(out["candidate"], out["plain_fp64_fixed_beta"]))
    out["rac_over_rp"] = ratio(out["candidate"], out["rp_candidate"])
    return out


def svm_rbf_leg(args, racmb, W, torch):
    """Gaussian-kernel C-SVC dual (Sec.3.2, Eq.(9)), 20000 training points x 128 features: the kernel
    matrix on the device, the paper's budget of 10 iterations (beta = 0.1 p), iterations/s with the
    dense sweep's roofline (one read of the n x n FP64 Hessian per sweep), the KKT residual after a
    fixed budget, the bias b = -mu and the held-out accuracy of the decision function."""
    X, y, Xt, yt, Cbox, gamma = W.svm_rbf(20000, 128, 5000)
    n, s = X.shape[0], 64
    p = -(-n // s)
    torch.cuda.synchronize()
    a = time.perf_counter()
    prob, Xd, yd = racmb.svm_kernel_problem(X, y, Cbox, gamma)
    torch.cuda.synchronize()
    t_kernel = time.perf_counter() - a
    kw = dict(s=s, beta0=0.1 * p, beta_mode=racmb.BETA_FIXED, check_every=T_CHECK)
    ips, ms, phases, info = throughput(racmb, torch, prob, args.dense_steps, 5, kw)
    so = racmb.Solver(prob, max_iter=10, tol=0.0, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    r10 = so.run()
    torch.cuda.synchronize()
    t10 = time.perf_counter() - a
    so.close()
    sb = racmb.Solver(prob, max_iter=args.svm_budget, tol=1e-6, **kw)
    a = time.perf_counter()
    rb = sb.run()
    torch.cuda.synchronize()
    tb = time.perf_counter() - a
    z = sb.state()[1]
    bias = -float(sb.multipliers()[0])
    sb.close()
    _, acc = racmb.svm_decision(Xd, yd, z, gamma, bias, Xt, labels=yt)
    _, acc_train = racmb.svm_decision(Xd, yd, z, gamma, bias, X, labels=y)
    avg = phases["sweep"][0] / phases["sweep"][1] / 1e3
    nbytes = float(n) * n * 8 + 6.0 * n * 8
    roof = {"bound": "hbm", "achieved": nbytes / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "kernel": "k_sweep2 (dense form)", "avg_launch_us": avg * 1e6, "bytes_per_launch": nbytes}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {"workload": "svm_rbf_20000x128", "n": n, "r": 128, "gamma": gamma, "C": Cbox, "block_size": s, "p": p,
           "kernel_matrix_seconds": t_kernel, "iters_per_s": ips, "ms_per_iteration": ms, "sweep_groups": info["K"],
           "roofline": roof, "phases": {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in phases.items()
                                         if v[1]},
           "paper_budget_10_iterations": {"seconds": t10, "kkt": r10.kkt},
           "budget": {"iterations": rb.iters, "seconds": tb, "kkt": rb.kkt,
                      "converged": rb.status == racmb.RUN_CONVERGED},
           "bias": bias, "test_accuracy": acc, "train_accuracy": acc_train}
    del prob, Xd, yd
    torch.cuda.empty_cache()
    log("svm_rbf_20000x128: %s" % out)
    return out


def dense_qp_leg(args, racmb, W, torch):
    """General QP of Eq.(1) with 8 equality rows (Eq.(4)) and the box [0, 1], dense 8192 x 8192
    Hessian: iterations/s with the dense sweep's roofline, and time to KKT <= 1e-6, RAC and RP."""
    n, meq, s = 8192, 8, 64
    H, c, A, beq = W.dense_qp_device(n, meq)
    prob = racmb.dense_problem(H, c, A=A, beq=beq, prox=racmb.PROX_BOX, lo=0.0, hi=1.0)
    kw = dict(s=s, beta0=1.0, beta_mode=racmb.BETA_RESBAL, check_every=T_CHECK)
    ips, ms, phases, info = throughput(racmb, torch, prob, args.dense_steps, 5, kw)
    avg = phases["sweep"][0] / phases["sweep"][1] / 1e3
    nbytes = float(n) * n * 8 + 6.0 * n * 8
    roof = {"bound": "hbm", "achieved": nbytes / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "kernel": "k_sweep2 (dense form)", "avg_launch_us": avg * 1e6, "bytes_per_launch": nbytes}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {"workload": "qp_dense_8192_eq8_box", "n": n, "meq": meq, "block_size": s, "iters_per_s": ips,
           "ms_per_iteration": ms, "sweep_groups": info["K"], "roofline": roof,
           "phases": {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in phases.items() if v[1]}}
    if not args.no_time_to_tol:
        rac, _ = time_to_tol(racmb, torch, prob, dict(kw, max_iter=5000), reps=1)
        rp, _ = time_to_tol(racmb, torch, prob, dict(kw, max_iter=5000, variant=racmb.VARIANT_RP), reps=1)
        out["time_to_tol"] = {"rac": rac, "rp": rp, "rac_over_rp": ratio(rac, rp)}
    del prob, H, A
    torch.cuda.empty_cache()
    log("qp_dense_8192_eq8: %s" % out)
    return out


def path_leg(args, racmb, W, torch, weights):
    """Warm-started regularisation paths (Sec.3.1): the first 64 instances of the batched workload,
    each path of 8 decreasing lambdas (lam_max .. 0.01 lam_max) solved stage by stage with every lane
    started from the previous stage's solution, against the same 8 stages started cold (mixed
    precision, BF16 data); total iterations and seconds to KKT <= 1e-6 at every point."""
    Ns, ns, insts, probs, lanes = batched_workload(racmb, W, torch)
    insts, probs = insts[:64], probs[:64]
    lams = [W.lambda_grid(d.lam_max, 8, 0.01) for d in insts]
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    kw = dict(alpha=0.5, s=64, seed=11, precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights,
              check_every=T_CHECK, max_iter=args.batched_cap, tol=1e-6, use_graph=True, tune=True)
    out = {"workload": "en_paths (first 64 instances) as 8 sequential stages of 64 lanes"}
    for name, warm in (("warm", True), ("cold", False)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        stages, iters = racmb.solve_path(probs, lams, warm=warm, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        conv = sum(1 for st in stages for r in st if r[0].status == racmb.RUN_CONVERGED)
        out[name] = {"seconds": dt, "stage_iterations": iters, "total_iterations": int(sum(iters)),
                     "points_converged": conv, "points": 8 * len(probs)}
        log("path %s: %s" % (name, out[name]))
    del probs, insts
    torch.cuda.empty_cache()
    return out


def sparse_leg(args, racmb, W, torch, name, N, n, density, s, tol_run):
    """Sparse elastic net (Sec.3.1, Tables 3-7 shapes), data in compressed sparse columns (FP32
    values): the paper's budget of 10 iterations, iterations/s, the one-workgroup sweep's time per
    launch against one read of the stored entries, and (tol_run) the time to KKT <= 1e-6."""
    t0 = time.time()
    colptr, rowidx, values, y, lam = W.sparse_regression_device(N, n, density)
    prob = racmb.sparse_regression_problem(colptr, rowidx, values, y, N, lam=lam, alpha=0.5, storage="f32")
    torch.cuda.synchronize()
    nnz = int(rowidx.numel())
    log("%s generated in %.1fs (%d stored entries)" % (name, time.time() - t0, nnz))
    kw = dict(s=s, beta0=0.1 * lam, beta_mode=racmb.BETA_RESBAL, check_every=T_CHECK)
    so = racmb.Solver(prob, max_iter=10, tol=0.0, **kw)
    so.set_timing(True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    r10 = so.run()
    torch.cuda.synchronize()
    t10 = time.perf_counter() - a
    ph = so.timing()
    so.close()
    avg = ph["sweep"][0] / ph["sweep"][1] / 1e3
    nbytes = nnz * 8.0 + 6.0 * n * 8
    roof = {"bound": "hbm", "achieved": nbytes / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "kernel": "k_ssweep_lds" if N <= 17408 else "k_ssweep", "avg_launch_us": avg * 1e6, "bytes_per_launch": nbytes,
            "blocks_per_launch": -(-n // s), "us_per_block": avg * 1e6 / -(-n // s)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {"workload": name, "N": N, "n": n, "density": density, "nnz": nnz, "block_size": s,
           "lambda": "0.1 lam_max", "alpha": 0.5, "values": "f32",
           "paper_budget_10_iterations": {"seconds": t10, "kkt": r10.kkt, "seconds_per_iteration": t10 / 10},
           "roofline": roof,
           "phases": {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in ph.items() if v[1]}}
    if tol_run and not args.no_time_to_tol:
        for variant, key in ((racmb.VARIANT_RAC, "rac"), (racmb.VARIANT_RP, "rp")):
            rec, _ = time_to_tol(racmb, torch, prob, dict(kw, max_iter=1000, variant=variant), reps=1)
            out.setdefault("time_to_tol", {})[key] = rec
        out["time_to_tol"]["rac_over_rp"] = ratio(out["time_to_tol"]["rac"], out["time_to_tol"]["rp"])
    del prob, colptr, rowidx, values, y
    torch.cuda.empty_cache()
    log("%s: %s" % (name, out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed iterations of the batched headline")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--cpu-lanes", type=int, default=32, help="sampled lanes of the oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations per sampled lane")
    ap.add_argument("--batched-cap", type=int, default=500)
    ap.add_argument("--batched-plain-cap", type=int, default=1500)
    ap.add_argument("--single-steps", type=int, default=200, help="timed iterations of each single-instance leg")
    ap.add_argument("--svm-budget", type=int, default=1000)
    ap.add_argument("--no-legs", action="store_true", help="headline only")
    ap.add_argument("--legs", default="ols,lasso,svm,hidim,svm_rbf,qp,path,sparse,sparse_big")
    ap.add_argument("--dense-steps", type=int, default=50, help="timed iterations of the dense-form legs")
    ap.add_argument("--hidim-cap", type=int, default=1500,
                    help="iteration cap of the plain FP64 solver in the high-dimensional leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="add plain 256 MiB device copies (counter calibration for rocprofv3 --pmc runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported (a single instance "
              "would shard by rows of F, batches by instance, neither is implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_01995_amd import racmb, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    weights = None
    if os.path.exists(WEIGHTS):
        weights = torch.as_tensor(np.load(WEIGHTS).astype(np.float32), device="cuda")

    out = batched_headline(args, racmb, W, torch, weights)
    if args.calibrate_copy:
        calibration_copy(torch)
    legs = {}
    want = set() if args.no_legs else set(args.legs.split(","))
    if "ols" in want:
        legs["ols_2000x200"] = ols_leg(args, racmb, W, torch)
    if "lasso" in want:
        legs["lasso_20000x2000"] = lasso_leg(args, racmb, W, torch, weights)
    if "svm" in want:
        legs["svm_20000x256"] = svm_leg(args, racmb, W, torch)
    if "hidim" in want and not args.no_time_to_tol:
        legs["lasso_10000x100000"] = hidim_leg(args, racmb, W, torch, weights)
    if "svm_rbf" in want:
        legs["svm_rbf_20000x128"] = svm_rbf_leg(args, racmb, W, torch)
    if "qp" in want:
        legs["qp_dense_8192_eq8_box"] = dense_qp_leg(args, racmb, W, torch)
    if "sparse" in want:
        legs["sparse_en_16087x150360"] = sparse_leg(args, racmb, W, torch, "sparse_en_16087x150360", 16087, 150360,
                                                    0.009, 64, True)
    if "sparse_big" in want:
        legs["sparse_en_40000x4000000"] = sparse_leg(args, racmb, W, torch, "sparse_en_40000x4000000", 40000,
                                                     4000000, 0.002, 100, False)
    if "path" in want and not args.no_time_to_tol:
        legs["en_paths_warm_vs_cold"] = path_leg(args, racmb, W, torch, weights)
    if legs:
        out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
