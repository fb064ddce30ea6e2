"""Benchmark of the RAC-MBADMM hot path on one MI355X.

Workload (default): LASSO, D 20000 x 2000 iid N(0,1) with unit-norm columns,
stored in FP32; x_true with 5% non-zeros of magnitude U(1,3); noise 0.05;
lambda = 0.1 lambda_max; blocks of 64 variables (p = 32); synthetic data.

A "step" is one RAC-MBADMM iteration (partition draw, all block Grams and
factors, the Gauss-Seidel sweep, z block, dual step, and every T = 10
iterations the KKT check and the penalty decision) of the candidate solver:
mixed precision (FP32 block Grams on the matrix cores, FP64 everything else)
with the learned penalty controller when trained weights are present, else
residual balancing.  `value` is iterations per second with the data already in
HBM.  The line also reports, on the same data:
  time_to_tol  -- wall time to the first KKT check <= 1e-6 for the candidate
                  and for the plain FP64 fixed-beta solver (FP64 data, FP64
                  Grams, beta = 0.1 lambda as in Sec.3.1),
  roofline     -- the dominant kernel's achieved rate from HIP events recorded
                  around every 8th launch inside the timed region,
  cpu_baseline -- the FP64 oracle on a bounded sample of the same workload,
  batched      -- the batched elastic-net paths (256 instances of uneven size,
                  N in [1000, 20000] and n in [100, 4000] log-uniform, BF16
                  data, 16 lambda lanes each): lane-iterations per second with
                  every lane active, per-launch phase times with the roofline of
                  the batched sweep, and the time until every lane reaches KKT
                  <= 1e-6 for the candidate (mixed precision, learned penalty)
                  and for the plain FP64 fixed-penalty batch on the same values,
  hidim        -- the high-dimensional LASSO, D 10000 x 100000 Gaussian (BF16),
                  1% non-zeros, lambda = 0.05 lambda_max, blocks of 128
                  (p = 782): time to KKT <= 1e-6 for the candidate (mixed
                  precision, learned penalty) and for the plain FP64
                  fixed-penalty solver on the same values (FP64 copy of the
                  data), the latter capped at --hidim-cap iterations.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
MFMA_PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}
METRIC = "time-to-1e-6 KKT residual & ADMM iters/s: learned-β batched vs plain FP64"
TIMING_STRIDE = 8            # sweeps timed with HIP events in the throughput run: iterations k % 8 == 0
WEIGHTS = os.path.join(ROOT, "paper_1907_01995_amd", "controller_weights.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def batched_leg(args, racmb, W, torch, weights, log):
    """Batched elastic-net paths: 256 uneven instances x 16 lambda lanes, BF16 data."""
    t0 = time.time()
    Ns, ns = W.en_batch_sizes(256)
    insts = [W.en_instance_device(int(N), int(n), 1000 + i, storage="bf16") for i, (N, n) in enumerate(zip(Ns, ns))]
    probs = [racmb.regression_problem_tensor(d.F, d.y, lam=0.1 * d.lam_max, alpha=0.5, storage="bf16")
             for d in insts]
    lanes = [(i, racmb.PROX_EN, float(l), 0.5, 0.1 * float(l))
             for i, d in enumerate(insts) for l in W.lambda_grid(d.lam_max, 16, 0.01)]
    torch.cuda.synchronize()
    elems = float(np.sum(Ns.astype(np.float64) * ns))
    log("batched workload generated in %.1fs (%d lanes, %.3e stored values)" % (time.time() - t0, len(lanes), elems))
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    cand = dict(s=64, seed=11, precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights, check_every=10)
    out = {"workload": "en_paths_256x16", "instances": 256, "lanes": len(lanes), "stored_values": elems,
           "data_storage": "bf16", "block_size": 64, "alpha": 0.5, "lambda_grid": "lam_max * 0.01^(j/15), j<16",
           "beta_mode": "mlp" if weights is not None else "residual_balancing"}

    # ---- throughput: every lane active (tol 0), chunks replayed from the hipGraph
    b = racmb.Batch(probs, lanes, max_iter=10, tol=0.0, use_graph=True, tune=True, **cand)
    for _ in range(max(args.batched_warmup // 10, 1)):
        b.run()
    torch.cuda.synchronize()
    a = time.perf_counter()
    k = 0
    for _ in range(max(args.batched_steps // 10, 1)):
        k += b.run()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    info = b.info()
    out.update({"iterations": k, "seconds": dt, "ms_per_iteration": 1e3 * dt / k,
                "lane_iterations_per_s": len(lanes) * k / dt, "team_size": info["team_size"],
                "teams": info["teams"], "graph": info["graph"]})
    log("batched throughput: %d iterations in %.3fs -> %.2f ms/iteration, %.3e lane-iterations/s %s"
        % (k, dt, 1e3 * dt / k, len(lanes) * k / dt, info))
    # ---- per-launch device time (events around every launch) for the roofline
    b.set_timing(True)
    for _ in range(max(args.batched_steps // 20, 1)):
        b.run()
    ph = b.timing()
    b.close()
    del b
    rows = {}
    for name, (ms, cnt) in ph.items():
        if cnt:
            rows[name] = {"avg_us": 1e3 * ms / cnt, "launches": cnt}
    sw = ph["sweep"]
    avg = sw[0] / sw[1] / 1e3
    flops = 4.0 * 16 * elems                       # F_B'u and F_B d, every lane, every block
    nbytes = 2.0 * elems + 16 * 8.0 * (2 * float(np.sum(Ns)) + 6 * float(np.sum(ns)))
    roof = {"bound": "mfma", "achieved": flops / avg / 1e12, "peak": MFMA_PEAK["f64"] / 1e12,
            "unit": "TFLOP/s", "kernel": "k_tsweep" if info["team_size"] else "k_bsweep",
            "avg_launch_us": avg * 1e6, "flops_per_launch": flops, "hbm_bytes_per_launch": nbytes,
            "hbm_GBps": nbytes / avg / 1e9, "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"]
    rows["sweep"]["TFLOPs"] = roof["achieved"]
    out["roofline"] = roof
    out["phases"] = rows
    log("batched phases %s" % rows)

    # ---- time until every lane's KKT <= 1e-6: candidate vs plain FP64 fixed beta
    if not args.no_time_to_tol:
        tt = {}
        plain = dict(s=64, seed=11, precision=racmb.PREC_FP64, beta_mode=racmb.BETA_FIXED, check_every=10)
        for name, kw, cap in (("candidate", cand, args.batched_cap), ("plain_fp64_fixed_beta", plain, 3 * args.batched_cap)):
            bb = racmb.Batch(probs, lanes, max_iter=cap, tol=1e-6, use_graph=True, tune=True, **kw)
            torch.cuda.synchronize()
            a = time.perf_counter()
            it, act = bb.run()
            torch.cuda.synchronize()
            tt[name] = {"seconds": time.perf_counter() - a, "iterations": it, "lanes_converged": len(lanes) - act,
                        "all_converged": act == 0, "iteration_cap": cap}
            got = {u: bb.lane(u) for u in range(0, len(lanes), 97)}
            if name == "candidate":
                zc = got
            else:
                zp = got
            bb.close()
            del bb
            log("batched time-to-tol %s: %s" % (name, tt[name]))
        tt["speedup"] = tt["plain_fp64_fixed_beta"]["seconds"] / tt["candidate"]["seconds"]
        both = [u for u in zc if zc[u][0].status == racmb.RUN_CONVERGED and zp[u][0].status == racmb.RUN_CONVERGED]
        tt["sampled_lanes_converged_in_both"] = len(both)
        tt["candidate_vs_plain_rel_z_sampled"] = float(max(
            (np.max(np.abs(zc[u][2] - zp[u][2])) / max(np.max(np.abs(zp[u][2])), 1e-300) for u in both), default=0.0))
        out["time_to_tol"] = tt
    return out


def hidim_leg(args, racmb, W, torch, weights, log):
    """High-dimensional LASSO 10000 x 100000: time to KKT <= 1e-6, candidate vs plain FP64."""
    t0 = time.time()
    w = W.lasso_10000x100000("bf16")
    log("hidim workload generated in %.1fs" % (time.time() - t0))
    s = w.block_size
    out = {"workload": "lasso_10000x100000", "N": w.N, "n": w.n, "block_size": s, "p": -(-w.n // s),
           "data_storage": "bf16", "lambda": "0.05 lam_max"}
    mode = racmb.BETA_MLP if weights is not None else racmb.BETA_RESBAL
    runs = (("candidate", "bf16", dict(precision=racmb.PREC_MIXED, beta_mode=mode, mlp_weights=weights,
                                        max_iter=5000)),
            ("plain_fp64_fixed_beta", "f64", dict(precision=racmb.PREC_FP64, beta_mode=racmb.BETA_FIXED,
                                                  max_iter=args.hidim_cap)))
    for name, storage, kw in runs:
        D = w.D if storage == "bf16" else w.D.astype(np.float64)
        gp = racmb.regression_problem(D, w.y, lam=w.lam, alpha=1.0, storage=storage)
        del D
        so = racmb.Solver(gp, s=s, beta0=w.beta0, check_every=10, tol=1e-6, **kw)
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = so.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        out[name] = {"seconds": dt, "iters": r.iters, "kkt": r.kkt, "converged": r.status == racmb.RUN_CONVERGED,
                     "objective": r.objective, "ms_per_iteration": 1e3 * dt / max(r.iters, 1),
                     "iteration_cap": kw["max_iter"]}
        so.close()
        del so, gp
        torch.cuda.empty_cache()
        log("hidim time-to-tol %s: %s" % (name, out[name]))
    ratio = out["plain_fp64_fixed_beta"]["seconds"] / out["candidate"]["seconds"]
    out["speedup" if out["plain_fp64_fixed_beta"]["converged"] else "speedup_at_least"] = ratio
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=40)
    ap.add_argument("--batched-warmup", type=int, default=10)
    ap.add_argument("--batched-cap", type=int, default=500)
    ap.add_argument("--no-hidim", action="store_true")
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
    t_gen = time.time()
    w = W.lasso_20000x2000("f32")
    log("workload generated in %.1fs" % (time.time() - t_gen))
    N, n, s = w.N, w.n, w.block_size
    p = -(-n // s)

    prob32 = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f32")
    weights = None
    beta_mode = racmb.BETA_RESBAL
    if os.path.exists(WEIGHTS):
        weights = torch.as_tensor(np.load(WEIGHTS).astype(np.float32), device="cuda")
        beta_mode = racmb.BETA_MLP
    cand_kw = dict(s=s, precision=racmb.PREC_MIXED, beta0=w.beta0, beta_mode=beta_mode,
                   mlp_weights=weights, check_every=10)

    # ---- throughput: K timed iterations after W warm-up iterations ----------
    sol = racmb.Solver(prob32, max_iter=args.steps, tol=0.0, **cand_kw)
    warm = racmb.Solver(prob32, max_iter=max(args.warmup, 1), tol=0.0, **cand_kw)
    if args.warmup > 0:
        warm.run()
    warm.close()
    # HIP events around the sweep launches (the dominant kernel) of every 8th
    # iteration only: the average launch time comes from the timed run itself,
    # and 25 event pairs disturb it far less than events around every launch
    sol.set_timing(True, phases=["sweep"], stride=TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sol.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    sweep_t = sol.timing()["sweep"]
    info = sol.info()
    ips = res.iters / elapsed
    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # every phase, timed in a separate run of the same length
    tim = racmb.Solver(prob32, max_iter=args.steps, tol=0.0, **cand_kw)
    tim.set_timing(True)
    tim.run()
    phases = tim.timing()
    tim.close()
    phases["sweep"] = sweep_t
    log("throughput: %d iterations in %.4fs -> %.1f it/s; phases %s" % (res.iters, elapsed, ips, phases))

    # ---- roofline of the dominant kernel --------------------------------------
    dom = "sweep"
    rows = {}
    for ph, (ms, cnt) in phases.items():
        if cnt == 0:
            continue
        avg = ms / cnt / 1e3
        by, fl = algorithmic(ph, N, n, p, 4)
        rows[ph] = dict(avg_us=avg * 1e6, launches=cnt, GBps=by / avg / 1e9, TFLOPs=fl / avg / 1e12)
    by, fl = algorithmic(dom, N, n, p, 4)
    avg = phases[dom][0] / phases[dom][1] / 1e3
    t_hbm, t_mfma = by / HBM_PEAK, fl / MFMA_PEAK["f32"]
    if dom == "gram" and t_mfma > t_hbm:
        roof = {"bound": "mfma", "achieved": fl / avg / 1e12, "peak": MFMA_PEAK["f32"] / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by / avg / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic("k_sweep2", "lasso_20000x2000")
    roof["kernel"] = {"sweep": "k_sweep2", "gram": "k_gram", "factor": "k_factor_wave",
                      "zdual": "k_zdual", "check": "k_kkt+k_control", "partition": "k_perm_*"}[dom]
    roof["avg_launch_us"] = avg * 1e6

    out = {"metric": METRIC, "value": ips, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / max(res.iters, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "lasso_20000x2000", "N": N, "n": n, "block_size": s, "p": p,
                      "data_storage": "f32", "precision": "mixed (f32 MFMA Gram, f64 rest)",
                      "beta_mode": "mlp" if weights is not None else "residual_balancing",
                      "check_every": 10, "sweep_groups": info["K"], "gram_row_chunks": info["R"]},
           "roofline": roof, "phases": rows}

    # ---- time to KKT <= 1e-6: candidate vs plain FP64 fixed beta ----------------
    if not args.no_time_to_tol:
        tt = {}
        prob64 = racmb.regression_problem(w.D, w.y, lam=w.lam, alpha=1.0, storage="f64")
        cfgs = {"candidate": (prob32, dict(cand_kw, max_iter=5000)),
                "plain_fp64_fixed_beta": (prob64, dict(s=s, precision=racmb.PREC_FP64, beta0=w.beta0,
                                                       beta_mode=racmb.BETA_FIXED, check_every=10,
                                                       max_iter=20000))}
        sols = {}
        for name, (pr, kw) in cfgs.items():
            times = []
            for rep in range(2):
                so = racmb.Solver(pr, tol=1e-6, **kw)
                torch.cuda.synchronize()
                a = time.perf_counter()
                r = so.run()
                torch.cuda.synchronize()
                times.append(time.perf_counter() - a)
                if rep == 1:
                    sols[name] = so.state()
                    tt[name] = {"seconds": min(times), "iters": r.iters, "kkt": r.kkt,
                                "converged": r.status == racmb.RUN_CONVERGED, "objective": r.objective}
                so.close()
            log("time-to-tol %s: %s" % (name, tt[name]))
        zc, zp = sols["candidate"][1], sols["plain_fp64_fixed_beta"][1]
        tt["speedup"] = tt["plain_fp64_fixed_beta"]["seconds"] / tt["candidate"]["seconds"]
        tt["candidate_vs_plain_rel_z"] = float(np.max(np.abs(zc - zp)) / np.max(np.abs(zp)))
        out["time_to_tol"] = tt
        del prob64

    # ---- CPU baseline: the FP64 oracle on a bounded sample ----------------------
    if not args.no_cpu_baseline:
        import oracle as O
        op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
        k = args.cpu_iters
        a = time.perf_counter()
        ro = O.solve(op, s=s, beta0=w.beta0, beta_mode=O.BETA_RESBAL, max_iter=k, check_every=10)
        dt = time.perf_counter() - a
        out["cpu_baseline"] = {"value": ro.iters / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
                               "sample": "%d iterations of lasso_20000x2000 (FP64 oracle, one thread, "
                                         "%.1f s)" % (ro.iters, dt)}
        if "time_to_tol" in out:
            xc = sols["candidate"]
            out["time_to_tol"]["oracle_kkt_of_candidate"] = O.kkt(op, xc[0], xc[1], xc[2], xc[3])
            out["time_to_tol"]["oracle_objective_rel_err"] = abs(
                O.objective(op, xc[1]) - out["time_to_tol"]["candidate"]["objective"]) / abs(
                O.objective(op, xc[1]))
    if not args.no_batched:
        out["batched"] = batched_leg(args, racmb, W, torch, weights, log)
    if not args.no_hidim and not args.no_time_to_tol:
        out["hidim"] = hidim_leg(args, racmb, W, torch, weights, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
