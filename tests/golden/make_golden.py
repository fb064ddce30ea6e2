"""Writes the converged oracle solutions that the full-size GPU tests compare with.

    python tests/golden/make_golden.py lasso [DIR]      # lasso_20000x2000, host only
    python tests/golden/make_golden.py en_paths [DIR]   # sampled lanes of the 256 x 16 batch

(files go to DIR, by default this folder)

Only the oracle computes here.  The inputs come from the seeded generators in
paper_1907_01995_amd/workloads.py; the batched instances are drawn by torch's seeded
device generator (their stored BF16 values exist only on a GPU), so the second form
needs one, for drawing the inputs alone.

Every solution is the oracle's FP64 RAC-MBADMM (Eq.(3)) with residual balancing, run
until its KKT residual is at most 1e-9.  A file holds a header (workload, lane, the
oracle's iterations and KKT residual, the objective of Eq.(5)/(6) and ||z||_2) and
then z, one value per line with 17 significant digits.
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1907_01995_amd import workloads as W  # noqa: E402

TOL = 1e-9
OUT = HERE
LANES = (0, 7, 15)          # lambda_max * 0.01^(j/15) for these j


def write(path, header, z):
    with open(path, "w") as f:
        for k, v in header.items():
            f.write("# %s: %s\n" % (k, v))
        for v in z:
            f.write("%.17g\n" % v)


def read(path):
    """(header dict, z) of a file written by this script."""
    head, vals = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                k, v = line[1:].split(":", 1)
                head[k.strip()] = v.strip()
            else:
                vals.append(float(line))
    return head, np.array(vals)


def converge(op, name, beta0, chunk=500, cap=200000, **kw):
    """The oracle run to KKT <= TOL in chunks of iterations, each continuing from the
    previous one's iterate, penalty and iteration count (a progress line per chunk)."""
    t0 = time.time()
    state, done, beta = None, 0, beta0
    while True:
        r = O.solve(op, beta_mode=O.BETA_RESBAL, check_every=10, max_iter=chunk, tol=TOL, beta0=beta,
                    state=state, iter0=done, **kw)
        done += r.iters
        beta = r.beta
        state = (r.x, r.z, r.xi, r.mu)
        k = O.kkt(op, r.x, r.z, r.xi, r.mu)
        print("%s: %d iterations, KKT %.3e, %.0f s" % (name, done, k, time.time() - t0), flush=True)
        if k <= TOL:
            return r, done, k, time.time() - t0
        if done >= cap:
            raise SystemExit("%s: the oracle stopped at KKT %.3e after %d iterations" % (name, k, done))


def lasso():
    w = W.lasso_20000x2000("f32")
    op = O.en_problem(w.D.astype(np.float64), w.y, lam=w.lam, alpha=1.0)
    r, iters, k, dt = converge(op, "lasso_20000x2000", w.beta0, chunk=50, s=w.block_size)
    head = {"workload": "lasso_20000x2000 (f32 stored values)", "iterations": iters, "kkt": "%.6e" % k,
            "objective": "%.17g" % O.objective(op, r.z), "znorm": "%.17g" % np.linalg.norm(r.z),
            "seconds": "%.0f" % dt}
    write(os.path.join(OUT, "lasso_20000x2000_solution.txt"), head, r.z)
    print(head, flush=True)


def en_paths_sample(Ns, ns):
    """The sampled instances of the batched workload: the two smallest, the median one,
    the smallest that needs a team of 32 workgroups, and the one with most blocks among
    those of at most 4e6 stored values."""
    size = Ns.astype(np.float64) * ns
    order = np.argsort(size, kind="stable")
    wide = min((i for i in range(len(Ns)) if Ns[i] > 16 * 640), key=lambda i: size[i])
    deep = max((i for i in range(len(Ns)) if size[i] <= 4e6), key=lambda i: ns[i])
    return sorted({int(order[0]), int(order[1]), int(order[len(order) // 2]), int(wide), int(deep)})


def en_paths():
    import torch
    assert torch.cuda.is_available(), "the batched instances are drawn on the GPU"
    Ns, ns = W.en_batch_sizes(256)
    jobs = []
    for i in en_paths_sample(Ns, ns):
        d = W.en_instance_device(int(Ns[i]), int(ns[i]), 1000 + i, storage="bf16")
        D, y = d.host_D(), np.asarray(d.y, dtype=np.float64)
        lams = W.lambda_grid(d.lam_max, 16, 0.01)
        for j in LANES:
            jobs.append((i, j, D, y, float(lams[j])))
        del d
    torch.cuda.empty_cache()

    def one(job):
        i, j, D, y, lam = job
        op = O.en_problem(D, y, lam=lam, alpha=0.5)
        r, iters, k, dt = converge(op, "lane %d" % (16 * i + j), 0.1 * lam, s=64, seed=11, inst=i)
        head = {"workload": "en_paths_256x16 (bf16 stored values)", "instance": i, "lane": 16 * i + j,
                "N": D.shape[0], "n": D.shape[1], "lambda": "%.17g" % lam, "alpha": 0.5, "iterations": iters,
                "kkt": "%.6e" % k, "objective": "%.17g" % O.objective(op, r.z),
                "znorm": "%.17g" % np.linalg.norm(r.z), "seconds": "%.0f" % dt}
        write(os.path.join(OUT, "en_paths_256x16_lane%d_solution.txt" % (16 * i + j)), head, r.z)
        print(head, flush=True)

    with ThreadPoolExecutor(max_workers=min(15, len(jobs))) as ex:   # the oracle releases the GIL
        list(ex.map(one, jobs))


if __name__ == "__main__":
    if len(sys.argv) > 2:
        OUT = sys.argv[2]
        os.makedirs(OUT, exist_ok=True)
    {"lasso": lasso, "en_paths": en_paths}[sys.argv[1]]()
