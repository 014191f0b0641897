#!/usr/bin/env python3
"""Benchmark: preconditioned least-squares solves per second on one MI355X.

A step is one whole solve (Algorithm 1 with Algorithm 3, every kernel on the
GPU) of the grid-shaped workload, m = 600,000, n = 400,000, from b resident in
HBM to x in HBM with the iteration count and ||A^T r|| on the host. Setup (the
host ILUP) is done once, outside the timed region.

Prints one JSON line with the throughput, p50/p99 latency, the roofline of the
dominant kernel (HIP events recorded by the library on the solve's stream over
the timed region) and the CPU oracle timed on a bounded sample of the same
solve.
"""

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "preconditioned LSQR solves/s to ||A^T r||/||A^T b||<=1e-8; % HBM peak; p99 latency"
HBM_PEAK = 8.0e12  # bytes/s, MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", help="c2 (grid 600000 x 400000), c2-small, c1, c3-mini")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--mu", type=float, default=1.0)
    ap.add_argument("--tau", type=float, default=1e-2)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--smode", default="identity", choices=["identity", "dense", "auto"])
    ap.add_argument("--trsv", default="hybrid", choices=["hybrid", "syncfree", "levels"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def kernel_bytes(st, cls):
    """Algorithmic HBM bytes of one launch of a kernel class: FP64 values and int32
    indices streamed once, row pointers and level lists once, every vector read or
    written once (a gathered vector counted once)."""
    m, n = st.m, st.n
    k = m - n
    a, l1, l2, u = st.nnz_a, st.nnz_l1, st.nnz_l2, st.nnz_u
    return {
        "spmv_A": 12 * a + 4 * (m + 1) + 8 * n + 8 * m,
        "spmv_AT": 12 * a + 4 * (n + 1) + 8 * m + 8 * n + 8 * n,
        "trsv_L1": 12 * l1 + 4 * (n + 1) + 4 * n + 8 * n * 3,
        "trsv_L1T": 12 * l1 + 4 * (n + 1) + 4 * n + 8 * n * 3 + 16 * n,
        "trsv_U": 12 * u + 4 * (n + 1) + 4 * n + 8 * n * 3 + 8 * n,
        "spmv_L2": 12 * l2 + 4 * (k + 1) + 8 * n + 16 * k,
        "spmv_L2T": 12 * l2 + 4 * (n + 1) + 8 * k + 8 * n,
        "dense_S": 8 * k * (k + 1) + 32 * k,
    }[cls]


def iteration_bytes(st, dense):
    """Algorithmic bytes of one iteration: 2 products with A, 3 sweeps of L1, 2 of L2,
    1 of U, row pointers, level lists and about 32 vector passes."""
    m, n = st.m, st.n
    b = 12 * (2 * st.nnz_a + 3 * st.nnz_l1 + 2 * st.nnz_l2 + st.nnz_u) + 4 * (2 * m + 5 * n) + 16 * n \
        + 8 * (24 * n + 5 * m + 3 * (m - n))
    if dense:
        b += 8 * (m - n) * (m - n + 1)
    return b


def cpu_baseline(prob, args, iters_per_solve):
    """The oracle's Algorithm 1 on the same problem, timed on a bounded number of
    iterations and scaled to whole solves of the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        F = oracle.factor_problem(prob, p=args.p, tau=args.tau, mu=args.mu,
                                  smode="dense" if args.smode == "dense" else "identity")
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.pcgls(F, prob.b, tol=0.0, maxit=2)
        est = max((time.perf_counter() - t0) / 2.0, 1e-6)
        k = int(max(2, min(iters_per_solve if iters_per_solve > 0 else 2, args.cpu_seconds / est)))
        t0 = time.perf_counter()
        res = oracle.pcgls(F, prob.b, tol=0.0, maxit=k)
        t = time.perf_counter() - t0
    per_iter = t / max(res.iters, 1)
    per_solve = per_iter * max(iters_per_solve, 1)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "oracle Algorithm 1 + Algorithm 3 (plain C substitutions, numpy vectors, 1 thread) on the same "
                  "workload: %d iterations timed (%.1f s, %.1f ms/iteration), scaled to the %d iterations of one "
                  "GPU solve; oracle setup %.1f s not counted; host %s, nproc %d"
                  % (res.iters, t, per_iter * 1e3, iters_per_solve, t_setup, cpu, os.cpu_count() or 0),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solve of one least-squares problem is not split across "
              "GPUs (independent solves shard with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    from paper_2603_28642_amd import rsilu as R

    torch.cuda.set_device(0)
    prob = gen.by_name(args.workload)
    smode = {"identity": R.S_IDENTITY, "dense": R.S_DENSE, "auto": R.S_AUTO}[args.smode]
    trsv = {"hybrid": R.TRSV_HYBRID, "syncfree": R.TRSV_SYNCFREE, "levels": R.TRSV_LEVELS}[args.trsv]
    t0 = time.perf_counter()
    S = R.Solver.from_problem(prob, p=args.p, tau=args.tau, mu=args.mu, smode=smode, maxit=args.maxit, trsv=trsv)
    t_setup = time.perf_counter() - t0
    S.upload()
    st = S.stats
    b = torch.from_numpy(prob.b).cuda()
    x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        S.solve(b, tol=args.tol, x_dev=x)
    torch.cuda.synchronize()

    R.rsilu_set_profiling(S.h, 1)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    result = None
    for _ in range(args.steps):
        t1 = time.perf_counter()
        result = S.solve(b, tol=args.tol, x_dev=x)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    prof = R.rsilu_get_profile(S.h)
    R.rsilu_set_profiling(S.h, 0)
    _, code, iters, atr, rel = result

    # dominant kernel by total time in the timed region
    dom = max(prof, key=lambda k: prof[k][1])
    launches, ms = prof[dom]
    avg_s = (ms / 1e3) / max(launches, 1)
    kb = kernel_bytes(st, dom)
    achieved = kb / avg_s if avg_s > 0 else 0.0
    t_solve = total / args.steps
    b_solve = (iters + 1) * iteration_bytes(st, st.smode == R.S_DENSE)
    status = {R.OK: "converged", R.NOT_CONVERGED: "not_converged", R.BREAKDOWN: "breakdown"}.get(code, str(code))

    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_solve,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": prob.name + " (%s)" % args.workload,
            "nnz": int(st.nnz_a),
            "ilup": {"p": args.p, "tau": args.tau, "mu": args.mu, "small": 1e-10},
            "S": "dense" if st.smode == R.S_DENSE else "identity",
            "krylov": "Algorithm 1 (PCGLS) + Algorithm 3",
            "trsv": args.trsv,
            "tol": args.tol,
            "maxit": args.maxit,
            "iters": iters,
            "status": status,
            "atr_rel": rel,
            "factors": {"nnz_l1": int(st.nnz_l1), "nnz_l2": int(st.nnz_l2), "nnz_u": int(st.nnz_u),
                        "levels_l1": int(st.levels_l1), "levels_l1t": int(st.levels_l1t),
                        "levels_u": int(st.levels_u), "nmod": int(st.nmod)},
            "setup_s": t_setup,
        },
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "hbm_frac_solve": b_solve / t_solve / HBM_PEAK,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved / 1e9,
            "peak": HBM_PEAK / 1e9,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK,
            "traffic": None,
            "bytes_per_launch": kb,
            "avg_launch_us": avg_s * 1e6,
            "launches": launches,
            "kernel_ms_share": {k: round(v[1] / max(sum(w[1] for w in prof.values()), 1e-12), 4)
                                for k, v in prof.items() if v[0]},
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args, iters)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
