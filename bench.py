#!/usr/bin/env python3
"""Benchmark: preconditioned least-squares solves per second on one MI355X.

A step is one whole preconditioned solve (LSQR or Algorithm 1, every kernel
on the GPU) of the grid-shaped workload, m = 600,000, n = 400,000, from
b resident in HBM to x in HBM with the iteration count and ||A^T r|| on the
host. Setup (the host ILUP) is done once, outside the timed region.

The default Krylov method is LSQR in the M-inner-product form (--krylov pcgls
runs Algorithm 1; both give the same iterates in exact arithmetic), with the
preconditioner applied by Algorithm 2 with k = n and M_a = (L1 U)^T (L1 U)
from the ILUP(10, 1e-2) factors (mu = 1), without the M_b correction: on this
workload it reaches ||A^T r|| <= 1e-8 ||A^T b||, whereas Algorithm 3 on the
residual stalls near its starting residual (--form alg3 --krylov pcgls runs
it; the solve then ends at maxit or on a breakdown).

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
    ap.add_argument("--smode", default="none", choices=["none", "identity", "dense", "auto"])
    ap.add_argument("--form", default="alg2", choices=["alg2", "alg3"])
    ap.add_argument("--krylov", default="lsqr", choices=["pcgls", "lsqr"],
                    help="Algorithm 1 (PCGLS) or LSQR in the M-inner-product form (needs --form alg2)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the preconditioner (factors and Algorithm 2/3); Krylov part is FP64")
    ap.add_argument("--trsv", default="hybrid", choices=["hybrid", "syncfree", "levels"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (three of them) and exit: the known-size "
                         "reference that scales the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_probe(mib):
    import torch

    n = mib * (1 << 20) // 8
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "copies": 3}), flush=True)


def step_bytes(st, vb=8):
    """Algorithmic HBM bytes of one use of each step: stored values (vb bytes: 8 for
    FP64, 4 for the FP32 preconditioner's factors and vectors) and int32 column indices
    read once, row pointers once, a triangular solve's level list, right-hand side and
    result once per row (plus its diagonal, and a fused addend and sum), every other
    vector read or written once."""
    m, n = st.m, st.n
    k = m - n
    a, l1, l2, u = st.nnz_a, st.nnz_l1, st.nnz_l2, st.nnz_u
    e = 4 + vb  # one stored entry
    tri = (8 + 2 * vb) * n  # pointer, level-list entry, rhs, result per row
    return {
        "spmv_A": 12 * a + 4 * (m + 1) + 8 * n + 8 * m,
        "spmv_AT": 12 * a + 4 * (n + 1) + 8 * m + 8 * n + 8 * n,
        "trsv_L1": e * l1 + tri,
        "trsv_L1T": e * l1 + tri,
        "trsv_L1T_fused": e * l1 + tri + 2 * vb * n,
        "trsv_U": e * u + tri + vb * n,
        "trsv_UT": e * u + tri + vb * n,
        "spmv_L2": e * l2 + 4 * (k + 1) + vb * (n + k),
        "spmv_L2_sub": e * l2 + 4 * (k + 1) + vb * (n + 2 * k),
        "spmv_L2T": e * l2 + 4 * (n + 1) + vb * (k + n),
        "dense_S": 8 * k * (k + 1) + 16 * k,
        # x += alpha p, r -= alpha q; rho = (z, h); p = h + beta p
        "vectors": 8 * (3 * n + 3 * m) + 16 * n + 24 * n,
        # FP32 preconditioner: input to FP32 and h back to FP64
        "convert": 12 * n + 12 * n if vb == 4 else 0,
    }


def iteration_bytes(st, form, smode, vb=8):
    """Algorithmic bytes of one iteration of Algorithm 1 with the given form."""
    b = step_bytes(st, vb)
    k = st.m - st.n
    it = b["spmv_A"] + b["spmv_AT"] + b["vectors"] + b["convert"]
    if vb == 4 and form == "alg3":
        it += 12 * (st.m - st.n)  # the m-vector r is converted, not only n entries
    corr = k > 0 and smode != "none"
    if form == "alg3":
        it += b["trsv_L1"] + b["trsv_U"]
        if corr:
            it += b["spmv_L2_sub"] + b["spmv_L2T"] + b["trsv_L1T_fused"] + b["trsv_L1"]
    else:
        it += b["trsv_UT"] + b["trsv_L1T"] + b["trsv_L1"] + b["trsv_U"]
        if corr:
            it += b["trsv_L1"] + b["spmv_L2"] + b["spmv_L2T"] + b["trsv_L1T_fused"]
    if corr and smode == "dense":
        it += b["dense_S"]
    return it


def measured_traffic(kernel, workload, args):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE counter
    runs (profiles/traffic_<kernel>_<workload>.json, calibrated by a copy of known size),
    or None when there is no record, the record was taken with another solver
    configuration than this run's, or the kernel's sources changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    cfg = rec.get("config")
    if cfg is None or any(getattr(args, k) != v for k, v in cfg.items()):
        return None
    h = hashlib.sha256()
    for fn in rec["sources"]:
        with open(os.path.join(ROOT, fn), "rb") as src:
            h.update(src.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(prob, args, iters_per_solve):
    """The oracle's Algorithm 1 on the same problem, timed on a bounded number of
    iterations and scaled to whole solves of the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        smode = args.smode if args.smode != "auto" else ("dense" if 0 < prob.m - prob.n <= 4096 else "identity")
        F = oracle.factor_problem(prob, p=args.p, tau=args.tau, mu=args.mu, smode=smode)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        def run(maxit):
            if args.krylov == "lsqr":
                return oracle.lsqr_m(F, prob.b, tol=0.0, maxit=maxit)
            return oracle.pcgls(F, prob.b, tol=0.0, maxit=maxit, form=args.form)

        run(2)
        est = max((time.perf_counter() - t0) / 2.0, 1e-6)
        k = int(max(2, min(iters_per_solve if iters_per_solve > 0 else 2, args.cpu_seconds / est)))
        t0 = time.perf_counter()
        res = run(k)
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
        "sample": "oracle " + ("LSQR" if args.krylov == "lsqr" else "Algorithm 1") + " + Algorithm " + args.form[-1] +
                  " (plain C substitutions, numpy vectors, 1 thread) on the same "
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

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import numpy as np
    import torch

    import gen
    from paper_2603_28642_amd import rsilu as R

    torch.cuda.set_device(0)
    prob = gen.by_name(args.workload)
    smode = {"none": R.S_NONE, "identity": R.S_IDENTITY, "dense": R.S_DENSE, "auto": R.S_AUTO}[args.smode]
    trsv = {"hybrid": R.TRSV_HYBRID, "syncfree": R.TRSV_SYNCFREE, "levels": R.TRSV_LEVELS}[args.trsv]
    form = {"alg2": R.FORM_ALG2, "alg3": R.FORM_ALG3}[args.form]
    t0 = time.perf_counter()
    precision = {"fp64": R.PREC_FP64, "fp32": R.PREC_FP32}[args.precision]
    krylov = {"pcgls": R.KRYLOV_PCGLS, "lsqr": R.KRYLOV_LSQR}[args.krylov]
    S = R.Solver.from_problem(prob, p=args.p, tau=args.tau, mu=args.mu, smode=smode, maxit=args.maxit, trsv=trsv,
                              form=form, precision=precision, krylov=krylov)
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

    # dominant kernel by total time in the timed region (single-kernel classes; the
    # library adds up the algorithmic bytes of every timed launch)
    kernels = [k for k in R.PROF_NAMES if k not in R.PROF_STEPS]
    dom = max(kernels, key=lambda k: prof[k][1])
    launches, ms, kbytes = prof[dom]
    avg_s = (ms / 1e3) / max(launches, 1)
    kb = kbytes / max(launches, 1)
    achieved = kb / avg_s if avg_s > 0 else 0.0
    t_solve = total / args.steps
    smode_used = {R.S_NONE: "none", R.S_IDENTITY: "identity", R.S_DENSE: "dense"}[st.smode]
    b_solve = (iters + 1) * iteration_bytes(st, args.form, smode_used, 4 if args.precision == "fp32" else 8)
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
        "dtype": "f64" if args.precision == "fp64" else "f64 (preconditioner f32)",
        "data": "synthetic",
        "config": {
            "workload": prob.name + " (%s)" % args.workload,
            "nnz": int(st.nnz_a),
            "ilup": {"p": args.p, "tau": args.tau, "mu": args.mu, "small": 1e-10},
            "S": smode_used,
            "krylov": ("LSQR (M-inner-product form)" if args.krylov == "lsqr" else "Algorithm 1 (PCGLS)") +
                      " + Algorithm %s" % args.form[-1],
            "trsv": args.trsv,
            "precond_precision": args.precision,
            "tol": args.tol,
            "maxit": args.maxit,
            "iters": iters,
            "status": status,
            "atr_rel": rel,
            "factors": {"nnz_l1": int(st.nnz_l1), "nnz_l2": int(st.nnz_l2), "nnz_u": int(st.nnz_u),
                        "levels_l1": int(st.levels_l1), "levels_l1t": int(st.levels_l1t),
                        "levels_u": int(st.levels_u), "levels_ut": int(st.levels_ut), "nmod": int(st.nmod)},
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
            "traffic": measured_traffic(dom, args.workload, args),
            "bytes_per_launch": kb,
            "avg_launch_us": avg_s * 1e6,
            "launches": launches,
            "step_ms_share": {k: round(prof[k][1] / max(sum(prof[w][1] for w in R.PROF_STEPS), 1e-12), 4)
                              for k in R.PROF_STEPS if prof[k][0]},
            "kernel_avg_us": {k: round(1e3 * prof[k][1] / prof[k][0], 2) for k in kernels if prof[k][0]},
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args, iters)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
