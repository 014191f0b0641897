"""Served stream of uneven least-squares requests on one GPU, against the plain path.

Requests (sizes from gen.served_stream: n log-uniform, m = n U(1.1, 2.0), a tenth
with dense rows) arrive as a Poisson process and go through the serving runtime
(include/rsilu_serve.h): host setup threads, admission by device footprint into one
HBM arena, concurrent solves on per-slot streams. The plain path handles the same
requests one at a time (setup, upload, solve). Prints one JSON line with solves/s and
p50/p99 latency of both, how many served results equal the plain ones bit for bit, and
the largest ||A^T A (x_served - x_plain)|| / ||A^T b|| (batched launches sum in another
order than the plain path).

Usage: python -m paper_2603_28642_amd.serve_bench [--requests 128] [--slots 8] ...
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=128)
    ap.add_argument("--n-lo", type=int, default=2000)
    ap.add_argument("--n-hi", type=int, default=100000)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--setup-threads", type=int, default=12)
    ap.add_argument("--hbm-gb", type=float, default=32.0)
    ap.add_argument("--load", type=float, default=0.8, help="offered load as a fraction of the served capacity "
                                                           "estimated from the plain path and the thread count")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--batch-max", type=int, default=32, help="requests per batched launch (0: rsilu_solve each)")
    ap.add_argument("--tune-slack", type=float, default=8.0, help="autotuner slack (0: default tile, no tuning)")
    args = ap.parse_args()
    # one hardware queue per solve slot (the runtime's default is 4)
    os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(max(args.slots, 4), 32)))

    import numpy as np
    import torch

    import gen
    from paper_2603_28642_amd import rsilu as R

    prec = {"fp32": R.PREC_FP32, "fp64": R.PREC_FP64}[args.precision]
    params = dict(mu=1.0, form=R.FORM_ALG2, smode=R.S_NONE, krylov=R.KRYLOV_LSQR, precision=prec)
    sizes = gen.served_stream(args.requests, seed=args.seed, n_lo=args.n_lo, n_hi=args.n_hi)
    probs = [gen.served_request(n, m, s, n_dense=nd) for n, m, s, nd in sizes]
    print("generated %d requests" % len(probs), file=sys.stderr, flush=True)

    # ---- plain path: one request at a time
    plain_x, plain_lat, plain_setup = [], [], []
    t0 = time.perf_counter()
    for p in probs:
        t1 = time.perf_counter()
        S = R.Solver.from_problem(p, **params)
        t2 = time.perf_counter()
        S.upload()
        x, code, it, atr, rel = S.solve(torch.from_numpy(p.b).cuda(), tol=args.tol)
        plain_x.append(x.cpu().numpy())
        S.close()
        plain_lat.append(time.perf_counter() - t1)
        plain_setup.append(t2 - t1)
    plain_total = time.perf_counter() - t0
    print("plain path done in %.1f s" % plain_total, file=sys.stderr, flush=True)

    # ---- served: Poisson arrivals at the offered load
    capacity = len(probs) / max(plain_total, 1e-9) * min(args.setup_threads, args.slots)
    rate = args.load * capacity
    rng = np.random.default_rng(args.seed + 1)
    gaps = rng.exponential(1.0 / rate, size=len(probs))
    srv = R.Server(hbm_bytes=int(args.hbm_gb * (1 << 30)), slots=args.slots, setup_threads=args.setup_threads,
                   batch_max=args.batch_max, tune_slack=args.tune_slack)
    results = {}
    ids = {}
    t_start = time.perf_counter()
    t_next = t_start
    for i, p in enumerate(probs):
        t_next += gaps[i]
        while True:
            for res, x in srv.poll(wait_ms=0):
                results[ids[res["id"]]] = (res, x, time.perf_counter())
            now = time.perf_counter()
            if now >= t_next:
                break
            time.sleep(min(t_next - now, 0.002))
        ids[srv.submit(p.m, p.n, p.rowptr, p.col, p.val, p.b, tol=args.tol, **params)] = i
    while len(results) < len(probs):
        for res, x in srv.poll(wait_ms=100):
            results[ids[res["id"]]] = (res, x, time.perf_counter())
    served_total = max(r[2] for r in results.values()) - t_start
    srv.close()

    lat = np.array([results[i][0]["total_ms"] for i in range(len(probs))])
    ok = sum(1 for i in range(len(probs)) if results[i][0]["status"] == R.OK)
    same = sum(1 for i in range(len(probs)) if np.array_equal(results[i][1].view(np.int64), plain_x[i].view(np.int64)))
    # batched results differ from the plain ones in the order of sums only: both in the stop-test ball
    ball = max(float(np.linalg.norm(probs[i].scipy().T @ (probs[i].scipy() @ (results[i][1] - plain_x[i]))) /
                     np.linalg.norm(probs[i].scipy().T @ probs[i].b)) for i in range(len(probs)))
    solve_ms = np.array([results[i][0]["solve_ms"] for i in range(len(probs))])
    setup_ms = np.array([results[i][0]["setup_ms"] for i in range(len(probs))])
    wait_ms = np.array([results[i][0]["wait_ms"] for i in range(len(probs))])
    out = {
        "metric": "served mixed-size least-squares solves/s; p50/p99 latency (submit to x on the host)",
        "requests": len(probs),
        "n_range": [args.n_lo, args.n_hi],
        "precision": args.precision,
        "slots": args.slots,
        "batch_max": args.batch_max,
        "tune_slack": args.tune_slack,
        "paths": {"batched": sum(1 for i in range(len(probs)) if results[i][0]["path"] == 0),
                  "plain": sum(1 for i in range(len(probs)) if results[i][0]["path"] == 1)},
        "median_launch_size": float(np.median([results[i][0]["launch_size"] for i in range(len(probs))])),
        "setup_threads": args.setup_threads,
        "offered_rate_per_s": rate,
        "served": {"solves_per_s": len(probs) / served_total, "p50_ms": float(np.percentile(lat, 50)),
                   "p99_ms": float(np.percentile(lat, 99)), "ok": ok,
                   "median_setup_ms": float(np.median(setup_ms)), "median_wait_ms": float(np.median(wait_ms)),
                   "median_solve_ms": float(np.median(solve_ms)), "p99_solve_ms": float(np.percentile(solve_ms, 99))},
        "plain": {"solves_per_s": len(probs) / plain_total, "p50_ms": 1e3 * float(np.percentile(plain_lat, 50)),
                  "p99_ms": 1e3 * float(np.percentile(plain_lat, 99)),
                  "median_setup_ms": 1e3 * float(np.median(plain_setup))},
        "identical_to_plain": same,
        "max_ball_vs_plain": ball,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
