"""Served stream of uneven least-squares requests on one GPU, against the plain path.

Requests (sizes from gen.served_stream: n log-uniform, m = n U(1.1, 2.0), a tenth with
8-32 dense rows) arrive as a Poisson process and go through the serving runtime
(include/rsilu_serve.h): host setup threads, admission by device footprint into one HBM
arena, concurrent solves on per-slot streams, requests admitted together sharing batched
persistent launches. Every request is LSQR with Algorithm 2, FP32 preconditioner and FP64
Krylov part by default; the sparse requests take the M_b correction by a degree-2 Chebyshev
polynomial in S~ through the explicit Y~ (the fixed two-step analogue of Table 3(a)'s
CG(2)), the requests with dense rows none by default (there S~'s interval reaches b = 60 to
20000: the degree that covers it costs hundreds of products with Y~ per application, and
degree 2, scaled to stay positive definite, weakens the preconditioner to over 1000
iterations on some of them).

The plain path is the same method with the FP64 preconditioner, one request at a time
(setup, upload, rsilu_solve, copy back), run on every `--plain-every`-th request of the
stream (the host setup of the whole stream takes over an hour on one core): its latency
per request is that request's service time with no queueing, and its solves/s is one over
the mean service time.

Prints one JSON line with solves/s and p50/p99 latency of both, the served device times,
how many requests took batched launches, and for the requests of the plain sample the
largest ||A^T A (x_served - x_plain)|| / ||A^T b||.

Usage: python -m paper_2603_28642_amd.serve_bench [--requests 512] [--mode served|plain|both] ...
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
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--n-lo", type=int, default=2000)
    ap.add_argument("--n-hi", type=int, default=200000)
    ap.add_argument("--mode", default="both", choices=["served", "plain", "both"])
    ap.add_argument("--plain-every", type=int, default=16, help="plain path on every k-th request")
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--setup-threads", type=int, default=16)
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--rate", type=float, default=1.5, help="Poisson arrival rate, requests/s")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--correction", default="cheb2", choices=["cheb2", "none"],
                    help="M_b of the sparse requests: degree-2 Chebyshev through the explicit Y~, or none")
    ap.add_argument("--dense-correction", default="none", choices=["cheb2", "none"],
                    help="M_b of the requests with dense rows")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--batch-max", type=int, default=32, help="requests per batched launch (0: rsilu_solve each)")
    ap.add_argument("--tune-slack", type=float, default=2.0, help="autotuner slack (0: default tile, no tuning)")
    ap.add_argument("--records", default="", help="write one JSON record per served request to this file")
    ap.add_argument("--batch-wait-ms", type=float, default=100.0,
                    help="batching window: a slot that admitted a request waits this long for more to finish setup")
    args = ap.parse_args()
    # one hardware queue per solve slot (the runtime's default is 4)
    os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(max(args.slots, 4), 32)))

    import numpy as np
    import torch

    import gen
    from paper_2603_28642_amd import rsilu as R

    def method_for(corr):
        kw = dict(mu=1.0, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR)
        if corr == "cheb2":
            kw.update(smode=R.S_CHEB, ystore=R.Y_EXPLICIT, ytau=1e-2, poly_degree=2)
        else:
            kw.update(smode=R.S_NONE)
        return kw

    def method(nd):
        return method_for(args.dense_correction if nd > 0 else args.correction)
    prec = {"fp32": R.PREC_FP32, "fp64": R.PREC_FP64}[args.precision]
    sizes = gen.served_stream(args.requests, seed=args.seed, n_lo=args.n_lo, n_hi=args.n_hi)
    out = {
        "metric": "served mixed-size least-squares solves/s; p50/p99 latency (submit to x on the host)",
        "requests": len(sizes), "n_range": [args.n_lo, args.n_hi], "method": "LSQR, Algorithm 2; M_b " +
        ("Chebyshev degree 2 on S~ (explicit Y~)" if args.correction == "cheb2" else "none") +
        " (requests with dense rows: " +
        ("Chebyshev degree 2" if args.dense_correction == "cheb2" else "none") + ")",
    }
    plain_idx = list(range(0, len(sizes), args.plain_every))
    plain_x = {}
    if args.mode in ("plain", "both"):
        lat, setup, solve = [], [], []
        for i in plain_idx:
            n, m, s, nd = sizes[i]
            p = gen.served_request(n, m, s, n_dense=nd)
            t1 = time.perf_counter()
            S = R.Solver.from_problem(p, precision=R.PREC_FP64, maxit=2000, **method(nd))
            t2 = time.perf_counter()
            S.upload()
            x, code, it, atr, rel = S.solve(torch.from_numpy(p.b).cuda(), tol=args.tol)
            plain_x[i] = x.cpu().numpy()
            t3 = time.perf_counter()
            S.close()
            lat.append(t3 - t1)
            setup.append(t2 - t1)
            solve.append(t3 - t2)
            print("plain %d: n %d m %d dense %d: setup %.2f s, device %.1f ms, %d its" % (
                i, n, m, nd, t2 - t1, 1e3 * (t3 - t2), it), file=sys.stderr, flush=True)
        lat = np.array(lat)
        out["plain"] = {"precision": "fp64", "sample": "every %d-th request (%d)" % (args.plain_every, len(plain_idx)),
                        "solves_per_s": 1.0 / float(lat.mean()), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                        "p99_ms": 1e3 * float(np.percentile(lat, 99)), "median_setup_ms": 1e3 * float(np.median(setup)),
                        "median_device_ms": 1e3 * float(np.median(solve)),
                        "p99_device_ms": 1e3 * float(np.percentile(solve, 99))}
    if args.mode in ("served", "both"):
        probs = []
        for n, m, s, nd in sizes:
            probs.append(gen.served_request(n, m, s, n_dense=nd))
        print("generated %d requests" % len(probs), file=sys.stderr, flush=True)
        rng = np.random.default_rng(args.seed + 1)
        gaps = rng.exponential(1.0 / args.rate, size=len(probs))
        srv = R.Server(hbm_bytes=int(args.hbm_gb * (1 << 30)), slots=args.slots, setup_threads=args.setup_threads,
                       batch_max=args.batch_max, tune_slack=args.tune_slack, batch_wait_ms=args.batch_wait_ms)
        results, ids = {}, {}
        t_start = time.perf_counter()
        t_next = t_start
        last_report = t_start
        for i, p in enumerate(probs):
            t_next += gaps[i]
            while True:
                for res, x in srv.poll(wait_ms=0):
                    results[ids[res["id"]]] = (res, x, time.perf_counter())
                now = time.perf_counter()
                if now >= t_next:
                    break
                time.sleep(min(t_next - now, 0.002))
            ids[srv.submit(p.m, p.n, p.rowptr, p.col, p.val, p.b, tol=args.tol, precision=prec, maxit=2000,
                           **method(sizes[i][3]))] = i
            if time.perf_counter() - last_report > 30:
                last_report = time.perf_counter()
                print("submitted %d, done %d" % (i + 1, len(results)), file=sys.stderr, flush=True)
        while len(results) < len(probs):
            for res, x in srv.poll(wait_ms=100):
                results[ids[res["id"]]] = (res, x, time.perf_counter())
            if time.perf_counter() - last_report > 30:
                last_report = time.perf_counter()
                print("done %d of %d" % (len(results), len(probs)), file=sys.stderr, flush=True)
        served_total = max(r[2] for r in results.values()) - t_start
        srv.close()
        res = [results[i][0] for i in range(len(probs))]
        if args.records:
            with open(args.records, "w") as f:
                for i, r in enumerate(res):
                    n, m, _, nd = sizes[i]
                    rec = {k: r[k] for k in ("status", "iters", "atr_rel", "setup_ms", "wait_ms", "solve_ms",
                                             "total_ms", "path", "launch_size")}
                    rec.update(i=i, n=n, m=m, dense=nd, tile=list(r["tile"]))
                    f.write(json.dumps(rec) + "\n")
        lat = np.array([r["total_ms"] for r in res])
        solve_ms = np.array([r["solve_ms"] for r in res])
        batched = [r for r in res if r["path"] == 0]
        ball = None
        if plain_x:
            ball = max(float(np.linalg.norm(probs[i].scipy().T @ (probs[i].scipy() @ (results[i][1] - plain_x[i]))) /
                             np.linalg.norm(probs[i].scipy().T @ probs[i].b)) for i in plain_x)
        out["served"] = {
            "precision": args.precision, "slots": args.slots, "setup_threads": args.setup_threads,
            "batch_max": args.batch_max, "tune_slack": args.tune_slack, "batch_wait_ms": args.batch_wait_ms,
            "arrival_rate_per_s": args.rate,
            "solves_per_s": len(probs) / served_total, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "ok": sum(1 for r in res if r["status"] == R.OK),
            "median_setup_ms": float(np.median([r["setup_ms"] for r in res])),
            "median_wait_ms": float(np.median([r["wait_ms"] for r in res])),
            "median_device_ms": float(np.median(solve_ms)), "p99_device_ms": float(np.percentile(solve_ms, 99)),
            "paths": {"batched": len(batched), "plain": len(res) - len(batched)},
            "batched_launch_sizes": sorted({int(r["launch_size"]) for r in batched}),
            "median_iters": float(np.median([r["iters"] for r in res])),
            "max_ball_vs_plain_sample": ball,
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
