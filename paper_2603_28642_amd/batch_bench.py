"""Batched persistent solves against the plain path on one GPU.

Two sets of independent least-squares problems, each factored once on the host and
uploaded (outside every timed region):
  * tiny: K problems of the 2000 x 1000 tiny-case recipe (different seeds);
  * mixed: K problems of the served-stream recipe, n log-uniform in [n_lo, n_hi],
    m = n U(1.1, 2.0), a tenth with 8-32 dense rows.
Each set is solved to ||A^T r|| <= tol ||A^T b|| (LSQR, Algorithm 2 form without the
M_b correction) four ways: one rsilu_solve after another (the plain multi-kernel
path), one rsilu_batch_solve launch with the default tile, one launch with the tile
the autotuner picked for the set's first problem, and rsilu_batch_solve_auto (every
signature tuned, the slowest problems moved to the plain path beside the launch). Prints one JSON line with
solves/s of each, the tuner's choice and the largest deviation of a batched solution
from its plain one, relative to the stop-test ball ||A^T A e|| / ||A^T b||.

Usage: python -m paper_2603_28642_amd.batch_bench [--k 256] [--set tiny|mixed] ...
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
    ap.add_argument("--set", default="tiny", choices=["tiny", "mixed"])
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--n-lo", type=int, default=2000)
    ap.add_argument("--n-hi", type=int, default=20000)
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()

    import numpy as np
    import torch

    import gen
    from paper_2603_28642_amd import rsilu as R

    prec = {"fp32": R.PREC_FP32, "fp64": R.PREC_FP64}[args.precision]
    params = dict(mu=1.0, form=R.FORM_ALG2, smode=R.S_NONE, krylov=R.KRYLOV_LSQR, precision=prec, maxit=2000)
    if args.set == "tiny":
        probs = [gen.tiny_c1(seed=1000 + i) for i in range(args.k)]
    else:
        sizes = gen.served_stream(args.k, seed=args.seed, n_lo=args.n_lo, n_hi=args.n_hi)
        probs = [gen.served_request(n, m, s, n_dense=nd) for n, m, s, nd in sizes]
    t0 = time.perf_counter()
    S = [R.Solver.from_problem(p, **params).upload() for p in probs]
    print("set %s: %d problems factored and uploaded in %.1f s" % (args.set, len(S), time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    bs = [torch.from_numpy(p.b).cuda() for p in probs]
    xp = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p in probs]
    xb = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p in probs]
    torch.cuda.synchronize()

    # plain path, one solve after another (each handle warmed once: graph capture)
    for s, b, x in zip(S, bs, xp):
        s.solve(b, tol=args.tol, x_dev=x)
    torch.cuda.synchronize()
    plain = []
    its_plain = []
    for _ in range(args.reps):
        t1 = time.perf_counter()
        for s, b, x in zip(S, bs, xp):
            _, code, it, _, _ = s.solve(b, tol=args.tol, x_dev=x)
            its_plain.append(it)
        torch.cuda.synchronize()
        plain.append(time.perf_counter() - t1)
    print("plain: %.3f s per set" % min(plain), file=sys.stderr, flush=True)

    tu = R.Tuner(slack=1.0, iters=8)
    t1 = time.perf_counter()
    choice = tu.tune(S[0], bs[0])
    tune_s = time.perf_counter() - t1
    bt = R.Batch(len(S))
    out = {}
    for label, tile in [("default", None), ("tuned", choice["tile"])]:
        bt.solve(S, bs, args.tol, x_devs=xb, tile=tile)  # capture
        times = []
        for _ in range(args.reps):
            t1 = time.perf_counter()
            _, res = bt.solve(S, bs, args.tol, x_devs=xb, tile=tile)
            times.append(time.perf_counter() - t1)
        ok = sum(r["status"] == R.OK for r in res)
        dev = 0.0
        for p, a, c in zip(probs, xp, xb):
            A = p.scipy()
            e = c.cpu().numpy() - a.cpu().numpy()
            dev = max(dev, float(np.linalg.norm(A.T @ (A @ e)) / np.linalg.norm(A.T @ p.b)))
        out[label] = {"tile": list(tile) if tile else [1024, 4, 4], "solves_per_s": len(S) / min(times),
                      "s_per_set": min(times), "ok": ok, "max_iters": max(r["iters"] for r in res),
                      "max_ball_vs_plain": dev}
        print("%s: %.3f s per set" % (label, min(times)), file=sys.stderr, flush=True)
    # the autotuner's split: one batched launch beside the plain path
    tu2 = R.Tuner(slack=1.0, iters=4)
    xs, res, paths, tile = bt.solve_auto(tu2, S, bs, args.tol, x_devs=xb)  # tunes every signature once
    times = []
    for _ in range(args.reps):
        t1 = time.perf_counter()
        xs, res, paths, tile = bt.solve_auto(tu2, S, bs, args.tol, x_devs=xb)
        times.append(time.perf_counter() - t1)
    dev = 0.0
    for p, a, c in zip(probs, xp, xb):
        A = p.scipy()
        e = c.cpu().numpy() - a.cpu().numpy()
        dev = max(dev, float(np.linalg.norm(A.T @ (A @ e)) / np.linalg.norm(A.T @ p.b)))
    out["auto"] = {"tile": list(tile), "solves_per_s": len(S) / min(times), "s_per_set": min(times),
                   "ok": sum(r["status"] == R.OK for r in res), "batched": int(sum(1 for q in paths if q == 0)),
                   "plain": int(sum(1 for q in paths if q == 1)), "signatures": tu2.size(), "max_ball_vs_plain": dev}
    print("auto: %.3f s per set (%d batched, %d plain)" % (min(times), out["auto"]["batched"], out["auto"]["plain"]),
          file=sys.stderr, flush=True)
    tu2.close()
    line = {
        "metric": "independent least-squares solves/s, one launch (batched persistent) vs one solve at a time",
        "set": args.set, "k": len(S), "precision": args.precision, "tol": args.tol,
        "n_range": [int(min(p.n for p in probs)), int(max(p.n for p in probs))],
        "plain": {"solves_per_s": len(S) / min(plain), "s_per_set": min(plain),
                  "median_iters": float(np.median(its_plain))},
        "batched": out,
        "tuner": {"tile": list(choice["tile"]), "path": choice["path"], "tune_s": tune_s,
                  "batched_ms_per_iter": choice["batched_ms_per_iter"],
                  "plain_ms_per_iter": choice["plain_ms_per_iter"]},
    }
    print(json.dumps(line), flush=True)
    bt.close()
    tu.close()
    for s in S:
        s.close()


if __name__ == "__main__":
    main()
