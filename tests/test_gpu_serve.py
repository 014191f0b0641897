"""The serving runtime (include/rsilu_serve.h) on the GPU: every result equals the
same request solved alone (by rsilu_solve on the plain path, by a lone batched launch
with the same tile on the batched path), admission by device footprint behaves, and served
requests with the M_b correction follow the oracle (four LSQR steps; converged solves in
its stop-test ball)."""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def requests():
    sizes = [(1500, 2400, 0), (4000, 5200, 0), (2500, 4500, 8), (6000, 7000, 0), (3000, 3500, 12),
             (5000, 9000, 0), (1200, 2300, 0), (7000, 9500, 0), (2000, 2600, 10), (4500, 6000, 0)]
    return [gen.served_request(n, m, 40 + i, n_dense=nd) for i, (n, m, nd) in enumerate(sizes)]


PARAMS = dict(mu=1.0, form=1, smode=2)  # Algorithm 2 form, no correction


@pytest.mark.parametrize("precision", [0, 1])
def test_served_results_equal_lone_solves(gpu_lib, precision):
    R = gpu_lib
    import torch

    probs = requests()
    srv = R.Server(hbm_bytes=512 << 20, slots=4, setup_threads=4)
    ids = {}
    for i, p in enumerate(probs):
        ids[srv.submit(p.m, p.n, p.rowptr, p.col, p.val, p.b, tol=1e-8, precision=precision, **PARAMS)] = i
    srv.drain()
    got = {}
    while len(got) < len(probs):
        for res, x in srv.poll(wait_ms=1000):
            got[ids[res["id"]]] = (res, x)
    srv.close()
    for i, p in enumerate(probs):
        res, x = got[i]
        assert res["status"] == R.OK, (i, res)
        S = R.Solver.from_problem(p, precision=precision, **PARAMS).upload()
        xl, code, it, atr, rel = S.solve(torch.from_numpy(p.b).cuda(), tol=1e-8)
        lone = xl.cpu().numpy()
        S.close()
        assert code == R.OK and it == res["iters"]
        assert np.array_equal(lone.view(np.int64), x.view(np.int64)), i
        assert res["atr_rel"] <= 2e-8


def test_request_larger_than_arena_fails_alone(gpu_lib):
    R = gpu_lib
    srv = R.Server(hbm_bytes=1 << 20, slots=2, setup_threads=2)
    big = gen.served_request(20000, 30000, 3)
    small = gen.served_request(300, 450, 4)
    srv.submit(big.m, big.n, big.rowptr, big.col, big.val, big.b, **PARAMS)
    srv.submit(small.m, small.n, small.rowptr, small.col, small.val, small.b, **PARAMS)
    srv.drain()
    out = {r["id"]: r for r, _ in srv.poll(max_results=8)}
    srv.close()
    assert out[0]["status"] == R.ENOMEM
    assert out[1]["status"] == R.OK and out[1]["device_bytes"] <= 1 << 20


LSQR = dict(mu=1.0, form=1, smode=2, krylov=1)  # accepted by the batched kernel


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tune_slack", [0.0, 8.0])
def test_batched_serving_equals_lone_solves(gpu_lib, precision, tune_slack):
    """Requests admitted together share persistent launches; each result is bit for bit
    that of the same request solved alone on its reported path (and tile)."""
    R = gpu_lib
    import torch

    probs = requests()
    srv = R.Server(hbm_bytes=512 << 20, slots=2, setup_threads=4, batch_max=6, tune_slack=tune_slack)
    ids = {}
    for i, p in enumerate(probs):
        ids[srv.submit(p.m, p.n, p.rowptr, p.col, p.val, p.b, tol=1e-8, precision=precision, **LSQR)] = i
    srv.drain()
    got = {}
    while len(got) < len(probs):
        for res, x in srv.poll(wait_ms=1000):
            got[ids[res["id"]]] = (res, x)
    srv.close()
    sizes = []
    bt = R.Batch(1)
    for i, p in enumerate(probs):
        res, x = got[i]
        assert res["status"] == R.OK, (i, res)
        assert res["path"] in (0, 1) and res["launch_size"] >= 1
        if tune_slack == 0.0:
            assert res["path"] == 0 and res["tile"] == (1024, 4, 4)
        S = R.Solver.from_problem(p, precision=precision, **LSQR).upload()
        b = torch.from_numpy(p.b).cuda()
        if res["path"] == 0:
            xs, rr = bt.solve([S], [b], 1e-8, tile=res["tile"])
            lone, it = xs[0].cpu().numpy(), rr[0]["iters"]
        else:
            xl, code, it, atr, rel = S.solve(b, tol=1e-8)
            lone = xl.cpu().numpy()
        S.close()
        assert it == res["iters"], i
        assert np.array_equal(lone.view(np.int64), x.view(np.int64)), i
        assert res["atr_rel"] <= 2e-8
        sizes.append(res["launch_size"])
    bt.close()
    print("launch sizes:", sizes)


# LSQR with the degree-2 Chebyshev M_b through the explicit Y~ (input scaled where two steps
# cannot cover S~'s interval: the requests with dense rows)
CHEB2 = dict(mu=1.0, form=1, smode=4, krylov=1, ystore=1, ytau=1e-2, poly_degree=2)


def serve(R, probs, tol, precision, **kw):
    # one slot; after admitting a request it waits (up to 5 s) for the others still in setup
    srv = R.Server(hbm_bytes=512 << 20, slots=1, setup_threads=4, batch_max=10, tune_slack=0.0,
                   batch_wait_ms=5000.0)
    ids = {}
    for i, p in enumerate(probs):
        ids[srv.submit(p.m, p.n, p.rowptr, p.col, p.val, p.b, tol=tol, precision=precision, **kw)] = i
    srv.drain()
    got = {}
    while len(got) < len(probs):
        for res, x in srv.poll(wait_ms=1000):
            got[ids[res["id"]]] = (res, x)
    srv.close()
    return got


@pytest.mark.parametrize("precision", [0, 1])
def test_served_correction_follows_oracle(gpu_lib, precision):
    """Served with shared batched launches (one slot, a batching window, up to ten requests per
    admission): each
    result equals its lone batched launch bit for bit, lies in the oracle's stop-test ball
    (FP64: iterations within 2% of the oracle's); four steps of a sample against the oracle's
    (x to 1e-8 in FP64; to 1e-3 with the FP32 preconditioner, whose applications are within
    about 1e-7 of the FP64 oracle's)."""
    R = gpu_lib
    import torch

    probs = requests()
    got = serve(R, probs, 1e-8, precision, **CHEB2)
    bt = R.Batch(1)
    sizes = []
    for i, p in enumerate(probs):
        res, x = got[i]
        assert res["status"] == R.OK and res["path"] == 0, (i, res)
        S = R.Solver.from_problem(p, precision=precision, **CHEB2).upload()
        xs, rr = bt.solve([S], [torch.from_numpy(p.b).cuda()], 1e-8, tile=res["tile"])
        S.close()
        assert rr[0]["iters"] == res["iters"] and np.array_equal(xs[0].cpu().numpy().view(np.int64), x.view(np.int64))
        F = oracle.factor_problem(p, mu=1.0, smode="cheb", ystore=True, ytau=1e-2, poly_degree=2)
        o = oracle.lsqr_m(F, p.b, tol=1e-8, maxit=2000)
        A = p.scipy()
        atb = np.linalg.norm(A.T @ p.b)
        assert o.status == "ok"
        if precision == 0:
            assert abs(res["iters"] - o.iters) <= max(1, int(0.02 * o.iters)), (i, res["iters"], o.iters)
        assert np.linalg.norm(A.T @ (p.b - A @ x)) <= 2e-8 * atb, i
        assert np.linalg.norm(A.T @ (A @ (x - o.x))) <= 4e-8 * atb, i
        sizes.append(res["launch_size"])
    bt.close()
    print("precision %d launch sizes %s" % (precision, sizes))
    assert max(sizes) >= 2  # the window made admissions share launches
    sample = probs[:4]
    got = serve(R, sample, 1e-14, precision, maxit=4, **CHEB2)
    for i, p in enumerate(sample):
        res, x = got[i]
        F = oracle.factor_problem(p, mu=1.0, smode="cheb", ystore=True, ytau=1e-2, poly_degree=2)
        o = oracle.lsqr_m(F, p.b, tol=1e-14, maxit=4)
        err = np.linalg.norm(x - o.x) / np.linalg.norm(o.x)
        print("request %d precision %d: four steps, x rel diff %.1e" % (i, precision, err))
        assert res["iters"] == o.iters == 4
        assert err <= (1e-8 if precision == 0 else 1e-3), (i, err)
