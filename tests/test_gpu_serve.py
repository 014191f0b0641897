"""The serving runtime (include/rsilu_serve.h) on the GPU: every result equals the
same request solved alone (by rsilu_solve on the plain path, by a lone batched launch
with the same tile on the batched path), and admission by device footprint behaves."""

import numpy as np
import pytest

import gen

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
