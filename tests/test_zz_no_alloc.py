"""The allocation-free batched solve (rsilu_batch_solve_static, include/rsilu_batch.h) against
the batched solve with a batch object (rsilu_batch_solve), through the C ABI.

Both run the same kernel on the same descriptors (only where the descriptor table lives
differs), so every solution and outcome must be identical bit for bit: two calls in a row,
the second with fewer and smaller problems than the first (the fixed table keeps the first
call's contents), FP64 and FP32 preconditioners; then the size limit and argument checks.
"""

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

LSQR = dict(mu=1.0, form=1, krylov=1, smode=2)  # Algorithm 2 form, LSQR, S^ none


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run_both(R, probs, precision, tile=None):
    import torch

    S = [R.Solver.from_problem(p, precision=precision, **LSQR).upload() for p in probs]
    bs = [to_dev(p.b) for p in probs]
    tols = [1e-8] * len(probs)
    x_obj = [torch.zeros(p.n, dtype=torch.float64, device="cuda") for p in probs]
    x_fix = [torch.full((p.n,), float("nan"), dtype=torch.float64, device="cuda") for p in probs]
    bt = R.Batch(len(probs))
    code_obj, res_obj = bt.solve_raw([s.h for s in S], bs, tols, x_obj, tile=tile)
    bt.close()
    code_fix, res_fix = R.rsilu_batch_solve_static([s.h for s in S], bs, tols, x_fix, tile=tile)
    torch.cuda.synchronize()
    for s in S:
        s.close()
    return (code_obj, res_obj, [x.cpu().numpy() for x in x_obj]), (code_fix, res_fix, [x.cpu().numpy() for x in x_fix])


@pytest.mark.parametrize("precision", [0, 1])
def test_static_batch_equals_batch_object(gpu_lib, precision):
    R = gpu_lib
    first = [gen.tiny_c1(), gen.served_request(5000, 6000, 32), gen.served_request(3000, 4500, 31, n_dense=12),
             gen.tiny_c1(seed=7), gen.by_name("c2-small")]
    second = [gen.served_request(2500, 3000, 33), gen.tiny_c1(seed=8)]  # fewer and smaller
    for probs, tile in ((first, None), (second, (512, 8, 1))):
        (co, ro, xo), (cf, rf, xf) = run_both(R, probs, precision, tile)
        print(f"precision {precision}, {len(probs)} problems: status {co} / {cf}, iterations "
              f"{[r['iters'] for r in ro]} / {[r['iters'] for r in rf]}")
        assert co == cf == R.OK
        for a, b_, r1, r2 in zip(xo, xf, ro, rf):
            assert r1 == r2
            assert r1["status"] == R.OK
            assert np.array_equal(a, b_)


def test_static_batch_limits(gpu_lib):
    import torch

    R = gpu_lib
    L = R.lib()
    mx = L.rsilu_batch_static_max()
    assert mx == 256
    res = (R.rsilu_batch_result_t * 1)()
    assert L.rsilu_batch_solve_static(mx + 1, None, None, None, None, None, res, None) == R.EINVAL
    assert L.rsilu_batch_solve_static(-1, None, None, None, None, None, res, None) == R.EINVAL
    assert L.rsilu_batch_solve_static(0, None, None, None, None, None, res, None) == R.OK
    p = gen.tiny_c1()
    S = R.Solver.from_problem(p, **LSQR).upload()
    b = to_dev(p.b)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda")
    code, _ = R.rsilu_batch_solve_static([S.h, S.h], [b, b], [1e-8, 1e-8], [x, x])
    assert code == R.EINVAL  # a repeated handle
    code, _ = R.rsilu_batch_solve_static([S.h], [b], [1e-8], [x], tile=(256, 2, 1))
    assert code == R.EINVAL  # a tile that is not compiled
    S.close()
    # a handle the batched kernel does not take (the A2 correction)
    T = R.Solver.from_problem(p, mu=1.0, form=1, smode=R.S_CG).upload()
    code, _ = R.rsilu_batch_solve_static([T.h], [b], [1e-8], [x])
    assert code == R.EINVAL
    T.close()
