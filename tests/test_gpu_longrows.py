"""Rows long enough for the segmented products (several 4096-entry segments per row, reduced in a
fixed order and finished on the device), through the C ABI, against the oracle.

The problem is the sparse-dense recipe's long-row feature at a size that sets up in seconds:
40000 x 30000 with 4 sparse entries per row (a transversal on the first 30000 rows) and 4
fully dense rows of 30000 entries (Section 3.3's sparse-dense problems). With mu = 1 its dense
rows are pivoted into A1; A_hat then has rows of 30000 entries (8 segments), the explicit Y~
rows of up to 11372 (3 segments) and L2 rows of up to 1426 entries.

* products with A_hat, A_hat^T, L2, L2^T, Y~ and Y~^T: componentwise |y - y_or| <= 2 k eps (|A| |x|)_i;
* four LSQR steps (A1 only) and four Algorithm 1 steps (Algorithm 2, CG(8) on S~ through the
  explicit Y~) against the oracle, x within 1e-8 (the oracle's own x moves by 3e-13 under a
  change of its inner-product order here).
"""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def prob():
    return gen.random_sparse(40000, 30000, k=4, seed=29, n_dense=4, dense_len=30000)


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_long_row_products(gpu_lib, prob):
    import torch

    R = gpu_lib
    F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=8, ystore=True, ytau=1e-2)
    assert np.diff(F.Ahat.rowptr).max() >= 3 * 4096 and np.diff(F.Y.rowptr).max() >= 2 * 4096
    S = R.Solver.from_problem(prob, mu=1.0, form=R.FORM_ALG2, smode=R.S_CG, cg_steps=8, ystore=R.Y_EXPLICIT,
                              ytau=1e-2).upload()
    rng = np.random.default_rng(81)
    for op, C in ((0, F.Ahat), (1, F.AhatT), (2, F.L2), (3, F.L2T), (4, F.Y), (5, F.YT)):
        x = rng.standard_normal(C.ncols)
        y = torch.empty(C.nrows, dtype=torch.float64, device="cuda")
        assert R.rsilu_spmv(S.h, op, to_dev(x), y) == R.OK
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        want = C.matvec(x)
        k = np.diff(C.rowptr)
        bound = 2 * k * EPS * (abs(C.scipy()) @ np.abs(x))
        worst = np.max(np.abs(got - want) / (bound + 1e-300))
        print(f"op {op}: longest row {k.max()}, worst error / bound {worst:.2e}")
        assert np.all(np.abs(got - want) <= bound + 1e-300), op
    S.close()


@pytest.mark.parametrize("cfg", ["lsqr-a1", "pcgls-cg8"])
def test_long_row_four_steps(gpu_lib, prob, cfg):
    R = gpu_lib
    if cfg == "lsqr-a1":
        kw = dict(mu=1.0, form=R.FORM_ALG2, smode=R.S_NONE, krylov=R.KRYLOV_LSQR)
        F = oracle.factor_problem(prob, mu=1.0, smode="none")
        res = oracle.lsqr_m(F, prob.b, tol=1e-14, maxit=4)
    else:
        kw = dict(mu=1.0, form=R.FORM_ALG2, smode=R.S_CG, cg_steps=8, ystore=R.Y_EXPLICIT, ytau=1e-2)
        F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=8, ystore=True, ytau=1e-2)
        res = oracle.pcgls(F, prob.b, tol=1e-14, maxit=4, form="alg2")
    S = R.Solver.from_problem(prob, maxit=4, **kw).upload()
    x, code, it, atr, rel = S.solve(to_dev(prob.b), tol=1e-14)
    import torch

    torch.cuda.synchronize()
    got = x.cpu().numpy()
    S.close()
    err = np.linalg.norm(got - res.x) / np.linalg.norm(res.x)
    print(f"{cfg}: its {it} / {res.iters}, x rel diff {err:.2e}")
    assert it == res.iters == 4
    assert err <= 1e-8
    assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm
