"""GPU parity: every step of the hot path, through the C ABI, against the CPU oracle.

Tolerances (FP64 everywhere, unit roundoff eps = 2^-53 ~ 1.1e-16):
  * products y = A x: the GPU sums a row's k terms in a different order than
    the oracle's sequential sum, so |y_gpu - y_or| <= 2 k eps (|A| |x|)_i;
  * triangular solves: both sides are backward stable per row, so the GPU
    solution must have a componentwise backward error |T x - rhs| <=
    c eps (|T| |x| + |rhs|); for well-conditioned factors (mu = 1) the forward
    difference to the oracle is also checked, normwise, at 1e-10;
    the sync-free and level-scheduled schedules use identical per-row
    arithmetic and must agree bit for bit (the hybrid schedule sums a narrow
    row sequentially, so it is held to the oracle bounds only);
  * Algorithm 3 and Algorithm 1: 1e-10 (a few iterations, mu = 1 factors) and
    the 1e-8 relative bound on x for converged solves.
"""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps / 2
IMAX = 2**31 - 1


def torch_dev():
    import torch

    return torch


def to_dev(a):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    torch = torch_dev()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(R, prob, **params):
    return R.Solver.from_problem(prob, **params).upload()


def long_row_problem():
    # rows far longer than the mean exercise the segmented path of the products
    return gen.random_sparse(3000, 2500, k=4, seed=17, n_dense=3, dense_len=2400)


PROBLEMS = {
    "c1": lambda: gen.tiny_c1(),
    "c2-small": lambda: gen.by_name("c2-small"),
    "c3-mini": lambda: gen.by_name("c3-mini"),
    "long-rows": long_row_problem,
}


def oracle_for(prob, **kw):
    return oracle.factor_problem(prob, **kw)


# --------------------------------------------------------------- products


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_spmv(gpu_lib, name):
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = make(R, prob, smode=R.S_IDENTITY)
    F = oracle_for(prob, smode="identity")
    rng = np.random.default_rng(1)
    torch = torch_dev()
    for op, C in [(0, F.Ahat), (1, F.AhatT), (2, F.L2), (3, F.L2T)]:
        if C.nrows == 0 or C.ncols == 0:
            continue
        x = rng.standard_normal(C.ncols)
        y = torch.full((C.nrows,), np.nan, dtype=torch.float64, device="cuda")
        assert R.rsilu_spmv(S.h, op, to_dev(x), y) == R.OK
        got = to_host(y)
        want = C.matvec(x)
        absax = np.abs(C.scipy()) @ np.abs(x)
        k = np.maximum(np.diff(C.rowptr), 1)
        assert np.all(np.abs(got - want) <= 2 * k * EPS * absax + 1e-300), (name, op)
    S.close()


# --------------------------------------------------------------- triangular solves


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini"])
@pytest.mark.parametrize("mu", [0.1, 1.0])
def test_trsv(gpu_lib, name, mu):
    R = gpu_lib
    prob = PROBLEMS[name]()
    F = oracle_for(prob, mu=mu, smode="identity")
    rng = np.random.default_rng(2)
    torch = torch_dev()
    outs = {}
    for mode in (R.TRSV_SYNCFREE, R.TRSV_LEVELS, R.TRSV_HYBRID):
        S = make(R, prob, mu=mu, smode=R.S_IDENTITY, trsv=mode)
        for which, T, diag, lower in [(0, F.L1, None, True), (1, F.L1T, None, False), (2, F.U, F.Udiag, False)]:
            rhs = rng.standard_normal(prob.n) if mode == R.TRSV_SYNCFREE else outs[(which, "rhs")]
            outs[(which, "rhs")] = rhs
            x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
            assert R.rsilu_trsv(S.h, which, to_dev(rhs), x) == R.OK
            got = to_host(x)
            outs[(which, mode)] = got
            if mode == R.TRSV_LEVELS:
                continue
            assert np.all(np.isfinite(got)) or mu < 1.0
            want = oracle.lower_solve(T, rhs, diag) if lower else oracle.upper_solve(T, rhs, diag)
            # componentwise backward error
            Td = T.scipy()
            d = np.ones(prob.n) if diag is None else diag
            resid = Td @ got + d * got - rhs
            scale = np.abs(Td) @ np.abs(got) + np.abs(d * got) + np.abs(rhs)
            k = np.diff(T.rowptr) + 2
            fin = np.isfinite(scale) & (scale < 1e300)
            assert np.all(np.abs(resid[fin]) <= 4 * k[fin] * EPS * scale[fin]), (name, which)
            if mu == 1.0:
                assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want), (name, which)
        S.close()
    for which in (0, 1, 2):
        a, b = outs[(which, R.TRSV_SYNCFREE)], outs[(which, R.TRSV_LEVELS)]
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), which


# --------------------------------------------------------------- Algorithm 3


@pytest.mark.parametrize("name,smode", [("c1", "identity"), ("c1", "dense"), ("c2-small", "identity"),
                                        ("c3-mini", "identity"), ("c3-mini", "dense"), ("long-rows", "identity")])
def test_apply_alg3(gpu_lib, name, smode):
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = make(R, prob, mu=1.0, smode=R.S_DENSE if smode == "dense" else R.S_IDENTITY)
    F = oracle_for(prob, mu=1.0, smode=smode)
    r = np.random.default_rng(3).standard_normal(prob.m)
    torch = torch_dev()
    h = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    assert R.rsilu_apply(S.h, to_dev(r), h) == R.OK
    got = to_host(h)
    want = oracle.apply_alg3(F, r)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    S.close()


# --------------------------------------------------------------- Algorithm 1


def run_solve(R, prob, tol, **params):
    S = make(R, prob, **params)
    x, code, it, atr, rel = S.solve(to_dev(prob.b), tol=tol)
    out = to_host(x)
    S.close()
    return out, code, it, atr, rel


@pytest.mark.parametrize("name,smode", [("c1", "dense"), ("c1", "identity"), ("c3-mini", "dense")])
def test_solve_exact_factors_converge(gpu_lib, name, smode):
    """Complete factors: one step reaches the least-squares solution (Section 3.1) with the
    dense S~; with S^ = I the iteration must follow the oracle step for step."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    kw = dict(p=IMAX, tau=0.0, mu=1.0)
    maxit = 50 if smode == "dense" else 6
    x, code, it, atr, rel = run_solve(R, prob, 1e-8, smode=R.S_DENSE if smode == "dense" else R.S_IDENTITY,
                                      maxit=maxit, **kw)
    F = oracle.factor_problem(prob, p=10**9, tau=0.0, mu=1.0, smode=smode)
    res = oracle.pcgls(F, prob.b, tol=1e-8, maxit=maxit)
    assert it == res.iters
    assert code == {"ok": R.OK, "not_converged": R.NOT_CONVERGED, "breakdown": R.BREAKDOWN}[res.status]
    assert np.linalg.norm(x - res.x) <= 1e-8 * np.linalg.norm(res.x)
    assert abs(rel - res.atr_rel) <= 1e-6 * max(res.atr_rel, 1e-12) + 1e-14


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini", "long-rows"])
@pytest.mark.parametrize("mode", ["syncfree", "levels", "hybrid"])
def test_solve_fixed_iterations(gpu_lib, name, mode):
    """A few iterations of the ILUP(10, 1e-2) preconditioned CGLS with mu = 1 follow the oracle."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    maxit = 4
    trsv = {"syncfree": R.TRSV_SYNCFREE, "levels": R.TRSV_LEVELS, "hybrid": R.TRSV_HYBRID}[mode]
    x, code, it, atr, rel = run_solve(R, prob, 1e-14, mu=1.0, smode=R.S_IDENTITY, maxit=maxit, trsv=trsv)
    F = oracle.factor_problem(prob, mu=1.0, smode="identity")
    res = oracle.pcgls(F, prob.b, tol=1e-14, maxit=maxit)
    assert it == res.iters
    assert np.linalg.norm(x - res.x) <= 1e-8 * np.linalg.norm(res.x)
    assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm


def test_solve_deterministic(gpu_lib):
    R = gpu_lib
    prob = gen.by_name("c2-small")
    a = run_solve(R, prob, 1e-12, mu=1.0, maxit=20)
    b = run_solve(R, prob, 1e-12, mu=1.0, maxit=20)
    assert np.array_equal(a[0].view(np.int64), b[0].view(np.int64))
    assert a[2] == b[2]


def test_solve_edge_cases(gpu_lib):
    R = gpu_lib
    torch = torch_dev()
    prob = gen.random_sparse(40, 30, k=3, seed=5)
    S = make(R, prob)
    # b = 0: x = 0, no iteration, OK
    x, code, it, atr, rel = S.solve(torch.zeros(prob.m, dtype=torch.float64, device="cuda"))
    assert code == R.OK and it == 0 and np.all(to_host(x) == 0)
    # aliasing and NULL arguments are rejected
    b = to_dev(prob.b)
    assert R.lib().rsilu_solve(S.h, R._dev(b), 1e-8, R._dev(b), None, None, None, None) == R.EINVAL
    assert R.rsilu_spmv(S.h, 7, b, torch.empty(prob.m, dtype=torch.float64, device="cuda")) == R.EINVAL
    S.close()
    # maxit = 1 stops as NOT_CONVERGED with one iteration done
    x, code, it, atr, rel = run_solve(R, prob, 1e-14, maxit=1)
    assert code == R.NOT_CONVERGED and it == 1
