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
  * one preconditioner application (Algorithm 3 or Algorithm 2), element by element:
    |h - h_or| <= rtol |h_or| + atol ||h_or||_inf (apply_tol below);
  * Algorithm 1 and LSQR: four steps with x within 1e-8 (the sparse-dense mini case in
    ||b - A x||, see test_solve_alg2_fixed_iterations); whole solves to 1e-8 with iteration
    counts within 2%, the true ||A^T r|| at the tolerance and x in the oracle's stop-test
    ball, and again at tol 1e-12 with x within 1e-6 (grid workload).
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


def elementwise(got, want, rtol, atol):
    """Largest ratio of |got - want| to rtol |want| + atol ||want||_inf (<= 1 passes)."""
    bound = rtol * np.abs(want) + atol * np.max(np.abs(want))
    return float(np.max(np.abs(got - want) / bound))


def apply_tol(name, cg=False):
    """Element-by-element bound of one preconditioner application: (1e-10, 1e-13) when only
    triangular solves and products separate the two sides, (1e-8, 1e-11) with CG steps on S~
    (exact line searches pass rounding differences on), 100x wider on the sparse-dense mini
    case, whose factors have kappa(L1 U) = 2.6e9 (against 4.3 on c1)."""
    rtol, atol = (1e-8, 1e-11) if cg else (1e-10, 1e-13)
    return (100 * rtol, 100 * atol) if name == "c3-mini" else (rtol, atol)


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
    ratio = elementwise(got, want, *apply_tol(name))
    print(f"{name} alg3 {smode}: elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
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


# --------------------------------------------------------------- Algorithm 2 form and S^ = none


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini"])
def test_trsv_ut(gpu_lib, name):
    """U^T x = rhs (forward, diagonal of U) in all three schedules."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    F = oracle_for(prob, mu=1.0, smode="identity")
    rhs = np.random.default_rng(6).standard_normal(prob.n)
    want = oracle.lower_solve(F.UT, rhs, F.Udiag)
    torch = torch_dev()
    outs = {}
    for mode in (R.TRSV_SYNCFREE, R.TRSV_LEVELS, R.TRSV_HYBRID):
        S = make(R, prob, mu=1.0, smode=R.S_IDENTITY, trsv=mode)
        x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        assert R.rsilu_trsv(S.h, R.T_UT, to_dev(rhs), x) == R.OK
        got = to_host(x)
        outs[mode] = got
        Td = F.UT.scipy()
        resid = Td @ got + F.Udiag * got - rhs
        scale = np.abs(Td) @ np.abs(got) + np.abs(F.Udiag * got) + np.abs(rhs)
        k = np.diff(F.UT.rowptr) + 2
        assert np.all(np.abs(resid) <= 4 * k * EPS * scale), (name, mode)
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want), (name, mode)
        S.close()
    assert np.array_equal(outs[R.TRSV_SYNCFREE].view(np.int64), outs[R.TRSV_LEVELS].view(np.int64))


@pytest.mark.parametrize("name,smode", [("c1", "none"), ("c1", "identity"), ("c1", "dense"),
                                        ("c2-small", "none"), ("c2-small", "identity"),
                                        ("c3-mini", "dense"), ("long-rows", "identity")])
@pytest.mark.parametrize("mode", ["syncfree", "hybrid"])
def test_apply_alg2(gpu_lib, name, smode, mode):
    R = gpu_lib
    prob = PROBLEMS[name]()
    sm = {"none": R.S_NONE, "identity": R.S_IDENTITY, "dense": R.S_DENSE}[smode]
    trsv = {"syncfree": R.TRSV_SYNCFREE, "hybrid": R.TRSV_HYBRID}[mode]
    S = make(R, prob, mu=1.0, smode=sm, trsv=trsv)
    F = oracle_for(prob, mu=1.0, smode=smode)
    z = np.random.default_rng(7).standard_normal(prob.n)
    torch = torch_dev()
    h = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
    got = to_host(h)
    want = oracle.apply_alg2(F, z)
    ratio = elementwise(got, want, *apply_tol(name))
    print(f"{name} alg2 {smode} {mode}: elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
    S.close()


@pytest.mark.parametrize("name", ["c1", "c2-small"])
def test_apply_alg3_none(gpu_lib, name):
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = make(R, prob, mu=1.0, smode=R.S_NONE)
    F = oracle_for(prob, mu=1.0, smode="none")
    r = np.random.default_rng(8).standard_normal(prob.m)
    torch = torch_dev()
    h = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    assert R.rsilu_apply(S.h, to_dev(r), h) == R.OK
    want = oracle.apply_alg3(F, r)
    assert elementwise(to_host(h), want, *apply_tol(name)) <= 1.0
    S.close()


@pytest.mark.parametrize("name,smode", [("c1", "none"), ("c1", "dense"), ("c2-small", "none"),
                                        ("c2-small", "identity"), ("c3-mini", "dense"), ("long-rows", "none")])
@pytest.mark.parametrize("mode", ["syncfree", "levels", "hybrid"])
def test_solve_alg2_fixed_iterations(gpu_lib, name, smode, mode):
    """A few iterations of Algorithm 1 with Algorithm 2 follow the oracle."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    maxit = 4
    sm = {"none": R.S_NONE, "identity": R.S_IDENTITY, "dense": R.S_DENSE}[smode]
    trsv = {"syncfree": R.TRSV_SYNCFREE, "levels": R.TRSV_LEVELS, "hybrid": R.TRSV_HYBRID}[mode]
    x, code, it, atr, rel = run_solve(R, prob, 1e-14, mu=1.0, smode=sm, maxit=maxit, trsv=trsv, form=R.FORM_ALG2)
    F = oracle.factor_problem(prob, mu=1.0, smode=smode)
    res = oracle.pcgls(F, prob.b, tol=1e-14, maxit=maxit, form="alg2")
    assert it == res.iters
    if name == "c3-mini":
        # Its factors (dense rows pivoted into A1 at mu = 1, kappa(L1 U) = 2.6e9) make x after
        # four steps move by 2.4e-4 relative, and ||A^T r|| by 2.9e-6, when the oracle merely
        # sums its inner products in another order; ||b - A x|| moves by 6.9e-10. It is held
        # to ||b - A x|| at 1e-7 and ||A^T r|| at 1e-4 (a wrong kernel is off by far more).
        A = prob.scipy()
        rn, rn_or = np.linalg.norm(prob.b - A @ x), np.linalg.norm(prob.b - A @ res.x)
        assert abs(rn - rn_or) <= 1e-7 * rn_or
        assert abs(atr - res.atr_norm) <= 1e-4 * res.atr_norm
    else:
        assert np.linalg.norm(x - res.x) <= 1e-8 * np.linalg.norm(res.x)
        assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm


@pytest.mark.parametrize("name", ["c1", "c2-small"])
def test_solve_alg2_converges_like_oracle(gpu_lib, name):
    """Whole solves to tol = 1e-8 with the uncorrected Algorithm 2 form. Iteration counts
    agree within 2% (at least one). Both solutions satisfy the stop test, so their
    difference e obeys ||A^T A e|| <= 2 tol ||A^T b||: that is checked with the true
    residuals. On the tiny workload (well conditioned) x itself must agree to 1e-8; the
    grid workload's columns span six decades of scale, so its x is only determined to
    about tol ||A^T b|| / sigma_min^2 and the residual checks carry the comparison."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    tol = 1e-8
    x, code, it, atr, rel = run_solve(R, prob, tol, mu=1.0, smode=R.S_NONE, maxit=2000, form=R.FORM_ALG2)
    F = oracle.factor_problem(prob, mu=1.0, smode="none")
    res = oracle.pcgls(F, prob.b, tol=tol, maxit=2000, form="alg2")
    assert res.status == "ok" and code == R.OK
    assert abs(it - res.iters) <= max(1, int(0.02 * res.iters))
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    assert np.linalg.norm(A.T @ (prob.b - A @ x)) <= 2 * tol * atb
    assert abs(atr - np.linalg.norm(A.T @ (prob.b - A @ x))) <= 1e-6 * atr + 1e-300
    e = x - res.x
    assert np.linalg.norm(A.T @ (A @ e)) <= 4 * tol * atb
    print("%s: gpu its %d oracle its %d, |x - x_or|/|x_or| = %.3e" % (
        name, it, res.iters, np.linalg.norm(e) / np.linalg.norm(res.x)))
    if name == "c1":
        assert np.linalg.norm(e) <= 1e-8 * np.linalg.norm(res.x)
    # both sides again at tol 1e-12, where x is determined far better: x to 1e-6
    x2, code2, it2, _, _ = run_solve(R, prob, 1e-12, mu=1.0, smode=R.S_NONE, maxit=2000, form=R.FORM_ALG2)
    res2 = oracle.pcgls(F, prob.b, tol=1e-12, maxit=2000, form="alg2")
    e2 = np.linalg.norm(x2 - res2.x) / np.linalg.norm(res2.x)
    print("%s at tol 1e-12: gpu its %d oracle its %d, |x - x_or|/|x_or| = %.3e" % (name, it2, res2.iters, e2))
    assert code2 == R.OK and res2.status == "ok"
    assert abs(it2 - res2.iters) <= max(1, int(0.02 * res2.iters))
    assert e2 <= 1e-6


# --------------------------------------------------------------- FP32 preconditioner

EPS32 = np.finfo(np.float32).eps / 2


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini"])
@pytest.mark.parametrize("mode", ["hybrid", "levels"])
def test_trsv_fp32(gpu_lib, name, mode):
    """FP32 triangular solves: componentwise backward error in FP32 with respect to the
    FP32-rounded factor and right-hand side, |T32 x - rhs32| <= 4 k eps32 (|T32| |x| + |rhs32|),
    evaluated in FP64 (x is exactly representable there)."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    trsv = {"hybrid": R.TRSV_HYBRID, "levels": R.TRSV_LEVELS}[mode]
    S = make(R, prob, mu=1.0, smode=R.S_NONE, trsv=trsv, precision=R.PREC_FP32)
    F = oracle_for(prob, mu=1.0, smode="none")
    rhs = np.random.default_rng(10).standard_normal(prob.n)
    rhs32 = rhs.astype(np.float32).astype(np.float64)
    torch = torch_dev()
    for which, T, diag in [(R.T_L1, F.L1, None), (R.T_L1T, F.L1T, None), (R.T_U, F.U, F.Udiag),
                           (R.T_UT, F.UT, F.Udiag)]:
        x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        assert R.rsilu_trsv(S.h, which, to_dev(rhs), x) == R.OK
        got = to_host(x)
        assert np.array_equal(got, got.astype(np.float32).astype(np.float64))
        T32 = T.scipy().astype(np.float32).astype(np.float64)
        d32 = np.ones(prob.n) if diag is None else diag.astype(np.float32).astype(np.float64)
        resid = T32 @ got + d32 * got - rhs32
        scale = abs(T32) @ np.abs(got) + np.abs(d32 * got) + np.abs(rhs32)
        k = np.diff(T.rowptr) + 2
        assert np.all(np.abs(resid) <= 4 * k * EPS32 * scale), (name, which)
    S.close()


def fp32_apply_error(R, prob, smode, form):
    """Relative difference of the FP32 application to the FP64 oracle's."""
    sm = {"none": R.S_NONE, "identity": R.S_IDENTITY}[smode]
    S = make(R, prob, mu=1.0, smode=sm, precision=R.PREC_FP32)
    F = oracle_for(prob, mu=1.0, smode=smode)
    torch = torch_dev()
    h = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(11)
    if form == "alg2":
        z = rng.standard_normal(prob.n)
        assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
        want = oracle.apply_alg2(F, z)
    else:
        r = rng.standard_normal(prob.m)
        assert R.rsilu_apply(S.h, to_dev(r), h) == R.OK
        want = oracle.apply_alg3(F, r)
    got = to_host(h)
    S.close()
    return np.linalg.norm(got - want) / np.linalg.norm(want)


@pytest.mark.parametrize("name,smode,form", [("c1", "none", "alg2"), ("c1", "identity", "alg2"),
                                             ("c1", "identity", "alg3"), ("c2-small", "none", "alg2"),
                                             ("c2-small", "identity", "alg3"), ("long-rows", "none", "alg2")])
def test_apply_fp32(gpu_lib, name, smode, form):
    """Stated bound for the FP32 preconditioner against the FP64 oracle: relative error
    <= 1e-4 (FP32 rounding of the factors and of every operation, eps32 = 6e-8, times the
    growth through four to six triangular solves of these mu = 1 factors)."""
    err = fp32_apply_error(gpu_lib, PROBLEMS[name](), smode, form)
    print("%s %s %s: |h32 - h64| / |h64| = %.2e" % (name, smode, form, err))
    assert err <= 1e-4


@pytest.mark.parametrize("name", ["c1", "c2-small"])
def test_solve_fp32_converges(gpu_lib, name):
    """Whole solves with the FP32 preconditioner (Algorithm 2, no correction): FP64 Krylov
    recurrences still reach tol = 1e-8 on the true residual; the solution lies in the same
    stop-test ball as the FP64 oracle's, ||A^T A (x32 - x64)|| <= 4 tol ||A^T b||."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    tol = 1e-8
    x, code, it, atr, rel = run_solve(R, prob, tol, mu=1.0, smode=R.S_NONE, maxit=2000, form=R.FORM_ALG2,
                                      precision=R.PREC_FP32)
    F = oracle.factor_problem(prob, mu=1.0, smode="none")
    res = oracle.pcgls(F, prob.b, tol=tol, maxit=2000, form="alg2")
    assert code == R.OK and res.status == "ok"
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    assert np.linalg.norm(A.T @ (prob.b - A @ x)) <= 2 * tol * atb
    e = x - res.x
    assert np.linalg.norm(A.T @ (A @ e)) <= 4 * tol * atb
    print("%s: fp32-preconditioner its %d, fp64 oracle its %d, |x - x_or|/|x_or| = %.2e" % (
        name, it, res.iters, np.linalg.norm(e) / np.linalg.norm(res.x)))


# --------------------------------------------------------------- S^ by CG on S~ (Table 3(a))


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini", "long-rows"])
@pytest.mark.parametrize("form,steps,mode", [("alg3", 2, "hybrid"), ("alg2", 2, "hybrid"), ("alg3", 5, "levels")])
def test_apply_cg(gpu_lib, name, form, steps, mode):
    R = gpu_lib
    prob = PROBLEMS[name]()
    trsv = {"hybrid": R.TRSV_HYBRID, "levels": R.TRSV_LEVELS}[mode]
    S = make(R, prob, mu=1.0, smode=R.S_CG, cg_steps=steps, trsv=trsv)
    F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=steps)
    torch = torch_dev()
    h = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(12)
    if form == "alg3":
        r = rng.standard_normal(prob.m)
        assert R.rsilu_apply(S.h, to_dev(r), h) == R.OK
        want = oracle.apply_alg3(F, r)
    else:
        z = rng.standard_normal(prob.n)
        assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
        want = oracle.apply_alg2(F, z)
    ratio = elementwise(to_host(h), want, *apply_tol(name, cg=True))
    print(f"{name} {form} CG({steps}) {mode}: elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
    S.close()


@pytest.mark.parametrize("name", ["c1", "c2-small"])
def test_solve_cg_fixed_iterations(gpu_lib, name):
    """Four iterations of Algorithm 1 with Algorithm 3 and CG(2) on S~ follow the oracle."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    x, code, it, atr, rel = run_solve(R, prob, 1e-14, mu=1.0, smode=R.S_CG, cg_steps=2, maxit=4)
    F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=2)
    res = oracle.pcgls(F, prob.b, tol=1e-14, maxit=4)
    assert it == res.iters
    assert np.linalg.norm(x - res.x) <= 1e-8 * np.linalg.norm(res.x)
    assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm


# --------------------------------------------------------------- LSQR (M-inner-product form)


@pytest.mark.parametrize("name,smode", [("c1", "none"), ("c1", "dense"), ("c2-small", "none"), ("long-rows", "none")])
@pytest.mark.parametrize("mode", ["hybrid", "levels"])
def test_lsqr_fixed_iterations(gpu_lib, name, smode, mode):
    """Four LSQR steps follow the oracle's lsqr_m."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    sm = {"none": R.S_NONE, "dense": R.S_DENSE}[smode]
    trsv = {"hybrid": R.TRSV_HYBRID, "levels": R.TRSV_LEVELS}[mode]
    x, code, it, atr, rel = run_solve(R, prob, 1e-14, mu=1.0, smode=sm, maxit=4, trsv=trsv, form=R.FORM_ALG2,
                                      krylov=R.KRYLOV_LSQR)
    F = oracle.factor_problem(prob, mu=1.0, smode=smode)
    res = oracle.lsqr_m(F, prob.b, tol=1e-14, maxit=4)
    assert it == res.iters == 4 and code == R.NOT_CONVERGED
    assert np.linalg.norm(x - res.x) <= 1e-8 * np.linalg.norm(res.x)
    assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm


@pytest.mark.parametrize("name,precision", [("c1", 0), ("c2-small", 0), ("c2-small", 1)])
def test_lsqr_converges_like_oracle(gpu_lib, name, precision):
    """Whole LSQR solves to tol = 1e-8: iteration counts within 2% (at least one) of the
    oracle's for the FP64 preconditioner; the true ||A^T r|| at the tolerance (the stop test
    uses the recurrence estimate, so 2 tol is allowed) and the solution in the oracle's
    stop-test ball, ||A^T A (x - x_or)|| <= 4 tol ||A^T b||."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    tol = 1e-8
    x, code, it, atr, rel = run_solve(R, prob, tol, mu=1.0, smode=R.S_NONE, maxit=2000, form=R.FORM_ALG2,
                                      krylov=R.KRYLOV_LSQR, precision=precision)
    F = oracle.factor_problem(prob, mu=1.0, smode="none")
    res = oracle.lsqr_m(F, prob.b, tol=tol, maxit=2000)
    assert code == R.OK and res.status == "ok"
    if precision == 0:
        assert abs(it - res.iters) <= max(1, int(0.02 * res.iters))
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    assert np.linalg.norm(A.T @ (prob.b - A @ x)) <= 2 * tol * atb
    e = x - res.x
    assert np.linalg.norm(A.T @ (A @ e)) <= 4 * tol * atb
    print("%s precision %d: LSQR its %d, oracle its %d" % (name, precision, it, res.iters))
    if precision == 0:
        # both sides again at tol 1e-12: x to 1e-6
        x2, code2, it2, _, _ = run_solve(R, prob, 1e-12, mu=1.0, smode=R.S_NONE, maxit=2000, form=R.FORM_ALG2,
                                         krylov=R.KRYLOV_LSQR)
        res2 = oracle.lsqr_m(F, prob.b, tol=1e-12, maxit=2000)
        e2 = np.linalg.norm(x2 - res2.x) / np.linalg.norm(res2.x)
        print("%s at tol 1e-12: LSQR its %d, oracle its %d, |x - x_or|/|x_or| = %.3e" % (name, it2, res2.iters, e2))
        assert code2 == R.OK and res2.status == "ok"
        assert abs(it2 - res2.iters) <= max(1, int(0.02 * res2.iters))
        assert e2 <= 1e-6


# --------------------------------------------------------------- captured iteration graphs


@pytest.mark.parametrize("name", ["c1", "c2-small", "long-rows"])
@pytest.mark.parametrize("cfg", ["pcgls-alg3", "lsqr-alg2", "pcgls-syncfree"])
def test_graph_replays_equal_eager(gpu_lib, name, cfg):
    """Solves that replay the captured iteration graph (several replays per solve, eager
    work and synchronisations in between, three solves, then a re-upload to a new buffer)
    give bit for bit the results of solves launched kernel by kernel."""
    R = gpu_lib
    torch = torch_dev()
    prob = PROBLEMS[name]()
    kw = {"pcgls-alg3": dict(smode=R.S_IDENTITY),
          "lsqr-alg2": dict(smode=R.S_NONE, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR),
          "pcgls-syncfree": dict(smode=R.S_NONE, form=R.FORM_ALG2, trsv=R.TRSV_SYNCFREE)}[cfg]
    b = to_dev(prob.b)
    eager = make(R, prob, mu=1.0, maxit=60, graph=0, **kw)
    xe, ce, ie, ae, re_ = eager.solve(b, tol=1e-10)
    want = to_host(xe)
    eager.close()
    S = make(R, prob, mu=1.0, maxit=60, graph=1, **kw)
    for rep in range(4):
        if rep == 3:
            S.upload()  # new buffer: the graph is captured again
        x, code, it, atr, rel = S.solve(b, tol=1e-10)
        got = to_host(x)
        assert code == ce and it == ie, (rep, code, ce, it, ie)
        assert np.array_equal(got.view(np.int64), want.view(np.int64)), rep
        # eager work on the same stream between replays
        torch.cuda.synchronize()
        _ = (b * 2.0).sum().item()
    S.close()
