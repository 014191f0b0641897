"""GPU parity of the explicit Y~ path (Section 3.2: Y~ = L2 L1^{-1} stored as a sparse matrix,
small entries dropped), through the C ABI, against the CPU oracle.

* products with Y~ and Y~^T: componentwise |y - y_or| <= 2 k eps (|Y~| |x|)_i (k entries per row);
* one preconditioner application (Algorithm 2 on z, Algorithm 3 on r; S^ = I or CG(8) on S~),
  element by element: |h - h_or| <= rtol |h_or| + atol ||h_or||_inf, with (rtol, atol) =
  (1e-10, 1e-13) for S^ = I (no iteration between the triangular solves) and (1e-8, 1e-11)
  with CG, whose steps are exact line searches that pass rounding differences on; both 100x
  wider on the sparse-dense mini case, whose factors have kappa(L1 U) = 2.6e9 (its dense rows
  are pivoted into A1 at mu = 1), so that the two sides' differently ordered sums in the
  triangular solves differ by up to that factor more than on c1 (kappa 4.3);
* CG(32): past some 16 steps the CG iterates on S~ depend on the rounding of their inner
  products well beyond eps (the oracle itself moves by up to 1e-3 relative when its inner
  products are summed in another order), so the GPU's application is held to what CG
  guarantees instead: its distance to the exact correction (the dense solve with
  S~ = I + Y~ Y~^T) is at most twice the oracle's;
* Algorithm 1 with Algorithm 2 and CG(8) on S~: 4 iterations step for step (x within 1e-8;
  the mini sparse-dense case 1e-6, see above), and whole solves with CG(32) to 1e-8
  (iterations within 2% of the oracle's, the true ||A^T r|| at the tolerance, x in the
  oracle's stop-test ball);
* with ytau = 0 (every nonzero of Y~ kept) the path equals the implicit one to rounding.
"""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps / 2


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(n):
    import torch

    return torch.empty(n, dtype=torch.float64, device="cuda")


def long_row_problem():
    return gen.random_sparse(3000, 2500, k=4, seed=17, n_dense=3, dense_len=2400)


PROBLEMS = {
    "c1": lambda: gen.tiny_c1(),
    "c2-small": lambda: gen.by_name("c2-small"),
    "c3-mini": lambda: gen.by_name("c3-mini"),
    "long-rows": long_row_problem,
}


def solver(R, prob, smode, steps=32, ytau=1e-2, trsv=None, **kw):
    params = dict(mu=1.0, form=R.FORM_ALG2, ystore=R.Y_EXPLICIT, ytau=ytau,
                  smode={"identity": R.S_IDENTITY, "cg": R.S_CG, "none": R.S_NONE}[smode], cg_steps=steps)
    if trsv is not None:
        params["trsv"] = trsv
    params.update(kw)
    return R.Solver.from_problem(prob, **params).upload()


def factors(prob, smode, steps=32, ytau=1e-2):
    return oracle.factor_problem(prob, mu=1.0, smode=smode, cg_steps=steps, ystore=True, ytau=ytau)


def elementwise(got, want, rtol, atol):
    """Largest ratio of |got - want| to rtol |want| + atol ||want||_inf (<= 1 passes)."""
    bound = rtol * np.abs(want) + atol * np.max(np.abs(want))
    return float(np.max(np.abs(got - want) / bound))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_products_with_Y(gpu_lib, name):
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = solver(R, prob, "cg", steps=2)
    F = factors(prob, "cg", steps=2)
    rng = np.random.default_rng(21)
    for op, C in ((4, F.Y), (5, F.YT)):
        x = rng.standard_normal(C.ncols)
        y = empty(C.nrows)
        assert R.rsilu_spmv(S.h, op, to_dev(x), y) == R.OK
        got = to_host(y)
        want = C.matvec(x)
        k = np.diff(C.rowptr)
        absprod = np.abs(C.scipy()) @ np.abs(x)
        assert np.all(np.abs(got - want) <= 2 * k * EPS * absprod + 1e-300), (name, op)
    S.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("form", ["alg2", "alg3"])
@pytest.mark.parametrize("smode,steps", [("identity", 0), ("cg", 8)])
@pytest.mark.parametrize("mode", ["hybrid", "levels"])
def test_apply_explicit_Y(gpu_lib, name, form, smode, steps, mode):
    R = gpu_lib
    prob = PROBLEMS[name]()
    trsv = {"hybrid": R.TRSV_HYBRID, "levels": R.TRSV_LEVELS}[mode]
    S = solver(R, prob, smode, steps=max(steps, 1), trsv=trsv)
    F = factors(prob, smode, steps=max(steps, 1))
    h = empty(prob.n)
    rng = np.random.default_rng(22)
    if form == "alg3":
        r = rng.standard_normal(prob.m)
        assert R.rsilu_apply(S.h, to_dev(r), h) == R.OK
        want = oracle.apply_alg3(F, r)
    else:
        z = rng.standard_normal(prob.n)
        assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
        want = oracle.apply_alg2(F, z)
    rtol, atol = (1e-10, 1e-13) if smode == "identity" else (1e-8, 1e-11)
    if name == "c3-mini":
        rtol, atol = 100 * rtol, 100 * atol  # kappa(L1 U) = 2.6e9 on this workload, against 4.3 on c1
    ratio = elementwise(to_host(h), want, rtol, atol)
    print(f"{name} {form} {smode}({steps}) {mode}: elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
    S.close()


def exact_correction(F, z):
    """Algorithm 2 through the explicit Y~ with M_b = S~ = I + Y~ Y~^T solved densely."""
    import scipy.linalg as sla

    Yd = F.Y.dense()
    S = np.eye(F.Y.nrows) + Yd @ Yd.T
    g = oracle.upper_solve(F.L1T, oracle.lower_solve(F.UT, z, F.Udiag))
    vb = sla.cho_solve(sla.cho_factor(S, lower=True), F.Y.matvec(g))
    return oracle.upper_solve(F.U, oracle.lower_solve(F.L1, g - F.YT.matvec(vb)), F.Udiag)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_apply_cg32_as_accurate_as_oracle(gpu_lib, name):
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = solver(R, prob, "cg", steps=32)
    F = factors(prob, "cg", steps=32)
    z = np.random.default_rng(24).standard_normal(prob.n)
    h = empty(prob.n)
    assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
    got = to_host(h)
    want = oracle.apply_alg2(F, z)
    exact = exact_correction(F, z)
    e_gpu = np.linalg.norm(got - exact)
    e_or = np.linalg.norm(want - exact)
    print(f"{name}: distance to the exact correction, GPU {e_gpu / np.linalg.norm(exact):.2e}, "
          f"oracle {e_or / np.linalg.norm(exact):.2e}")
    assert e_gpu <= 2 * e_or + 1e-10 * np.linalg.norm(exact)
    S.close()


def run(R, prob, tol, maxit, smode="cg", steps=32, ytau=1e-2, **kw):
    S = solver(R, prob, smode, steps=steps, ytau=ytau, maxit=maxit, **kw)
    x, code, it, atr, rel = S.solve(to_dev(prob.b), tol=tol)
    out = to_host(x)
    S.close()
    return out, code, it, atr, rel


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_pcgls_alg2_cg_steps(gpu_lib, name):
    """Algorithm 1 with Algorithm 2, CG(8) on S~ through the explicit Y~: 4 steps, step for step."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    maxit = 4
    x, code, it, atr, rel = run(R, prob, 1e-14, maxit, steps=8)
    res = oracle.pcgls(factors(prob, "cg", steps=8), prob.b, tol=1e-14, maxit=maxit, form="alg2")
    err = np.linalg.norm(x - res.x) / np.linalg.norm(res.x)
    print(f"{name} {maxit} steps: its {it} / {res.iters}, x rel diff {err:.2e}")
    assert it == res.iters
    assert err <= (1e-6 if name == "c3-mini" else 1e-8)
    assert abs(atr - res.atr_norm) <= 1e-6 * res.atr_norm


@pytest.mark.parametrize("name,ytau,steps", [("c1", 1e-2, 32), ("c2-small", 1e-2, 32)])
def test_pcgls_alg2_cg_converges_like_oracle(gpu_lib, name, ytau, steps):
    R = gpu_lib
    prob = PROBLEMS[name]()
    tol = 1e-8
    x, code, it, atr, rel = run(R, prob, tol, 2000, steps=steps, ytau=ytau)
    res = oracle.pcgls(factors(prob, "cg", steps=steps, ytau=ytau), prob.b, tol=tol, maxit=2000, form="alg2")
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    ball = np.linalg.norm(A.T @ (A @ (x - res.x))) / atb
    xerr = np.linalg.norm(x - res.x) / np.linalg.norm(res.x)
    print(f"{name} ytau {ytau} CG({steps}): its {it} / {res.iters}, rel {rel:.2e}, ball {ball:.2e}, x {xerr:.2e}")
    assert code == R.OK and res.status == "ok"
    assert abs(it - res.iters) <= max(1, int(0.02 * res.iters))
    assert rel <= 2 * tol
    assert ball <= 4 * tol


def test_exact_Y_equals_implicit_path(gpu_lib):
    """ytau = 0 keeps every nonzero of Y~: the explicit path computes the implicit one's
    operator, so one application agrees to rounding."""
    R = gpu_lib
    prob = gen.by_name("c2-small")
    Se = solver(R, prob, "cg", steps=8, ytau=0.0)
    Si = R.Solver.from_problem(prob, mu=1.0, form=R.FORM_ALG2, smode=R.S_CG, cg_steps=8).upload()
    z = to_dev(np.random.default_rng(23).standard_normal(prob.n))
    he, hi = empty(prob.n), empty(prob.n)
    assert R.rsilu_apply_z(Se.h, z, he) == R.OK and R.rsilu_apply_z(Si.h, z, hi) == R.OK
    a, b = to_host(he), to_host(hi)
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    Se.close()
    Si.close()


def test_graph_replays_equal_eager_explicit_Y(gpu_lib):
    R = gpu_lib
    prob = gen.by_name("c2-small")
    b = to_dev(prob.b)
    outs = []
    for graph in (0, 1, 1):
        S = solver(R, prob, "cg", steps=32, maxit=40, graph=graph)
        x, code, it, atr, rel = S.solve(b, tol=1e-14)
        x2, code2, it2, _, _ = S.solve(b, tol=1e-14)
        outs.append((to_host(x), it))
        assert np.array_equal(to_host(x2), outs[-1][0]) and it2 == it
        S.close()
    assert all(np.array_equal(o[0], outs[0][0]) and o[1] == outs[0][1] for o in outs)


# ------------------------------------------------------------------ Jacobi-preconditioned CG


def jacobi_solver(R, prob, steps, **kw):
    return solver(R, prob, "cg", steps=steps, cg_precond=R.CG_JACOBI, **kw)


def jacobi_factors(prob, steps):
    return oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=steps, ystore=True, ytau=1e-2, cg_jacobi=True)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("mode", ["hybrid", "levels"])
def test_apply_jacobi_cg(gpu_lib, name, mode):
    """One Algorithm 2 application with 8 Jacobi-preconditioned CG steps on S~ against the
    oracle's, element by element (the bounds of the plain CG(8) application)."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    trsv = {"hybrid": R.TRSV_HYBRID, "levels": R.TRSV_LEVELS}[mode]
    S = jacobi_solver(R, prob, 8, trsv=trsv)
    F = jacobi_factors(prob, 8)
    z = np.random.default_rng(25).standard_normal(prob.n)
    h = empty(prob.n)
    assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
    want = oracle.apply_alg2(F, z)
    rtol, atol = (1e-8, 1e-11) if name != "c3-mini" else (1e-6, 1e-9)
    ratio = elementwise(to_host(h), want, rtol, atol)
    print(f"{name} Jacobi CG(8) {mode}: elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
    S.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_pcgls_jacobi_cg_steps(gpu_lib, name):
    """Algorithm 1 with Jacobi CG(8): four steps, step for step."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    S = jacobi_solver(R, prob, 8, maxit=4)
    x, code, it, atr, rel = S.solve(to_dev(prob.b), tol=1e-14)
    got = to_host(x)
    S.close()
    res = oracle.pcgls(jacobi_factors(prob, 8), prob.b, tol=1e-14, maxit=4, form="alg2")
    err = np.linalg.norm(got - res.x) / np.linalg.norm(res.x)
    print(f"{name} Jacobi CG(8), 4 steps: its {it} / {res.iters}, x rel diff {err:.2e}")
    assert it == res.iters
    assert err <= (1e-6 if name == "c3-mini" else 1e-8)


@pytest.mark.parametrize("name", ["c1", "c2-small"])
def test_pcgls_jacobi_cg20_converges_like_oracle(gpu_lib, name):
    """20 Jacobi-preconditioned CG steps (the benchmark takes 28, with ytau 5e-2 and ILUP(20) factors):
    iterations within 2% of the oracle's, the true ||A^T r|| at the tolerance, the solution in its
    stop-test ball."""
    R = gpu_lib
    prob = PROBLEMS[name]()
    tol = 1e-8
    S = jacobi_solver(R, prob, 20, maxit=2000)
    x, code, it, atr, rel = S.solve(to_dev(prob.b), tol=tol)
    got = to_host(x)
    S.close()
    res = oracle.pcgls(jacobi_factors(prob, 20), prob.b, tol=tol, maxit=2000, form="alg2")
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    ball = np.linalg.norm(A.T @ (A @ (got - res.x))) / atb
    print(f"{name} Jacobi CG(20): its {it} / {res.iters}, rel {rel:.2e}, ball {ball:.2e}")
    assert code == R.OK and res.status == "ok"
    assert abs(it - res.iters) <= max(1, int(0.02 * res.iters))
    assert rel <= 2 * tol and ball <= 4 * tol


@pytest.mark.parametrize("steps", [1, 2, 3])
@pytest.mark.parametrize("precond", ["plain", "jacobi"])
def test_apply_few_cg_steps(gpu_lib, steps, precond):
    """One Algorithm 2 application with 1, 2 (Table 3(a)) and 3 CG steps on S~, plain and
    Jacobi-preconditioned, against the oracle's element by element: the first and last steps,
    where the scalars come from the initial inner product and no new direction is formed."""
    R = gpu_lib
    prob = PROBLEMS["c2-small"]()
    jac = precond == "jacobi"
    S = solver(R, prob, "cg", steps=steps, cg_precond=R.CG_JACOBI if jac else R.CG_NONE)
    F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=steps, ystore=True, ytau=1e-2, cg_jacobi=jac)
    z = np.random.default_rng(26).standard_normal(prob.n)
    h = empty(prob.n)
    assert R.rsilu_apply_z(S.h, to_dev(z), h) == R.OK
    ratio = elementwise(to_host(h), oracle.apply_alg2(F, z), 1e-10, 1e-13)
    print(f"c2-small {precond} CG({steps}): elementwise ratio {ratio:.2e}")
    assert ratio <= 1.0
    S.close()


@pytest.mark.parametrize("precond", ["plain", "jacobi"])
def test_apply_cg_zero_input(gpu_lib, precond):
    """z = 0: every inner product of the CG steps is 0, so alpha and beta take their zero rules
    and the application returns exactly 0 (no 0/0)."""
    R = gpu_lib
    prob = PROBLEMS["c2-small"]()
    S = solver(R, prob, "cg", steps=4, cg_precond=R.CG_JACOBI if precond == "jacobi" else R.CG_NONE)
    h = empty(prob.n)
    assert R.rsilu_apply_z(S.h, to_dev(np.zeros(prob.n)), h) == R.OK
    got = to_host(h)
    S.close()
    assert np.all(got == 0.0)
