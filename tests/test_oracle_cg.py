"""Pins of the oracle's CG on S~ (Section 3.2; Table 3(a) takes two steps).

* the implicit product S~ d equals (I + Y~ Y~^T) d with Y~ = L2 L1^{-1} formed densely;
* one CG step from w = 0 is the closed form w = (u.u / u.S~u) u;
* m - n steps reach the dense solve S~^{-1} u (CG terminates in at most m - n steps);
* Algorithm 3 and Algorithm 2 with that many steps equal their dense-S~ forms;
* Jacobi-preconditioned CG (diag(S~) from the explicit Y~): the diagonal equals that of the
  dense S~; one step is w = ((u, D^{-1}u) / (D^{-1}u, S~ D^{-1}u)) D^{-1}u; m - n steps reach
  the dense solve; every iterate equals plain CG on D^{-1/2} S~ D^{-1/2} mapped back (the
  textbook equivalence, with the symmetric scaling formed densely).
"""

import numpy as np
import pytest

import gen
import oracle

INF = 10**9


@pytest.fixture(scope="module")
def prob():
    return gen.random_sparse(45, 30, k=4, seed=61)  # m - n = 15


def dense_S(F):
    n = F.n
    Y = F.L2.dense() @ np.linalg.inv(F.L1.dense() + np.eye(n))
    return np.eye(F.m - n) + Y @ Y.T


def test_implicit_product(prob):
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cg")
    d = np.random.default_rng(1).standard_normal(F.m - F.n)
    assert np.allclose(oracle.S_product(F, d), dense_S(F) @ d, rtol=1e-12, atol=1e-12)


def test_one_step_closed_form(prob):
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=1)
    u = np.random.default_rng(2).standard_normal(F.m - F.n)
    S = dense_S(F)
    want = (u @ u) / (u @ S @ u) * u
    assert np.allclose(oracle.cg_S(F, u), want, rtol=1e-12, atol=1e-14)


def test_full_steps_reach_dense_solve(prob):
    k = prob.m - prob.n
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=k)
    u = np.random.default_rng(3).standard_normal(k)
    want = np.linalg.solve(dense_S(F), u)
    assert np.linalg.norm(oracle.cg_S(F, u) - want) <= 1e-8 * np.linalg.norm(want)


@pytest.mark.parametrize("form", ["alg3", "alg2"])
def test_applications_with_full_cg_equal_dense(prob, form):
    k = prob.m - prob.n
    Fc = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=k)
    Fd = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="dense")
    rng = np.random.default_rng(4)
    if form == "alg3":
        r = rng.standard_normal(prob.m)
        a, b = oracle.apply_alg3(Fc, r), oracle.apply_alg3(Fd, r)
    else:
        z = rng.standard_normal(prob.n)
        a, b = oracle.apply_alg2(Fc, z), oracle.apply_alg2(Fd, z)
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)


def test_zero_rhs_stops():
    p = gen.random_sparse(40, 30, k=3, seed=62)
    F = oracle.factor_problem(p, p=4, tau=1e-2, mu=1.0, smode="cg")
    assert np.all(oracle.cg_S(F, np.zeros(10)) == 0.0)


def _jacobi(prob, steps):
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=steps, ystore=True, ytau=0.0,
                              cg_jacobi=True)
    Yd = F.Y.dense()
    return F, np.eye(F.m - F.n) + Yd @ Yd.T


def test_jacobi_diagonal(prob):
    F, S = _jacobi(prob, 1)
    assert np.allclose(F.S_diag, np.diag(S), rtol=1e-15, atol=0)
    assert F.cg_jacobi and np.all(F.S_diag >= 1.0)


def test_jacobi_one_step_closed_form(prob):
    F, S = _jacobi(prob, 1)
    u = np.random.default_rng(3).standard_normal(F.m - F.n)
    z = u / np.diag(S)
    want = (u @ z) / (z @ S @ z) * z
    assert np.allclose(oracle.cg_S(F, u), want, rtol=1e-12, atol=1e-14)


def test_jacobi_full_steps_reach_dense_solve(prob):
    F, S = _jacobi(prob, prob.m - prob.n)
    u = np.random.default_rng(4).standard_normal(F.m - F.n)
    want = np.linalg.solve(S, u)
    assert np.allclose(oracle.cg_S(F, u), want, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("steps", [2, 5])
def test_jacobi_equals_cg_on_scaled_system(prob, steps):
    """PCG with D on S~ w = u is CG on (D^{-1/2} S~ D^{-1/2}) v = D^{-1/2} u with w = D^{-1/2} v."""
    import dataclasses

    F, S = _jacobi(prob, steps)
    u = np.random.default_rng(5).standard_normal(F.m - F.n)
    d = np.sqrt(np.diag(S))
    Ss = S / d[:, None] / d[None, :]
    v = np.zeros_like(u)
    r = u / d
    pdir = r.copy()
    rr = r @ r
    for i in range(steps):
        q = Ss @ pdir
        a = rr / (pdir @ q)
        v = v + a * pdir
        r = r - a * q
        rr_new = r @ r
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
    assert np.allclose(oracle.cg_S(F, u), v / d, rtol=1e-10, atol=1e-13)
    # and it differs from plain CG (the pin has teeth)
    G = dataclasses.replace(F, cg_jacobi=False)
    assert not np.allclose(oracle.cg_S(G, u), v / d, rtol=1e-6, atol=0)
