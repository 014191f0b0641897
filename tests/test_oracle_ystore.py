"""Pins of the oracle's explicit Y~ (Section 3.2: Y~ = L2 L1^{-1} computed by back
substitution with L1^T and stored as a sparse matrix) and of the preconditioner
applications that use it.

* tauY = 0: Y~ equals L2 L1^{-1} formed by a dense triangular solve (SciPy), entry by entry;
* tauY > 0: every row y of Y~ satisfies the dropping substitution's defining relations,
  checked on the dense residual v = l - y L1: v_j = 0 (to rounding) where y_j is kept,
  |v_j| < tauY where it was dropped, and every kept |y_j| >= tauY;
* the S~ product through Y~ equals (I + Y~ Y~^T) d, and m - n CG steps reach the dense solve;
* with tauY = 0, Algorithm 3 and Algorithm 2 through the explicit Y~ equal their implicit
  forms (S^ = I; and CG with m - n steps against the dense S~);
* Algorithm 1 with Algorithm 2 and CG on the explicit Y~ converges to the least-squares
  solution (dense QR) within the stop test's bound;
* the oracle's inner product is the correctly rounded sum of the rounded products.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla

import gen
import oracle


@pytest.fixture(scope="module")
def small():
    return gen.random_sparse(45, 30, k=4, seed=61)  # m - n = 15


@pytest.fixture(scope="module")
def tiny_factors():
    prob = gen.tiny_c1()
    return prob, oracle.factor_problem(prob, mu=1.0, smode="identity")


def dense_Y(F):
    L1d = F.L1.dense() + np.eye(F.n)
    return sla.solve_triangular(L1d.T, F.L2.dense().T, lower=False, unit_diagonal=True).T


def test_exact_Y_equals_dense_solve(tiny_factors):
    _, F = tiny_factors
    Y = oracle.explicit_Y(F.L1, F.L2, 0.0)
    want = dense_Y(F)
    got = Y.dense()
    # componentwise: |Y - Y_dense| <= c eps (|L2| |L1^{-1}|-sized terms), bounded here by the row scale
    scale = np.abs(want).max(axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(got - want) / scale) <= 1e-12
    # structure: no stored zeros, ascending columns within each row
    assert np.all(Y.val != 0.0)
    for i in range(Y.nrows):
        c = Y.col[Y.rowptr[i]:Y.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


@pytest.mark.parametrize("tauY", [1e-3, 1e-2, 1e-1])
def test_dropped_Y_satisfies_its_substitution(tiny_factors, tauY):
    _, F = tiny_factors
    Y = oracle.explicit_Y(F.L1, F.L2, tauY)
    Yd = Y.dense()
    L1d = F.L1.dense() + np.eye(F.n)
    L2d = F.L2.dense()
    v = L2d - Yd @ L1d  # v_j = l_j - y_j - sum_{k>j} y_k l_kj
    bound = 8 * np.finfo(float).eps * (np.abs(L2d) + np.abs(Yd) @ np.abs(L1d))
    kept = Yd != 0.0
    assert np.all(np.abs(Yd[kept]) >= tauY)
    assert np.all(np.abs(v[kept]) <= bound[kept])
    assert np.all(np.abs(v[~kept]) < tauY + bound[~kept])
    # dropping removes something on this workload, and the drop tolerance orders the fill
    exact = oracle.explicit_Y(F.L1, F.L2, 0.0)
    assert Y.nnz < exact.nnz


def test_dropped_fill_is_monotone(tiny_factors):
    _, F = tiny_factors
    nnz = [oracle.explicit_Y(F.L1, F.L2, t).nnz for t in (0.0, 1e-4, 1e-3, 1e-2, 1e-1)]
    assert all(a >= b for a, b in zip(nnz, nnz[1:])), nnz


def test_explicit_S_product_and_cg(small):
    k = small.m - small.n
    F = oracle.factor_problem(small, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=k, ystore=True, ytau=0.0)
    Y = dense_Y(F)
    S = np.eye(k) + Y @ Y.T
    rng = np.random.default_rng(5)
    d = rng.standard_normal(k)
    assert np.allclose(oracle.S_product(F, d), S @ d, rtol=1e-12, atol=1e-12)
    u = rng.standard_normal(k)
    want = np.linalg.solve(S, u)
    assert np.linalg.norm(oracle.cg_S(F, u) - want) <= 1e-8 * np.linalg.norm(want)


def test_alg3_identity_explicit_equals_implicit(tiny_factors):
    prob, F = tiny_factors
    Fy = oracle.factor_problem(prob, mu=1.0, smode="identity", ystore=True, ytau=0.0)
    r = np.random.default_rng(6).standard_normal(prob.m)
    a, b = oracle.apply_alg3(Fy, r), oracle.apply_alg3(F, r)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("form", ["alg3", "alg2"])
def test_explicit_full_cg_equals_dense(small, form):
    k = small.m - small.n
    Fy = oracle.factor_problem(small, p=4, tau=1e-2, mu=1.0, smode="cg", cg_steps=k, ystore=True, ytau=0.0)
    Fd = oracle.factor_problem(small, p=4, tau=1e-2, mu=1.0, smode="dense")
    rng = np.random.default_rng(7)
    if form == "alg3":
        r = rng.standard_normal(small.m)
        a, b = oracle.apply_alg3(Fy, r), oracle.apply_alg3(Fd, r)
    else:
        z = rng.standard_normal(small.n)
        a, b = oracle.apply_alg2(Fy, z), oracle.apply_alg2(Fd, z)
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)


def test_alg2_explicit_none_is_uncorrected(tiny_factors):
    prob, _ = tiny_factors
    Fy = oracle.factor_problem(prob, mu=1.0, smode="none", ystore=True, ytau=1e-2)
    Fn = oracle.factor_problem(prob, mu=1.0, smode="none")
    z = np.random.default_rng(8).standard_normal(prob.n)
    assert np.array_equal(oracle.apply_alg2(Fy, z), oracle.apply_alg2(Fn, z))


def test_pcgls_alg2_cg_explicit_reaches_least_squares(tiny_factors):
    prob, _ = tiny_factors
    F = oracle.factor_problem(prob, mu=1.0, smode="cg", cg_steps=16, ystore=True, ytau=1e-2)
    res = oracle.pcgls(F, prob.b, tol=1e-10, maxit=200, form="alg2")
    assert res.status == "ok"
    A = prob.dense()
    xls = np.linalg.lstsq(A, prob.b, rcond=None)[0]
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    atb = np.linalg.norm(A.T @ prob.b)
    # ||x - x_LS|| <= ||A^T r|| / sigma_min^2 (plus rounding)
    assert np.linalg.norm(res.x - xls) <= 2 * res.atr_norm / smin**2 + 1e-12 * np.linalg.norm(xls)
    assert res.atr_norm <= 2e-10 * atb


def test_dot_is_correctly_rounded():
    # the exactly rounded sum of the rounded products, in any order of the terms
    a = np.array([1.0] + [2.0**-53] * 7)
    b = np.ones_like(a)
    want = 1.0 + 4 * 2.0**-52  # 1 + 3.5 ulp, ties to even
    assert oracle.dot(a, b) == want
    assert oracle.dot(a[::-1].copy(), b) == want
    # cancellation that a sequential or pairwise sum loses entirely
    c = np.array([1e16, 1.0, -1e16])
    assert oracle.dot(c, np.ones(3)) == 1.0
    # products are rounded first: (1 + 2^-30)^2 has a term below the last bit of the product
    d = np.array([1.0 + 2.0**-30])
    assert oracle.dot(d, d) == float((1.0 + 2.0**-30) * (1.0 + 2.0**-30))


def test_dot_non_finite():
    assert oracle.dot(np.array([1e200, 1e200]), np.array([1e200, 1.0])) == float("inf")
    assert math.isnan(oracle.dot(np.array([np.inf, -np.inf]), np.array([1.0, 1.0])))
    assert oracle.dot(np.array([1e308, 1e308]), np.array([1.0, 1.0])) == float("inf")
