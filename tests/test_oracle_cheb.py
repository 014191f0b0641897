"""Pins of the oracle's Chebyshev M_b (a fixed polynomial in S~ standing for S~^{-1}; Section 3.2
allows any approximation S^ of S~ that is cheaper to solve with).

* after K steps, w = p(S~) u with p(t) = (1 - r_K(t)) / t and r_K the scaled Chebyshev
  polynomial of the interval [1, b] (numpy's Chebyshev series and a dense eigendecomposition);
* the degree rule: K even, (b - 1) eps_K <= delta, and K - 2 would not satisfy it;
* the power-iteration estimate is a lower bound of lambda_max(S~) and close to it;
* the Algorithm 2 operator is symmetric positive definite, and M^{-1} C~ (C~ = A~^T A~ of the
  factors, A~ = [L1; Y~ L1] U) has its eigenvalues in [1 - delta, 1 + delta];
* an even degree keeps it positive definite even when b underestimates lambda_max (an odd
  one need not), which is why the rule takes even degrees;
* LSQR with this M^{-1} converges to the least-squares solution (dense QR);
* a degree fixed too low for the interval scales the input by omega = 1 / (1 + eps_K): the
  eigenvalues of M^{-1} C~ are then t - omega (t - 1)(1 - r_K(t)) over the spectrum of S~
  (and 1 on the null space of Y~), all positive, where the unscaled operator has a negative
  one; LSQR with degree 2 then converges on a request with dense rows, where the unscaled
  polynomial breaks down.
"""

import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import gen
import oracle


@pytest.fixture(scope="module")
def small():
    prob = gen.random_sparse(60, 40, k=4, seed=63)  # m - n = 20
    return prob, oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cheb", ystore=True, ytau=0.0)


@pytest.fixture(scope="module")
def tiny():
    prob = gen.tiny_c1()
    return prob, oracle.factor_problem(prob, mu=1.0, smode="cheb", ystore=True, ytau=1e-2)


def dense_S(F):
    Yd = F.Y.dense()
    return np.eye(F.Y.nrows) + Yd @ Yd.T


def r_K(t, K, b):
    """T_K((b + 1 - 2t)/(b - 1)) / T_K((b + 1)/(b - 1)) by numpy's Chebyshev series."""
    coef = np.zeros(K + 1)
    coef[K] = 1.0
    return C.chebval((b + 1 - 2 * t) / (b - 1), coef) / C.chebval((b + 1) / (b - 1), coef)


@pytest.mark.parametrize("which", ["small", "tiny"])
def test_chebyshev_is_the_scaled_polynomial(which, small, tiny):
    prob, F = small if which == "small" else tiny
    lam, V = np.linalg.eigh(dense_S(F))
    u = np.random.default_rng(31).standard_normal(F.Y.nrows)
    p = (1 - r_K(lam, F.cheb_degree, F.cheb_b)) / lam
    want = V @ (p * (V.T @ u))
    got = oracle.cheb_S(F, u)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


@pytest.mark.parametrize("lam,delta", [(2.0, 0.5), (220.3, 0.9), (488.2, 0.9), (488.2, 0.1), (5e4, 0.9)])
def test_degree_rule(lam, delta):
    b, K = oracle.cheb_plan(lam, delta)
    assert b == 1.05 * lam and K % 2 == 0 and 2 <= K <= 512
    eps = lambda k: 1.0 / math.cosh(k * math.acosh((b + 1) / (b - 1)))
    assert (b - 1) * eps(K) <= delta or K == 512  # the cap
    if K > 2:
        assert (b - 1) * eps(K - 2) > delta
    assert oracle.cheb_plan(1.0, delta) == (1.0, 0)
    assert oracle.cheb_plan(lam, delta, degree=7) == (b, 7)


@pytest.mark.parametrize("which", ["small", "tiny"])
def test_power_iteration_estimate(which, small, tiny):
    _, F = small if which == "small" else tiny
    top = np.linalg.eigvalsh(dense_S(F))[-1]
    est = oracle.lambda_max_S(F)
    assert est <= top * (1 + 1e-12) and est >= 0.9 * top
    assert F.cheb_b == 1.05 * est


def alg2_operator(F):
    return np.column_stack([oracle.apply_alg2(F, e) for e in np.eye(F.n)])


def factor_normal_matrix(F):
    """C~ = A~^T A~ for A~ = [L1; Y~ L1] U."""
    L1 = F.L1.dense() + np.eye(F.n)
    U = F.U.dense() + np.diag(F.Udiag)
    At = np.vstack([L1, F.Y.dense() @ L1]) @ U
    return At.T @ At


def test_operator_spd_and_spectrum(small):
    _, F = small
    M = alg2_operator(F)
    assert np.allclose(M, M.T, rtol=0, atol=1e-10 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    ev = np.linalg.eigvals(M @ factor_normal_matrix(F)).real
    delta = 0.9
    assert ev.min() >= 1 - delta - 1e-8 and ev.max() <= 1 + delta + 1e-8


def test_even_degree_keeps_spd_when_b_is_too_small(small):
    import dataclasses

    _, F = small
    top = np.linalg.eigvalsh(dense_S(F))[-1]
    G = dataclasses.replace(F, cheb_b=1 + 0.3 * (top - 1), cheb_degree=6)
    ev = np.linalg.eigvals(alg2_operator(G) @ factor_normal_matrix(G)).real
    assert ev.min() > 0
    # an odd degree makes 1 + (t - 1) r_K(t) negative beyond b on this spectrum
    H = dataclasses.replace(F, cheb_b=1 + 0.3 * (top - 1), cheb_degree=5)
    t = np.linalg.eigvalsh(dense_S(H))
    assert np.min(1 + (t - 1) * r_K(t, 5, H.cheb_b)) < 0
    assert np.linalg.eigvals(alg2_operator(H) @ factor_normal_matrix(H)).real.min() < 0


def test_lsqr_with_chebyshev_reaches_least_squares(tiny):
    prob, F = tiny
    res = oracle.lsqr_m(F, prob.b, tol=1e-10, maxit=200)
    assert res.status == "ok"
    A = prob.dense()
    xls = np.linalg.lstsq(A, prob.b, rcond=None)[0]
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    assert np.linalg.norm(res.x - xls) <= 2 * res.atr_norm / smin**2 + 1e-12 * np.linalg.norm(xls)
    pc = oracle.pcgls(F, prob.b, tol=1e-10, maxit=200, form="alg2")
    assert pc.status == "ok" and abs(pc.iters - res.iters) <= 1


def test_scale_rule():
    for lam in (2.0, 220.3, 488.2, 5e4):
        b, K = oracle.cheb_plan(lam, 0.9)
        eps = 1.0 / math.cosh(K * math.acosh((b + 1) / (b - 1)))
        want = 1.0 if (b - 1) * eps <= 0.9 else 1.0 / (1.0 + eps)  # the cap of 512 at 5e4
        assert oracle.cheb_scale(b, K, 0.9) == want
    assert oracle.cheb_scale(1.05 * 488.2, 88, 0.9) == 1.0
    b = 1.05 * 488.2
    sig = (b + 1) / (b - 1)
    eps2 = 1.0 / (2 * sig * sig - 1)  # T_2(x) = 2 x^2 - 1
    assert abs(oracle.cheb_scale(b, 2, 0.9) - 1 / (1 + eps2)) <= 1e-15
    assert oracle.cheb_scale(1.0, 0, 0.9) == 1.0


def test_low_degree_scaled_spectrum():
    import dataclasses

    prob = gen.random_sparse(60, 40, k=4, seed=63)
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode="cheb", ystore=True, ytau=0.0, poly_degree=2)
    assert F.cheb_degree == 2 and 0.5 < F.cheb_omega < 1
    t = np.linalg.eigvalsh(dense_S(F))
    r = r_K(t, 2, F.cheb_b)
    want = np.sort(np.concatenate([t - F.cheb_omega * (t - 1) * (1 - r), np.ones(F.n - F.Y.nrows)]))
    got = np.sort(np.linalg.eigvals(alg2_operator(F) @ factor_normal_matrix(F)).real)
    assert np.allclose(got, want, rtol=1e-8, atol=1e-10)
    assert got[0] > 0
    G = dataclasses.replace(F, cheb_omega=1.0)
    assert np.linalg.eigvals(alg2_operator(G) @ factor_normal_matrix(G)).real.min() < 0


def test_low_degree_lsqr_on_dense_rows():
    import dataclasses

    prob = gen.served_request(3000, 4500, 31, n_dense=12)
    F = oracle.factor_problem(prob, mu=1.0, smode="cheb", ystore=True, ytau=1e-2, poly_degree=2)
    assert F.cheb_omega < 1
    res = oracle.lsqr_m(F, prob.b, tol=1e-8, maxit=500)
    A = prob.scipy()
    assert res.status == "ok"
    assert np.linalg.norm(A.T @ (prob.b - A @ res.x)) <= 2e-8 * np.linalg.norm(A.T @ prob.b)
    bad = oracle.lsqr_m(dataclasses.replace(F, cheb_omega=1.0), prob.b, tol=1e-8, maxit=500)
    assert bad.status == "breakdown"
