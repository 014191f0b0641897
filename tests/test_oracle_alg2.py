"""Pins of the oracle's Algorithm 2 form (k = n) and of the "none" S^ mode.

Each preconditioner is checked against a closed form evaluated with dense
linear algebra on the factors the oracle's ILUP produced (any incomplete
factors will do, so these hold whatever the ILUP computed):
  * dense S~:  h = (A~^T A~)^{-1} z with A~ = [L1; L2] U  (Woodbury, Lemma 3.1
    applied to A~);
  * none:      h = (A~1^T A~1)^{-1} z with A~1 = L1 U;
  * S^ = I:    h = M_a^{-1} (z - A~2^T A~2 M_a^{-1} z), M_a = A~1^T A~1, A~2 = L2 U.
The Krylov tests pin the whole method to dense least squares.
"""

import numpy as np
import pytest

import gen
import oracle

INF = 10**9


def dense_factors(F):
    n = F.n
    L1 = F.L1.dense() + np.eye(n)
    L2 = F.L2.dense()
    U = F.U.dense() + np.diag(F.Udiag)
    return L1, L2, U


@pytest.fixture(scope="module")
def small():
    return gen.random_sparse(90, 60, k=4, seed=51)


def test_alg2_dense_is_inverse_normal_matrix_of_factored_A(small):
    F = oracle.factor_problem(small, p=3, tau=1e-2, mu=1.0, smode="dense")
    L1, L2, U = dense_factors(F)
    At = np.vstack([L1, L2]) @ U
    z = np.random.default_rng(1).standard_normal(F.n)
    want = np.linalg.solve(At.T @ At, z)
    got = oracle.apply_alg2(F, z)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_alg2_none_is_inverse_normal_matrix_of_A1(small):
    F = oracle.factor_problem(small, p=3, tau=1e-2, mu=1.0, smode="none")
    L1, _, U = dense_factors(F)
    A1 = L1 @ U
    z = np.random.default_rng(2).standard_normal(F.n)
    want = np.linalg.solve(A1.T @ A1, z)
    got = oracle.apply_alg2(F, z)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_alg2_identity_closed_form(small):
    F = oracle.factor_problem(small, p=3, tau=1e-2, mu=1.0, smode="identity")
    L1, L2, U = dense_factors(F)
    A1, A2 = L1 @ U, L2 @ U
    Mi = np.linalg.inv(A1.T @ A1)
    z = np.random.default_rng(3).standard_normal(F.n)
    want = Mi @ (z - A2.T @ (A2 @ (Mi @ z)))
    got = oracle.apply_alg2(F, z)
    assert np.allclose(got, want, rtol=1e-8, atol=1e-8 * np.abs(want).max())


@pytest.mark.parametrize("smode", ["none", "dense"])
def test_alg2_operator_is_spd(smode):
    """Algorithm 1 assumes M^{-1} symmetric positive definite: the dense and the
    uncorrected forms are, as operators assembled column by column."""
    prob = gen.random_sparse(50, 35, k=4, seed=52)
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode=smode)
    P = np.column_stack([oracle.apply_alg2(F, e) for e in np.eye(F.n)])
    assert np.allclose(P, P.T, rtol=1e-9, atol=1e-9 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0.0


def test_alg3_none_is_A1_inverse_on_r1(small):
    """S^ mode "none" (w = 0): Algorithm 3 reduces to h = (L1 U)^{-1} r1."""
    F = oracle.factor_problem(small, p=3, tau=1e-2, mu=1.0, smode="none")
    L1, _, U = dense_factors(F)
    r = np.random.default_rng(4).standard_normal(F.m)
    want = np.linalg.solve(L1 @ U, r[:F.n])
    got = oracle.apply_alg3(F, r)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


@pytest.mark.parametrize("seed", [53, 54])
def test_alg2_exact_factors_give_least_squares_in_one_step(seed):
    """Complete factors + dense S~: M^{-1} = (A_hat^T A_hat)^{-1}, so the first step of
    Algorithm 1 lands on the least-squares solution (Section 3.1)."""
    prob = gen.random_sparse(70, 45, k=4, seed=seed, rhs="uniform")
    F = oracle.factor_problem(prob, p=INF, tau=0.0, mu=1.0, smode="dense")
    assert F.nmod == 0
    res = oracle.pcgls(F, prob.b, tol=1e-10, maxit=10, form="alg2")
    x_ls = np.linalg.lstsq(prob.dense(), prob.b, rcond=None)[0]
    assert res.status == "ok" and res.iters <= 2
    assert np.linalg.norm(res.x - x_ls) <= 1e-9 * np.linalg.norm(x_ls)


@pytest.mark.parametrize("smode", ["none", "dense"])
def test_alg2_pcgls_converges_to_least_squares(smode):
    """ILUP(10, 1e-2) factors on the 2000 x 1000 tiny workload: with an SPD M^{-1},
    Algorithm 1 is CG on the preconditioned normal equations, so it reaches the stop
    test and then ||x - x_LS|| <= tol ||A^T b|| / sigma_min^2; ||r|| never grows and
    the new A^T r is orthogonal to the previous direction (first iterations)."""
    prob = gen.tiny_c1()
    F = oracle.factor_problem(prob, p=10, tau=1e-2, mu=1.0, smode=smode)
    tol = 1e-10
    res = oracle.pcgls(F, prob.b, tol=tol, maxit=500, form="alg2", trace=True)
    assert res.status == "ok"
    rn = np.array(res.rnorm)
    assert np.all(np.diff(rn) <= 1e-12 * rn[0])
    assert np.abs(np.array(res.orth[:8])).max() < 1e-12
    A = prob.dense()
    x_ls = np.linalg.lstsq(A, prob.b, rcond=None)[0]
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    atb = np.linalg.norm(A.T @ prob.b)
    assert res.atr_rel <= 10 * tol
    assert np.linalg.norm(res.x - x_ls) <= 10 * tol * atb / smin**2 + 1e-12 * np.linalg.norm(x_ls)


def test_alg2_square_matrix_is_A_inverse_squared():
    """m = n: no A2, M^{-1} = (A^T A)^{-1} for complete factors."""
    prob = gen.random_sparse(40, 40, k=4, seed=55)
    F = oracle.factor_problem(prob, p=INF, tau=0.0, mu=1.0, smode="dense")
    Ah = F.Ahat.dense()
    z = np.random.default_rng(5).standard_normal(40)
    want = np.linalg.solve(Ah.T @ Ah, z)
    assert np.allclose(oracle.apply_alg2(F, z), want, rtol=1e-8, atol=1e-8 * np.abs(want).max())
