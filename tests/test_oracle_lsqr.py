"""Pins of the oracle's LSQR in the M-inner-product form (lsqr_m).

* its iterates equal SciPy's textbook LSQR (a library routine) run on the explicitly
  preconditioned dense operator A_hat N, N = chol(M^{-1}), mapped back by x_hat = N y;
* in exact arithmetic they are Algorithm 1's iterates with the same SPD M (CGLS and LSQR
  are the same method), checked on the first steps;
* it converges to the dense least-squares solution within the stop-test bound;
* its ||A^T r|| estimate matches the true value along the way.
"""

import numpy as np
import pytest
from scipy.sparse.linalg import lsqr as scipy_lsqr

import gen
import oracle


def setup(smode="none", seed=71):
    prob = gen.random_sparse(60, 40, k=4, seed=seed)
    F = oracle.factor_problem(prob, p=4, tau=1e-2, mu=1.0, smode=smode)
    return prob, F


def preconditioner_matrix(F):
    return np.column_stack([oracle.apply_alg2(F, e) for e in np.eye(F.n)])


@pytest.mark.parametrize("smode", ["none", "dense"])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_iterates_equal_textbook_lsqr(smode, k):
    prob, F = setup(smode)
    P = preconditioner_matrix(F)
    N = np.linalg.cholesky(0.5 * (P + P.T))
    Ah = F.Ahat.dense()
    rb = prob.b[F.perm.astype(np.int64)]
    y = scipy_lsqr(Ah @ N, rb, damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    want = (N @ y) / F.colnorm
    got = oracle.lsqr_m(F, prob.b, tol=0.0, maxit=k)
    assert got.iters == k
    assert np.linalg.norm(got.x - want) <= 1e-9 * np.linalg.norm(want)


def test_equals_pcgls_with_same_preconditioner():
    prob, F = setup("none", seed=72)
    for k in (1, 2, 4):
        a = oracle.lsqr_m(F, prob.b, tol=0.0, maxit=k)
        b = oracle.pcgls(F, prob.b, tol=0.0, maxit=k, form="alg2")
        assert np.linalg.norm(a.x - b.x) <= 1e-9 * np.linalg.norm(b.x), k


def test_converges_to_least_squares_and_estimate_is_true():
    prob = gen.tiny_c1()
    F = oracle.factor_problem(prob, p=10, tau=1e-2, mu=1.0, smode="none")
    tol = 1e-10
    res = oracle.lsqr_m(F, prob.b, tol=tol, maxit=500)
    assert res.status == "ok"
    A = prob.dense()
    x_ls = np.linalg.lstsq(A, prob.b, rcond=None)[0]
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    atb = np.linalg.norm(A.T @ prob.b)
    assert res.atr_rel <= 10 * tol
    assert np.linalg.norm(res.x - x_ls) <= 10 * tol * atb / smin**2 + 1e-12 * np.linalg.norm(x_ls)
    # the recurrence estimate at exit agrees with the recomputed ||A^T r||
    assert abs(res.hist[-1] - res.atr_norm) <= 1e-3 * res.atr_norm + 1e-12 * atb


def test_rejects_non_spd_operator():
    prob, F = setup("identity")
    with pytest.raises(ValueError):
        oracle.lsqr_m(F, prob.b)
