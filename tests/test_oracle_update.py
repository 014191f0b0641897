"""Pins of the oracle's row updates (Section 3.4, adding and removing rows).

* With no dropping, every new L2 row l satisfies l U = a_hat (the definition: the kept
  factorization P A_hat ~ [L1; L2] U extended by the new rows).
* With complete factors and the dense S~, Algorithm 2 after the update is the inverse
  normal matrix of the augmented A_hat, and LSQR reaches the augmented least-squares
  solution in one or two steps (dense least squares as the reference).
* Dropping keeps exactly the entries of the undropped row with |l_j| >= tau.
"""

import numpy as np
import pytest

import gen
import oracle

INF = 10**9


def new_rows(count, n, seed):
    return gen.random_sparse(count, n, k=5, seed=seed, transversal=False)


def test_new_l2_rows_solve_u_transposed():
    p = gen.random_sparse(120, 80, k=4, seed=61)
    F = oracle.factor_problem(p, p=10, tau=1e-2, mu=1.0, smode="none")
    q = new_rows(15, 80, 62)
    G = oracle.add_rows(F, q.rowptr, q.col, q.val, tau=0.0)
    U = G.U.dense() + np.diag(G.Udiag)
    Lnew = G.L2.dense()[-15:]
    Anew = G.Ahat.dense()[-15:]
    assert np.allclose(Lnew @ U, Anew, rtol=0, atol=1e-12 * np.abs(Anew).max())
    assert np.array_equal(G.perm[:F.m], F.perm) and np.array_equal(G.perm[F.m:], np.arange(F.m, F.m + 15))
    # the kept parts are untouched and the new A_hat rows carry the setup's scaling
    assert np.array_equal(G.L1.val, F.L1.val) and np.array_equal(G.U.val, F.U.val)
    assert np.array_equal(G.L2.dense()[:-15], F.L2.dense())
    assert np.allclose(Anew, q.dense() / F.colnorm[None, :], rtol=1e-15, atol=0)


def test_dropping_keeps_entries_at_or_above_tau():
    p = gen.random_sparse(100, 70, k=4, seed=63)
    F = oracle.factor_problem(p, p=10, tau=1e-2, mu=1.0, smode="none")
    q = new_rows(10, 70, 64)
    full = oracle.add_rows(F, q.rowptr, q.col, q.val, tau=0.0).L2.dense()[-10:]
    tau = 5e-2
    kept = oracle.add_rows(F, q.rowptr, q.col, q.val, tau=tau).L2.dense()[-10:]
    want = np.where(np.abs(full) >= tau, full, 0.0)
    assert np.array_equal(kept, want)


def test_complete_factors_give_augmented_least_squares():
    p = gen.random_sparse(70, 45, k=4, seed=65, rhs="uniform")
    F = oracle.factor_problem(p, p=INF, tau=0.0, mu=1.0, smode="dense")
    q = new_rows(12, 45, 66)
    G = oracle.add_rows(F, q.rowptr, q.col, q.val, tau=0.0)
    Ah = G.Ahat.dense()
    z = np.random.default_rng(7).standard_normal(45)
    want = np.linalg.solve(Ah.T @ Ah, z)
    assert np.allclose(oracle.apply_alg2(G, z), want, rtol=1e-8, atol=1e-8 * np.abs(want).max())
    b = np.concatenate([p.b, np.random.default_rng(8).uniform(-1, 1, 12)])
    res = oracle.lsqr_m(G, b, tol=1e-10, maxit=10)
    A = np.vstack([p.dense(), q.dense()])
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert res.status == "ok" and res.iters <= 2
    assert np.linalg.norm(res.x - x_ls) <= 1e-8 * np.linalg.norm(x_ls)


# ---------------------------------------------------------------- removing rows


def test_removal_complete_factors_gives_reduced_normal_matrix():
    """Complete factors, dense S~: removing rows of A1 and A2 leaves the Woodbury-updated
    operator equal to the inverse normal matrix of the reduced A_hat, and LSQR reaches the
    reduced least-squares solution in one or two steps."""
    p = gen.random_sparse(70, 45, k=4, seed=67, rhs="uniform")
    F = oracle.factor_problem(p, p=INF, tau=0.0, mu=1.0, smode="dense")
    pos = np.empty(p.m, dtype=np.int64)
    pos[F.perm] = np.arange(p.m)
    rows = np.array([2, 9, 17, 30, 44, 51, 63])
    assert np.any(pos[rows] < p.n) and np.any(pos[rows] >= p.n)  # both blocks
    G = oracle.remove_rows(F, rows)
    keep = np.setdiff1d(np.arange(p.m), rows)
    Ah = p.dense()[keep] / F.colnorm[None, :]
    z = np.random.default_rng(3).standard_normal(45)
    want = np.linalg.solve(Ah.T @ Ah, z)
    assert np.allclose(oracle.apply_alg2(G, z), want, rtol=1e-8, atol=1e-8 * np.abs(want).max())
    assert G.R is not None and G.R.nrows == int(np.sum(pos[rows] < p.n))
    res = oracle.lsqr_m(G, p.b[keep], tol=1e-10, maxit=10)
    x_ls = np.linalg.lstsq(p.dense()[keep], p.b[keep], rcond=None)[0]
    assert res.status == "ok" and res.iters <= 2
    assert np.linalg.norm(res.x - x_ls) <= 1e-8 * np.linalg.norm(x_ls)


def test_removal_renumbers_and_keeps_factors():
    p = gen.random_sparse(90, 50, k=4, seed=68)
    F = oracle.factor_problem(p, mu=1.0, smode="dense")
    rows = np.array([0, 5, 33, 89])
    G = oracle.remove_rows(F, rows)
    keep = np.setdiff1d(np.arange(p.m), rows)
    assert G.m == p.m - 4 and sorted(G.perm.tolist()) == list(range(G.m))
    # position order of the kept rows is unchanged; numbers are compacted
    old = F.perm[np.isin(F.perm, keep)]
    assert np.array_equal(keep[G.perm], old)
    assert np.array_equal(G.L1.val, F.L1.val) and np.array_equal(G.U.val, F.U.val)
    assert np.array_equal(G.A.dense(), p.dense()[keep])


def test_removal_rejects():
    p = gen.random_sparse(60, 40, k=4, seed=69)
    F = oracle.factor_problem(p, mu=1.0, smode="none")
    with pytest.raises(ValueError):
        oracle.remove_rows(F, [1])  # needs the dense S~
    Fd = oracle.factor_problem(p, mu=1.0, smode="dense")
    for bad in ([], [3, 3], [-1], [60], list(range(21))):
        with pytest.raises(ValueError):
            oracle.remove_rows(Fd, bad)
