"""Row updates (Section 3.4) on the GPU. Appending rows: after rsilu_add_rows and a new upload, the
solve of the augmented problem follows the oracle's LSQR on the oracle's updated factors
(four steps: x to 1e-8; whole solves: iterations within 2%, the true ||A^T r|| at 2 tol and
the oracle's stop-test ball), in both preconditioner precisions and in the batched kernel;
a solve between the update and the upload is refused. Removing rows (the Woodbury update
of the preconditioner, dense S~): four steps against the oracle's updated operator, whole
solves like it, with LSQR and Algorithm 1; removal followed by appending."""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

LSQR = dict(mu=1.0, form=1, krylov=1, smode=2)


def augmented(name, count, seed):
    """New rows of the same kind as the data: rows of A drawn at random, values perturbed
    by 10% (more measurements of a streaming least-squares problem); b extended with
    A_new x_true plus noise when the generator kept x_true."""
    import copy

    import scipy.sparse as sp

    p = gen.by_name(name) if name != "c1" else gen.tiny_c1()
    rng = np.random.default_rng(seed)
    A = p.scipy()
    pick = rng.choice(p.m, size=count, replace=False)
    Q = A[pick].tocsr()
    Q.data = Q.data * (1.0 + 0.1 * rng.standard_normal(Q.data.size))
    q = copy.copy(p)
    q.m, q.rowptr, q.col, q.val = count, Q.indptr.astype(np.int64), Q.indices.astype(np.int32), Q.data
    q.b = None
    x_true = p.x_true if p.x_true is not None else rng.standard_normal(p.n)
    b = np.concatenate([p.b, Q @ x_true + 1e-3 * rng.standard_normal(count)])
    return p, q, b


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("name,count", [("c1", 50), ("c2-small", 300)])
def test_update_four_steps_and_convergence(gpu_lib, name, count):
    R = gpu_lib
    import torch
    import scipy.sparse as sp

    p, q, b = augmented(name, count, 80)
    S = R.Solver.from_problem(p, maxit=4, **LSQR).upload()
    S.add_rows(q.rowptr, q.col, q.val)
    F = oracle.add_rows(oracle.factor_problem(p, mu=1.0, smode="none"), q.rowptr, q.col, q.val, tau=1e-2)
    x, code, it, atr, rel = S.solve(to_dev(b), tol=1e-14)
    o = oracle.lsqr_m(F, b, tol=1e-14, maxit=4)
    got = x.cpu().numpy()
    assert it == o.iters == 4 and np.linalg.norm(got - o.x) <= 1e-8 * np.linalg.norm(o.x)
    S.close()
    A = sp.vstack([p.scipy(), sp.csr_matrix((q.val, q.col, q.rowptr), shape=(q.m, p.n))]).tocsr()
    atb = np.linalg.norm(A.T @ b)
    for prec in (0, 1):
        S = R.Solver.from_problem(p, maxit=2000, precision=prec, **LSQR).upload()
        S.add_rows(q.rowptr, q.col, q.val)
        x, code, it, atr, rel = S.solve(to_dev(b), tol=1e-8)
        got = x.cpu().numpy()
        o = oracle.lsqr_m(F, b, tol=1e-8, maxit=2000)
        assert code == R.OK and o.status == "ok"
        if prec == 0:
            assert abs(it - o.iters) <= max(1, int(0.02 * o.iters)), (it, o.iters)
        assert np.linalg.norm(A.T @ (b - A @ got)) <= 2e-8 * atb
        assert np.linalg.norm(A.T @ (A @ (got - o.x))) <= 4e-8 * atb
        # the batched kernel on the updated handle
        bt = R.Batch(1)
        xs, res = bt.solve([S], [to_dev(b)], 1e-8)
        gb = xs[0].cpu().numpy()
        assert res[0]["status"] == R.OK
        assert np.linalg.norm(A.T @ (A @ (gb - o.x))) <= 4e-8 * atb
        bt.close()
        print("%s + %d rows precision %d: its %d (oracle %d), batched its %d" % (name, count, prec, it, o.iters,
                                                                              res[0]["iters"]))
        S.close()


def test_solve_before_upload_is_refused(gpu_lib):
    R = gpu_lib
    import torch

    p, q, b = augmented("c1", 10, 81)
    S = R.Solver.from_problem(p, **LSQR).upload()
    assert R.rsilu_add_rows(S.h, q.rowptr, q.col, q.val) == R.OK
    x = torch.empty(p.n, dtype=torch.float64, device="cuda")
    code, it, atr, rel = R.rsilu_solve(S.h, to_dev(b), 1e-8, x)
    assert code == R.ESTATE
    S.close()


def removal_case(seed=5, count=30):
    p = gen.tiny_c1()
    rows = np.sort(np.random.default_rng(seed).choice(p.m, count, replace=False))
    keep = np.setdiff1d(np.arange(p.m), rows)
    return p, rows, keep


DENSE = dict(mu=1.0, form=1, smode=1)  # Algorithm 2 form with the dense S~


@pytest.mark.parametrize("krylov", [0, 1])
def test_removal_four_steps_and_convergence(gpu_lib, krylov):
    """Rows removed (Section 3.4, Woodbury update for the A1 rows): the reduced solve follows
    the oracle on its updated operator for four steps and converges like it."""
    R = gpu_lib
    p, rows, keep = removal_case()
    b = p.b[keep]
    G = oracle.remove_rows(oracle.factor_problem(p, mu=1.0, smode="dense"), rows)
    assert G.R is not None and G.R.nrows > 0
    S = R.Solver.from_problem(p, maxit=4, krylov=krylov, **DENSE).upload()
    S.remove_rows(rows)
    x, code, it, atr, rel = S.solve(to_dev(b), tol=1e-14)
    o = oracle.lsqr_m(G, b, tol=1e-14, maxit=4) if krylov else oracle.pcgls(G, b, tol=1e-14, maxit=4, form="alg2")
    got = x.cpu().numpy()
    assert it == o.iters == 4 and np.linalg.norm(got - o.x) <= 1e-8 * np.linalg.norm(o.x)
    S.close()
    A = p.scipy()[keep]
    atb = np.linalg.norm(A.T @ b)
    S = R.Solver.from_problem(p, maxit=2000, krylov=krylov, **DENSE).upload()
    S.remove_rows(rows)
    x, code, it, atr, rel = S.solve(to_dev(b), tol=1e-8)
    got = x.cpu().numpy()
    o = oracle.lsqr_m(G, b, tol=1e-8, maxit=2000) if krylov else oracle.pcgls(G, b, tol=1e-8, maxit=2000,
                                                                               form="alg2")
    assert code == R.OK and o.status == "ok"
    assert abs(it - o.iters) <= max(1, int(0.02 * o.iters)), (it, o.iters)
    assert np.linalg.norm(A.T @ (b - A @ got)) <= 2e-8 * atb
    assert np.linalg.norm(A.T @ (A @ (got - o.x))) <= 4e-8 * atb
    print("tiny - 30 rows (%d from A1), krylov %d: its %d (oracle %d)" % (G.R.nrows, krylov, it, o.iters))
    # the batched kernel does not take the updated handle
    bt = R.Batch(1)
    import torch

    xb = torch.empty(p.n, dtype=torch.float64, device="cuda")
    assert bt.solve_raw([S.h], [to_dev(b)], [1e-8], [xb])[0] == R.EINVAL
    bt.close()
    S.close()


def test_removal_then_addition(gpu_lib):
    """Rows removed, then rows appended: W is rebuilt for the new operator; the solve
    follows the oracle's updated factors."""
    R = gpu_lib
    p, rows, keep = removal_case(seed=6, count=20)
    q = gen.random_sparse(15, p.n, k=5, seed=82, transversal=False)
    b = np.concatenate([p.b[keep], np.random.default_rng(83).standard_normal(15)])
    G = oracle.remove_rows(oracle.factor_problem(p, mu=1.0, smode="dense"), rows)
    G = oracle.add_rows(G, q.rowptr, q.col, q.val, tau=1e-2)
    S = R.Solver.from_problem(p, maxit=4, krylov=1, **DENSE).upload()
    S.remove_rows(rows)
    S.add_rows(q.rowptr, q.col, q.val)
    x, code, it, atr, rel = S.solve(to_dev(b), tol=1e-14)
    o = oracle.lsqr_m(G, b, tol=1e-14, maxit=4)
    assert it == o.iters == 4
    assert np.linalg.norm(x.cpu().numpy() - o.x) <= 1e-8 * np.linalg.norm(o.x)
    S.close()
