"""GPU parity of every level scheme of the single-workgroup sweeps, forced through
rsilu_params_t.sweep, against the oracle's substitutions.

Each scheme solves a row as rhs minus the sum of its products times the
reciprocal diagonal; they differ in how threads share the work and in the order
of the row sums. Held to the same bounds as the hybrid schedule in
test_gpu_parity.py (unit roundoff eps = 2^-53):
  * componentwise backward error |T x - rhs| <= 4 k eps (|T| |x| + |rhs|) per row
    (k = stored entries + 2), in FP64, and in FP32 against the FP32-rounded operands;
  * with mu = 1 (well-conditioned factors) the forward difference to the oracle's
    solution, normwise, at 1e-10 (not for the fill-heavy long-factor problem);
  * the two-phase and rows-per-thread schemes add a row's chunk sums in chunk order,
    so they must agree bit for bit; the segmented scheme sums over lanes in a tree.
The long-factor problem (ILUP(60, 0) on 40 entries per row) has factor rows of up
to 204 entries (51 chunks): under the segmented scheme those rows span several
16-lane groups of a wavefront and are summed with the wavefront-wide scan.
"""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps / 2
EPS32 = np.finfo(np.float32).eps / 2

PROBLEMS = {
    "c1": (lambda: gen.tiny_c1(), {}),
    "c2-small": (lambda: gen.by_name("c2-small"), {}),
    "long-factor": (lambda: gen.random_sparse(900, 600, k=40, seed=5), {"p": 60, "tau": 0.0}),
}


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def _solves(R, prob, F, params, sweep, rhs, precision=None):
    """The four triangular solves (L1, L1^T, U, U^T) of one handle, host results."""
    import torch

    kw = dict(mu=1.0, smode=R.S_IDENTITY, trsv=R.TRSV_HYBRID, sweep=sweep, **params)
    if precision is not None:
        kw.update(precision=precision, smode=R.S_NONE)
    S = R.Solver.from_problem(prob, **kw).upload()
    out = {}
    for which in (R.T_L1, R.T_L1T, R.T_U, R.T_UT):
        x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        assert R.rsilu_trsv(S.h, which, _dev(rhs), x) == R.OK
        out[which] = _host(x)
    S.close()
    return out


def _operators(R, F):
    return [(R.T_L1, F.L1, None, True), (R.T_L1T, F.L1T, None, False), (R.T_U, F.U, F.Udiag, False),
            (R.T_UT, F.UT, F.Udiag, True)]


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_every_scheme_against_oracle(gpu_lib, name):
    R = gpu_lib
    make, params = PROBLEMS[name]
    prob = make()
    F = oracle.factor_problem(prob, mu=1.0, smode="identity", **params)
    rhs = np.random.default_rng(21).standard_normal(prob.n)
    got = {}
    for sweep in (R.SWEEP_AUTO, R.SWEEP_TWO_PHASE, R.SWEEP_SEGMENTED, R.SWEEP_ROWS):
        got[sweep] = _solves(R, prob, F, params, sweep, rhs)
        for which, T, diag, lower in _operators(R, F):
            x = got[sweep][which]
            assert np.all(np.isfinite(x)), (name, sweep, which)
            Td = T.scipy()
            d = np.ones(prob.n) if diag is None else diag
            resid = Td @ x + d * x - rhs
            scale = np.abs(Td) @ np.abs(x) + np.abs(d * x) + np.abs(rhs)
            k = np.diff(T.rowptr) + 2
            assert np.all(np.abs(resid) <= 4 * k * EPS * scale), (name, sweep, which)
            if name != "long-factor":  # its fill-heavy factors are not well conditioned
                want = oracle.lower_solve(T, rhs, diag) if lower else oracle.upper_solve(T, rhs, diag)
                assert np.linalg.norm(x - want) <= 1e-10 * np.linalg.norm(want), (name, sweep, which)
    for which, _, _, _ in _operators(R, F):
        a, b = got[R.SWEEP_TWO_PHASE][which], got[R.SWEEP_ROWS][which]
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), (name, which)


def _schemes(R, prob, params, sweep, precision):
    """Level schemes the setup chose, per factor (bit s of byte f: scheme s in factor f)."""
    kw = dict(mu=1.0, smode=R.S_NONE, trsv=R.TRSV_HYBRID, sweep=sweep, precision=precision, **params)
    S = R.Solver.from_problem(prob, **kw)
    mask = S.stats.sweep_schemes
    S.close()
    return [(mask >> (8 * f)) & 0xFF for f in range(4)]


@pytest.mark.parametrize("name", ["c2-small", "long-factor"])
@pytest.mark.parametrize("sweep", ["two_phase", "segmented", "rows"])
def test_every_scheme_fp32(gpu_lib, sweep, name):
    """FP32 sweeps: backward error in FP32 against the FP32-rounded operands. On the
    long-factor problem the segmented scheme takes its wavefront-wide instantiation (rows of
    17 to 64 chunks), which the setup reports."""
    R = gpu_lib
    sw = {"two_phase": R.SWEEP_TWO_PHASE, "segmented": R.SWEEP_SEGMENTED, "rows": R.SWEEP_ROWS}[sweep]
    make, params = PROBLEMS[name]
    prob = make()
    F = oracle.factor_problem(prob, mu=1.0, smode="none", **params)
    schemes = _schemes(R, prob, params, sw, R.PREC_FP32)
    want_bit = {"two_phase": 1, "rows": 4}.get(sweep, 8 if name == "long-factor" else 2)
    assert any(m & want_bit for m in schemes), (sweep, name, schemes)
    rhs = np.random.default_rng(22).standard_normal(prob.n)
    rhs32 = rhs.astype(np.float32).astype(np.float64)
    got = _solves(R, prob, F, params, sw, rhs, precision=R.PREC_FP32)
    for which, T, diag, _ in _operators(R, F):
        x = got[which]
        assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
        T32 = T.scipy().astype(np.float32).astype(np.float64)
        d32 = np.ones(prob.n) if diag is None else diag.astype(np.float32).astype(np.float64)
        resid = T32 @ x + d32 * x - rhs32
        scale = abs(T32) @ np.abs(x) + np.abs(d32 * x) + np.abs(rhs32)
        k = np.diff(T.rowptr) + 2
        assert np.all(np.abs(resid) <= 4 * k * EPS32 * scale), (sweep, name, which)


@pytest.mark.parametrize("sweep", ["two_phase", "segmented", "rows"])
def test_every_scheme_lsqr_converges(gpu_lib, sweep):
    """A whole LSQR solve (Algorithm 2, no correction) with each scheme: converged, the
    true ||A^T r|| at the tolerance, iterations within 2% of the oracle's."""
    R = gpu_lib
    sw = {"two_phase": R.SWEEP_TWO_PHASE, "segmented": R.SWEEP_SEGMENTED, "rows": R.SWEEP_ROWS}[sweep]
    prob = gen.by_name("c2-small")
    tol = 1e-8
    S = R.Solver.from_problem(prob, mu=1.0, form=R.FORM_ALG2, smode=R.S_NONE, krylov=R.KRYLOV_LSQR,
                              sweep=sw).upload()
    x, code, it, atr, rel = S.solve(_dev(prob.b), tol=tol)
    got = _host(x)
    S.close()
    F = oracle.factor_problem(prob, mu=1.0, smode="none")
    res = oracle.lsqr_m(F, prob.b, tol=tol, maxit=2000)
    assert code == R.OK and res.status == "ok"
    assert abs(it - res.iters) <= max(1, int(0.02 * res.iters)), (it, res.iters)
    A = prob.scipy()
    atb = np.linalg.norm(A.T @ prob.b)
    assert np.linalg.norm(A.T @ (prob.b - A @ got)) <= 2 * tol * atb
