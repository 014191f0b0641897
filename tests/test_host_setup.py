"""The library's host setup (rsilu_factor) against the oracle, through the C ABI.

The row permutation, every factor entry, the column norms and the level
schedules must be bit-identical: both sides take the same floating-point
decisions in the same order (Algorithms 4-6). No GPU is needed: rsilu_factor
and the getters are host code.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import gen
import oracle
from paper_2603_28642_amd import rsilu as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dense_problem(A):
    A = np.asarray(A, dtype=float)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return m, n, rowptr, cols.astype(np.int32), A[rows, cols]


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.int64)


def compare(m, n, rowptr, col, val, p=10, tau=1e-2, mu=0.1, small=1e-10, colscale=1):
    prm = R.rsilu_params_default(p=p, tau=tau, mu=mu, small=small, colscale=colscale, smode=R.S_IDENTITY)
    code, h = R.rsilu_factor(m, n, rowptr, col, val, prm)
    assert code == R.OK, R.status_string(code)
    try:
        F = oracle.factor(m, n, rowptr, col, val, p=p, tau=tau, mu=mu, small=small, colscale=bool(colscale))
        st = R.rsilu_get_stats(h)
        assert np.array_equal(R.rsilu_get_perm(h, m), F.perm)
        assert st.nmod == F.nmod
        for which, C in [(R.L1, F.L1), (R.L2, F.L2), (R.U, F.U), (R.AHAT, F.Ahat)]:
            rp, cc, vv = R.rsilu_get_factor(h, which, C.nrows)
            assert np.array_equal(rp, C.rowptr), which
            assert np.array_equal(cc, C.col), which
            assert np.array_equal(bits(vv), bits(C.val)), which
        assert np.array_equal(bits(R.rsilu_get_factor(h, R.UDIAG, n)), bits(F.Udiag))
        assert np.array_equal(bits(R.rsilu_get_colnorm(h, n)), bits(F.colnorm))
        for which, key, nl in [(R.LEV_L1, "L1", st.levels_l1), (R.LEV_L1T, "L1T", st.levels_l1t),
                               (R.LEV_U, "U", st.levels_u), (R.LEV_UT, "UT", st.levels_ut)]:
            ptr, rows = R.rsilu_get_levels(h, which, n, nl)
            assert np.array_equal(ptr, F.lev[key][0]), key
            assert np.array_equal(rows, F.lev[key][1]), key
        assert st.psize == F.psize
        return st
    finally:
        R.rsilu_destroy(h)


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini"])
@pytest.mark.parametrize("mu", [0.1, 1.0])
def test_named_workloads(name, mu):
    p = gen.by_name(name)
    compare(p.m, p.n, p.rowptr, p.col, p.val, mu=mu)


@pytest.mark.parametrize("key", list(gen.PAPER_SHAPES))
@pytest.mark.parametrize("tau", [0.0, 0.1])
def test_paper_shapes(key, tau):
    p = gen.paper_shape(key, scale=0.15, seed=3)
    compare(p.m, p.n, p.rowptr, p.col, p.val, tau=tau)


@pytest.mark.parametrize("p_,tau,mu", [(1, 0.0, 0.1), (3, 0.05, 0.5), (10**9, 0.0, 1.0), (0, 0.0, 0.1)])
def test_parameter_corners(p_, tau, mu):
    p = gen.random_sparse(120, 90, k=5, seed=4)
    compare(p.m, p.n, p.rowptr, p.col, p.val, p=p_, tau=tau, mu=mu)


def test_edge_matrices():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((12, 8)) * (rng.random((12, 8)) < 0.4)
    A[:, 3] = 0.0  # empty column
    A[:, 5] = A[:, 4]  # duplicated column
    compare(*dense_problem(A))
    compare(*dense_problem(np.zeros((4, 3))))  # all pivots modified
    compare(*dense_problem(np.eye(5)))  # m = n
    B = np.ones((6, 4))  # exact ties everywhere
    compare(*dense_problem(B))
    compare(*dense_problem(B), colscale=0)
    C = rng.standard_normal((30, 10))
    C[29, :] = 1.0  # a dense row
    compare(*dense_problem(C), p=2)


def test_explicit_zeros_are_stripped():
    m, n, rp, c, v = dense_problem(np.array([[1.0, 2.0], [3.0, 0.0], [0.0, 4.0]]))
    v2 = v.copy()
    v2[1] = 0.0  # (0,1) becomes an explicit zero
    code, h = R.rsilu_factor(m, n, rp, c, v2)
    assert code == R.OK
    st = R.rsilu_get_stats(h)
    assert st.nnz_a == 3
    R.rsilu_destroy(h)


@pytest.mark.parametrize("case", ["m<n", "bad col", "unsorted", "duplicate", "nan", "inf", "bad ptr", "bad mu",
                                  "bad tau", "bad small", "bad form", "bad smode", "bad precision",
                                  "fp32 syncfree", "fp32 dense", "cg fp32", "cg syncfree", "cg steps",
                                  "lsqr alg3", "lsqr identity", "lsqr syncfree", "bad krylov", "bad sweep",
                                  "negative sweep"])
def test_invalid_input(case):
    m, n, rp, c, v = dense_problem(np.array([[1.0, 2.0], [3.0, 0.0], [0.0, 4.0]]))
    prm = R.rsilu_params_default()
    if case == "m<n":
        m2, n2, rp2, c2, v2 = dense_problem(np.array([[1.0, 2.0, 3.0]]))
        code, h = R.rsilu_factor(m2, n2, rp2, c2, v2)
    else:
        c = c.copy()
        v = v.copy()
        rp = rp.copy()
        if case == "bad col":
            c[0] = 7
        elif case == "unsorted":
            c[0], c[1] = c[1], c[0]
        elif case == "duplicate":
            c[1] = c[0]
        elif case == "nan":
            v[2] = np.nan
        elif case == "inf":
            v[2] = np.inf
        elif case == "bad ptr":
            rp[1] = 3
            rp[2] = 1
        elif case == "bad mu":
            prm.mu = 1.5
        elif case == "bad tau":
            prm.tau = -1.0
        elif case == "bad small":
            prm.small = 0.0
        elif case == "bad form":
            prm.form = 2
        elif case == "bad smode":
            prm.smode = 5
        elif case == "bad precision":
            prm.precision = 2
        elif case == "fp32 syncfree":
            prm.precision = R.PREC_FP32
            prm.trsv = R.TRSV_SYNCFREE
        elif case == "fp32 dense":
            prm.precision = R.PREC_FP32
            prm.smode = R.S_DENSE
        elif case == "cg fp32":
            prm.smode = R.S_CG
            prm.precision = R.PREC_FP32
        elif case == "cg syncfree":
            prm.smode = R.S_CG
            prm.trsv = R.TRSV_SYNCFREE
        elif case == "cg steps":
            prm.smode = R.S_CG
            prm.cg_steps = 0
        elif case == "lsqr alg3":
            prm.krylov = R.KRYLOV_LSQR
        elif case == "lsqr identity":
            prm.krylov = R.KRYLOV_LSQR
            prm.form = R.FORM_ALG2
            prm.smode = R.S_IDENTITY
        elif case == "lsqr syncfree":
            prm.krylov = R.KRYLOV_LSQR
            prm.form = R.FORM_ALG2
            prm.trsv = R.TRSV_SYNCFREE
        elif case == "bad krylov":
            prm.krylov = 2
        elif case == "bad sweep":
            prm.sweep = 4
        elif case == "negative sweep":
            prm.sweep = -1
        code, h = R.rsilu_factor(m, n, rp, c, v, prm)
    assert code == R.EINVAL and h is None


def test_dense_S_setup():
    p = gen.random_sparse(90, 60, k=4, seed=8)
    prm = R.rsilu_params_default(smode=R.S_DENSE, mu=1.0)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    st = R.rsilu_get_stats(h)
    F = oracle.factor_problem(p, mu=1.0, smode="dense")
    assert st.smode == R.S_DENSE and st.psize == F.psize
    R.rsilu_destroy(h)
    # AUTO picks dense for small m - n and identity otherwise
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, R.rsilu_params_default())
    assert R.rsilu_get_stats(h).smode == R.S_DENSE
    R.rsilu_destroy(h)


def test_device_calls_need_upload():
    p = gen.random_sparse(30, 20, k=3, seed=1)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val)
    assert R.rsilu_device_bytes(h) > 0
    dummy = ctypes.c_void_p(0x1000)
    assert R.lib().rsilu_solve(h, dummy, 1e-8, ctypes.c_void_p(0x2000), None, None, None, None) == R.ESTATE
    assert R.lib().rsilu_spmv(h, 0, dummy, ctypes.c_void_p(0x2000), None) == R.ESTATE
    assert R.lib().rsilu_upload(h, ctypes.c_void_p(0x1001), 1 << 30, None) == R.EINVAL  # misaligned
    assert R.lib().rsilu_upload(h, ctypes.c_void_p(0x1000), 16, None) == R.ENOMEM  # too small
    # profiling classes: bits below RSILU_PROF_COUNT only
    assert R.lib().rsilu_set_profiling_mask(h, 1 << len(R.PROF_NAMES)) == R.EINVAL
    assert R.lib().rsilu_set_profiling_mask(None, 1) == R.EINVAL
    assert R.rsilu_set_profiling_mask(h, R.PROF_NAMES) == R.OK
    assert R.rsilu_set_profiling_mask(h, []) == R.OK
    R.rsilu_destroy(h)
    R.rsilu_destroy(None)


def test_exports_match_header():
    """Every function declared in include/*.h is exported by the library."""
    text = ""
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            with open(os.path.join(ROOT, "include", fn)) as f:
                text += f.read()
    declared = sorted(set(re.findall(r"\b(rsilu_[a-z_]+)\s*\(", text)))
    assert declared == sorted(R.EXPORTS)
    for name in declared:
        assert hasattr(R.lib(), name)
    for code in [0, 1, 2, -1, -2, -3, -4, -5]:
        assert R.status_string(code)


def test_no_oracle_in_product():
    """The library and its binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2603_28642_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    src = f.read()
                assert "oracle" not in src.lower(), fn


def test_fp32_auto_resolves_to_identity_and_shrinks_footprint():
    p = gen.random_sparse(90, 60, k=4, seed=8)
    code, h64 = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, R.rsilu_params_default(smode=R.S_AUTO, mu=1.0))
    code2, h32 = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val,
                                R.rsilu_params_default(smode=R.S_AUTO, mu=1.0, precision=R.PREC_FP32))
    assert code == R.OK and code2 == R.OK
    s64, s32 = R.rsilu_get_stats(h64), R.rsilu_get_stats(h32)
    assert s64.smode == R.S_DENSE and s32.smode == R.S_IDENTITY
    big = gen.by_name("c2-small")
    a = R.rsilu_factor(big.m, big.n, big.rowptr, big.col, big.val, R.rsilu_params_default(mu=1.0, smode=R.S_NONE))[1]
    b = R.rsilu_factor(big.m, big.n, big.rowptr, big.col, big.val,
                       R.rsilu_params_default(mu=1.0, smode=R.S_NONE, precision=R.PREC_FP32))[1]
    # factor values and sweep blobs shrink by about a third
    assert R.rsilu_device_bytes(b) < 0.8 * R.rsilu_device_bytes(a)
    for hh in (h64, h32, a, b):
        R.rsilu_destroy(hh)


def test_lsqr_auto_resolves_to_spd_modes():
    small = gen.random_sparse(90, 60, k=4, seed=8)
    big = gen.by_name("c2-small")
    for p, want in [(small, R.S_DENSE), (big, R.S_NONE)]:
        prm = R.rsilu_params_default(mu=1.0, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR, smode=R.S_AUTO)
        code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
        assert code == R.OK
        assert R.rsilu_get_stats(h).smode == want
        R.rsilu_destroy(h)


def test_full_size_grid_setup_bit_exact():
    """The grid workload at its full size (600000 x 400000): permutation, factors and level
    schedules bit-identical to the oracle's."""
    p = gen.by_name("c2")
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_NONE)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    F = oracle.factor_problem(p, mu=1.0, smode="none")
    st = R.rsilu_get_stats(h)
    assert np.array_equal(R.rsilu_get_perm(h, p.m), F.perm)
    for which, C in [(R.L1, F.L1), (R.L2, F.L2), (R.U, F.U)]:
        rp, col, val = R.rsilu_get_factor(h, which, C.nrows)
        assert np.array_equal(rp, C.rowptr) and np.array_equal(col, C.col) and np.array_equal(bits(val), bits(C.val))
    assert np.array_equal(bits(R.rsilu_get_factor(h, R.UDIAG, p.n)), bits(F.Udiag))
    for which, key, nl in [(R.LEV_L1, "L1", st.levels_l1), (R.LEV_U, "U", st.levels_u)]:
        ptr, rows = R.rsilu_get_levels(h, which, p.n, nl)
        want_ptr, want_rows = F.lev[key]
        assert np.array_equal(ptr, want_ptr) and np.array_equal(rows, want_rows)
    R.rsilu_destroy(h)


def test_batch_api_host_checks():
    """Argument checks of the batched-solve and autotuner entry points that need no device."""
    L = R.lib()
    tiles = R.rsilu_batch_tiles()
    assert len(tiles) == 12 and len(set(tiles)) == 12
    assert all(t in {256, 512, 1024} and s in {4, 8} and g in {1, 4} for t, s, g in tiles)
    h = ctypes.c_void_p()
    assert L.rsilu_batch_create(0, ctypes.byref(h)) == R.EINVAL
    assert L.rsilu_batch_create(70000, ctypes.byref(h)) == R.EINVAL
    assert L.rsilu_batch_create(4, None) == R.EINVAL
    assert L.rsilu_tuner_create(0.0, 8, ctypes.byref(h)) == R.EINVAL
    assert L.rsilu_tuner_create(float("inf"), 8, ctypes.byref(h)) == R.EINVAL
    assert L.rsilu_tuner_create(1.0, 1, ctypes.byref(h)) == R.EINVAL
    res = (R.rsilu_batch_result_t * 1)()
    assert L.rsilu_batch_solve(None, 0, None, None, None, None, None, res, None) == R.EINVAL
    tr = R.rsilu_tune_result_t()
    assert L.rsilu_tune(None, None, None, None, ctypes.byref(tr), None) == R.EINVAL
    assert L.rsilu_tuner_size(None) == 0
    L.rsilu_batch_destroy(None)
    L.rsilu_tuner_destroy(None)


@pytest.mark.parametrize("precision", [0, 1])
def test_add_rows_bit_exact(precision):
    """rsilu_add_rows against the oracle's add_rows: row order, A_hat and every L2 entry
    bit-identical; L1, U and the level schedules unchanged; the device layout must be
    uploaded again."""
    p = gen.by_name("c2-small")
    q = gen.random_sparse(300, p.n, k=5, seed=71, transversal=False)
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_NONE, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR, precision=precision)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    before = R.rsilu_device_bytes(h)
    assert R.rsilu_add_rows(h, q.rowptr, q.col, q.val) == R.OK
    F = oracle.add_rows(oracle.factor_problem(p, mu=1.0, smode="none"), q.rowptr, q.col, q.val, tau=1e-2)
    st = R.rsilu_get_stats(h)
    assert st.m == p.m + 300 and st.nnz_a == p.nnz + q.nnz and R.rsilu_device_bytes(h) > before
    assert np.array_equal(R.rsilu_get_perm(h, st.m), F.perm)
    for which, C in [(R.L1, F.L1), (R.L2, F.L2), (R.U, F.U), (R.AHAT, F.Ahat)]:
        rp, cc, vv = R.rsilu_get_factor(h, which, C.nrows)
        assert np.array_equal(rp, C.rowptr) and np.array_equal(cc, C.col), which
        assert np.array_equal(bits(vv), bits(C.val)), which
    for which, key, nl in [(R.LEV_L1, "L1", st.levels_l1), (R.LEV_U, "U", st.levels_u)]:
        ptr, rows = R.rsilu_get_levels(h, which, p.n, nl)
        assert np.array_equal(ptr, F.lev[key][0]) and np.array_equal(rows, F.lev[key][1])
    R.rsilu_destroy(h)


def test_add_rows_rejects_bad_rows():
    p = gen.tiny_c1()
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_NONE)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    st0 = R.rsilu_get_stats(h)
    bad = [
        ([0, 2], [5, 3], [1.0, 2.0]),          # unsorted
        ([0, 2], [3, 3], [1.0, 2.0]),          # repeated
        ([0, 1], [p.n], [1.0]),                # out of range
        ([0, 1], [-1], [1.0]),
        ([0, 1], [4], [float("nan")]),
        ([1, 2], [4, 5], [1.0, 1.0]),          # pointer not from 0
        ([0], [], []),                         # no row
    ]
    for rp, cc, vv in bad:
        assert R.rsilu_add_rows(h, np.array(rp), np.array(cc, dtype=np.int32), np.array(vv)) == R.EINVAL, rp
    st = R.rsilu_get_stats(h)
    assert st.m == st0.m and st.nnz_a == st0.nnz_a and R.rsilu_device_bytes(h) == st0.device_bytes
    assert R.lib().rsilu_add_rows(None, 1, None, None, None) == R.EINVAL
    R.rsilu_destroy(h)


def test_remove_rows_bit_exact():
    """rsilu_remove_rows against the oracle's remove_rows: row order, A_hat and every L2
    entry bit-identical, R the removed A1 rows; other configurations are refused with the
    handle unchanged."""
    p = gen.tiny_c1()
    rows = np.sort(np.random.default_rng(5).choice(p.m, 30, replace=False))
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_DENSE, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    assert R.rsilu_remove_rows(h, rows) == R.OK
    F = oracle.remove_rows(oracle.factor_problem(p, mu=1.0, smode="dense"), rows)
    st = R.rsilu_get_stats(h)
    assert st.m == p.m - 30
    assert np.array_equal(R.rsilu_get_perm(h, st.m), F.perm)
    for which, C in [(R.L1, F.L1), (R.L2, F.L2), (R.U, F.U), (R.AHAT, F.Ahat)]:
        rp, cc, vv = R.rsilu_get_factor(h, which, C.nrows)
        assert np.array_equal(rp, C.rowptr) and np.array_equal(cc, C.col), which
        assert np.array_equal(bits(vv), bits(C.val)), which
    R.rsilu_destroy(h)
    # refused: S^ none, bad indices (handle unchanged)
    prm2 = R.rsilu_params_default(mu=1.0, smode=R.S_NONE, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR)
    code, h2 = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm2)
    assert R.rsilu_remove_rows(h2, np.array([1])) == R.EINVAL
    R.rsilu_destroy(h2)
    code, h3 = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    b0 = R.rsilu_device_bytes(h3)
    for bad in ([3, 3], [-1], [p.m], list(range(p.m - p.n + 1))):
        assert R.rsilu_remove_rows(h3, np.array(bad, dtype=np.int64)) == R.EINVAL, bad
    assert R.rsilu_get_stats(h3).m == p.m and R.rsilu_device_bytes(h3) == b0
    assert R.lib().rsilu_remove_rows(h3, 0, None) == R.EINVAL
    R.rsilu_destroy(h3)


@pytest.mark.parametrize("sweep", [0, 1, 2, 3])
def test_every_sweep_scheme_sets_up(sweep):
    """Every level scheme of the sweeps builds, and leaves the factors and level
    schedules as they are (the scheme only changes the sweep blobs)."""
    import gen

    p = gen.random_sparse(900, 600, k=40, seed=5)
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_IDENTITY, p=60, tau=0.0, sweep=sweep)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    ref_prm = R.rsilu_params_default(mu=1.0, smode=R.S_IDENTITY, p=60, tau=0.0)
    code, h0 = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, ref_prm)
    assert code == R.OK
    for which in (R.L1, R.U):
        a, b = R.rsilu_get_factor(h, which, p.n), R.rsilu_get_factor(h0, which, p.n)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    st, st0 = R.rsilu_get_stats(h), R.rsilu_get_stats(h0)
    assert (st.levels_l1, st.levels_u) == (st0.levels_l1, st0.levels_u)
    R.rsilu_destroy(h)
    R.rsilu_destroy(h0)


def compare_Y(prob, ytau, mu=1.0, precision=0):
    prm = R.rsilu_params_default(mu=mu, smode=R.S_CG, form=R.FORM_ALG2, ystore=R.Y_EXPLICIT, ytau=ytau,
                                 cg_steps=8, precision=precision)
    if precision == 1:
        prm.smode = R.S_IDENTITY
    code, h = R.rsilu_factor(prob.m, prob.n, prob.rowptr, prob.col, prob.val, prm)
    assert code == R.OK, R.status_string(code)
    try:
        F = oracle.factor_problem(prob, mu=mu, smode="cg", ystore=True, ytau=ytau)
        st = R.rsilu_get_stats(h)
        assert st.nnz_y == F.Y.nnz
        rp, cc, vv = R.rsilu_get_factor(h, R.YEXP, F.Y.nrows)
        assert np.array_equal(rp, F.Y.rowptr) and np.array_equal(cc, F.Y.col)
        assert np.array_equal(bits(vv), bits(F.Y.val))
        return st
    finally:
        R.rsilu_destroy(h)


@pytest.mark.parametrize("name", ["c1", "c2-small", "c3-mini"])
@pytest.mark.parametrize("ytau", [0.0, 1e-3, 1e-2])
def test_explicit_Y_bit_exact(name, ytau):
    """The explicit Y~ = L2 L1^{-1} with dropping (Section 3.2): every entry bit-identical to
    the oracle's substitution (same finishing order, same separately rounded updates)."""
    compare_Y(gen.by_name(name), ytau)


def test_explicit_Y_fp32_handle_and_stats():
    st = compare_Y(gen.by_name("c2-small"), 1e-2, precision=1)
    assert st.nnz_y > 0


def test_explicit_Y_full_size_bit_exact():
    """The explicit Y~ of the 600000 x 400000 grid workload (ytau = 1e-2): bit-identical."""
    st = compare_Y(gen.by_name("c2"), 1e-2)
    assert st.nnz_y > 10_000_000


def test_explicit_Y_rejected_configurations():
    p = gen.tiny_c1()
    bad = [dict(ystore=R.Y_EXPLICIT, smode=R.S_DENSE), dict(ystore=R.Y_EXPLICIT, trsv=R.TRSV_SYNCFREE),
           dict(ystore=R.Y_EXPLICIT, ytau=-1.0), dict(ystore=R.Y_EXPLICIT, ytau=float("nan")), dict(ystore=2),
           dict(smode=R.S_CG, cg_steps=257), dict(smode=R.S_CG, cg_steps=0)]
    for kw in bad:
        prm = R.rsilu_params_default(mu=1.0, **kw)
        code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
        assert code == R.EINVAL and h is None, kw
    # AUTO with the explicit Y~ never picks the dense S~
    prm = R.rsilu_params_default(mu=1.0, ystore=R.Y_EXPLICIT)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK and R.rsilu_get_stats(h).smode == R.S_IDENTITY
    assert R.rsilu_factor_nnz(h, R.YEXP) == R.rsilu_get_stats(h).nnz_y > 0
    R.rsilu_destroy(h)
    # without it, Y~ cannot be exported
    prm = R.rsilu_params_default(mu=1.0)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert R.rsilu_factor_nnz(h, R.YEXP) == -1 and R.rsilu_get_stats(h).nnz_y == 0
    R.rsilu_destroy(h)


def test_add_rows_rebuilds_explicit_Y():
    p = gen.by_name("c2-small")
    q = gen.random_sparse(300, p.n, k=5, seed=71, transversal=False)
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_CG, cg_steps=8, form=R.FORM_ALG2, ystore=R.Y_EXPLICIT, ytau=1e-2)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    assert R.rsilu_add_rows(h, q.rowptr, q.col, q.val) == R.OK
    F = oracle.add_rows(oracle.factor_problem(p, mu=1.0, smode="cg", ystore=True, ytau=1e-2), q.rowptr, q.col,
                        q.val, tau=1e-2)
    rp, cc, vv = R.rsilu_get_factor(h, R.YEXP, F.Y.nrows)
    assert F.Y.nrows == p.m - p.n + 300
    assert np.array_equal(rp, F.Y.rowptr) and np.array_equal(cc, F.Y.col) and np.array_equal(bits(vv), bits(F.Y.val))
    R.rsilu_destroy(h)


@pytest.mark.parametrize("name,ystore", [("c1", 1), ("c2-small", 1), ("c2-small", 0), ("c3-mini", 1)])
def test_chebyshev_plan_matches_oracle(name, ystore):
    """The Chebyshev interval (b = 1.05 x a 50-step power-iteration estimate of lambda_max(S~))
    and its degree agree with the oracle's; the two sums are ordered differently, so b to
    1e-12 relative and the degree exactly."""
    p = gen.by_name(name)
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_CHEB, form=R.FORM_ALG2, ystore=ystore, ytau=1e-2)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK
    st = R.rsilu_get_stats(h)
    F = oracle.factor_problem(p, mu=1.0, smode="cheb", ystore=bool(ystore), ytau=1e-2)
    assert st.smode == R.S_CHEB
    assert abs(st.cheb_b - F.cheb_b) <= 1e-12 * F.cheb_b and st.cheb_degree == F.cheb_degree
    assert st.cheb_degree % 2 == 0 and st.cheb_degree > 0
    assert st.cheb_scale == F.cheb_omega == 1.0  # the default degree meets its bound
    R.rsilu_destroy(h)
    # a fixed degree is taken as given; LSQR accepts the Chebyshev M_b; bad settings are rejected
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_CHEB, form=R.FORM_ALG2, krylov=R.KRYLOV_LSQR, ystore=ystore,
                                 poly_degree=7)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    assert code == R.OK and R.rsilu_get_stats(h).cheb_degree == 7
    R.rsilu_destroy(h)
    # degree 2 on an interval it cannot cover: the input scale 1 / (1 + eps_2), as the oracle's
    prm = R.rsilu_params_default(mu=1.0, smode=R.S_CHEB, form=R.FORM_ALG2, ystore=ystore, poly_degree=2)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
    st = R.rsilu_get_stats(h)
    F2 = oracle.factor_problem(p, mu=1.0, smode="cheb", ystore=bool(ystore), ytau=1e-2, poly_degree=2)
    assert code == R.OK and st.cheb_degree == 2 and (F2.cheb_omega < 1) == (name != "c1")  # c1: b = 3.3
    assert abs(st.cheb_scale - F2.cheb_omega) <= 1e-13 * F2.cheb_omega
    R.rsilu_destroy(h)
    for kw in (dict(poly_degree=-1), dict(poly_degree=513), dict(poly_delta=0.0), dict(poly_delta=1.0),
               dict(trsv=R.TRSV_SYNCFREE), dict(precision=R.PREC_FP32, ystore=0)):
        prm = R.rsilu_params_default(mu=1.0, smode=R.S_CHEB, form=R.FORM_ALG2, ystore=ystore)
        for k_, v_ in kw.items():
            setattr(prm, k_, v_)
        code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
        assert code == R.EINVAL and h is None, kw


def test_sweep_schemes_reported():
    """The level schemes the setup picks per factor (stats.sweep_schemes): forced schemes
    everywhere; the segmented one takes its wavefront-wide instantiation (bit 3) for the
    factors with rows of 17 to 64 chunks, in FP64 and FP32; multi-CU levels (bit 7) on the
    grid case's wide levels."""
    long_factor = (gen.random_sparse(900, 600, k=40, seed=5), dict(p=60, tau=0.0))
    grid = (gen.by_name("c2-small"), {})

    def masks(case, sweep, precision):
        p, kw = case
        prm = R.rsilu_params_default(mu=1.0, smode=R.S_NONE, sweep=sweep, precision=precision, **kw)
        code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
        assert code == R.OK
        m = R.rsilu_get_stats(h).sweep_schemes
        R.rsilu_destroy(h)
        return [(m >> (8 * f)) & 0xFF for f in range(4)]

    for prec in (R.PREC_FP64, R.PREC_FP32):
        assert masks(long_factor, R.SWEEP_TWO_PHASE, prec) == [1, 1, 1, 1]
        assert masks(long_factor, R.SWEEP_ROWS, prec) == [4, 4, 4, 4]
        seg = masks(long_factor, R.SWEEP_SEGMENTED, prec)
        assert seg[0] == 8 and seg[2] == 8 and seg[1] == 2 and seg[3] == 2  # L1, U: rows up to 51 chunks
        assert masks(long_factor, R.SWEEP_AUTO, prec) == seg
        g = masks(grid, R.SWEEP_AUTO, prec)
        assert all(m & 0x7F == 2 for m in g) and g[0] & 0x80 and g[3] & 0x80


def test_jacobi_cg_settings():
    """The Jacobi-preconditioned CG steps need the CG M_b and the explicit Y~; its diagonal is
    that of the oracle's (1 + squared row norms of Y~, here in Y~'s device row order)."""
    p = gen.by_name("c1")
    ok = R.rsilu_params_default(mu=1.0, smode=R.S_CG, form=R.FORM_ALG2, ystore=R.Y_EXPLICIT, cg_precond=R.CG_JACOBI)
    code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, ok)
    assert code == R.OK
    R.rsilu_destroy(h)
    for kw in (dict(ystore=R.Y_IMPLICIT), dict(smode=R.S_CHEB), dict(smode=R.S_IDENTITY), dict(cg_precond=2),
               dict(cg_precond=-1)):
        prm = R.rsilu_params_default(mu=1.0, smode=R.S_CG, form=R.FORM_ALG2, ystore=R.Y_EXPLICIT,
                                     cg_precond=R.CG_JACOBI)
        for k_, v_ in kw.items():
            setattr(prm, k_, v_)
        code, h = R.rsilu_factor(p.m, p.n, p.rowptr, p.col, p.val, prm)
        assert code == R.EINVAL and h is None, kw
