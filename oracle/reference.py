"""CPU FP64 oracle for the row-splitting ILU least-squares method.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the GPU library never imports it, and it
imports nothing from the library.

It follows the paper step by step:
  * prescale            Section 5.1 (unit 2-norm columns)
  * ilup                Algorithms 4-6 (rectangular ILUP(p, tau), threshold
                        partial pivoting, minimum row count, Li-Shao pivot
                        modification), sequential C in oracle_core.c
  * extract             the splitting (3.8): P A ~ [L1; L2] U
  * levels              dependency depths of the triangular factors
  * dense_S             S~ = I + Y~ Y~^T with Y~ = L2 L1^{-1}, (3.9), factored
                        once by Cholesky (Section 3.2)
  * explicit_Y          Y~ stored as a sparse matrix (Section 3.2), by back
                        substitution with L1^T on each row of L2, entries
                        below a drop tolerance dropped
  * cg_S                S~ w = u by a fixed number of CG steps, S~ applied
                        implicitly (Section 3.2, Table 3(a))
  * apply_alg3          Algorithm 3 on the residual components (r1, r2)
  * apply_alg2          Algorithm 2 with k = n on z = A^T r, M_a = (L1 U)^T
                        (L1 U) standing for C1 and A2 for its factored image
                        L2 U (Section 3.3 gives Y~ = L2 L1^{-1} in that sense)
  * pcgls               Algorithm 1 (left-preconditioned, factorization-free
                        CGLS) with Algorithm 3 (or Algorithm 2) in place of
                        h = M^{-1} A^T r
  * lsqr_m              LSQR (Paige and Saunders) on A_hat N with N N^T = M^{-1}
                        the SPD Algorithm 2 operator, written so that only
                        M^{-1} is applied (mathematically the same iterates
                        as Algorithm 1 with that M, which the paper notes for
                        CGLS and LSQR in exact arithmetic)
The method does not converge to anything faster than it converges; its limit
is the least-squares solution, which the tests pin with dense QR.
"""

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build(quiet=True)
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.orc_prescale.argtypes = [I64, P, P, P, P, P]
        lib.orc_prescale.restype = ctypes.c_int
        lib.orc_ilup.argtypes = [I64, I64, P, P, P, I64, D, D, D, P, P, P, P, I64, P, P, P, I64, P]
        lib.orc_ilup.restype = ctypes.c_int
        lib.orc_csr_matvec.argtypes = [I64, P, P, P, P, P]
        lib.orc_csr_matvec.restype = None
        lib.orc_lower_solve.argtypes = [I64, P, P, P, P, P, P]
        lib.orc_lower_solve.restype = I64
        lib.orc_upper_solve.argtypes = [I64, P, P, P, P, P, P]
        lib.orc_upper_solve.restype = I64
        lib.orc_levels.argtypes = [I64, P, P, ctypes.c_int, P]
        lib.orc_levels.restype = None
        lib.orc_explicit_y.argtypes = [I64, I64, I64, P, P, P, P, P, P, D, I64, P, P, P]
        lib.orc_explicit_y.restype = I64
        lib.orc_dot.argtypes = [I64, P, P]
        lib.orc_dot.restype = D
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ----------------------------------------------------------------------------
# sparse containers (plain CSR triples)


@dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: np.ndarray  # int64
    col: np.ndarray  # int32
    val: np.ndarray  # float64

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def scipy(self):
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))

    def dense(self):
        return self.scipy().toarray()

    def matvec(self, x):
        """y = A x, sequential sums in stored order."""
        x = _c(x, np.float64)
        assert x.shape == (self.ncols,)
        y = np.empty(self.nrows)
        _load().orc_csr_matvec(self.nrows, _p(self.rowptr), _p(self.col), _p(self.val), _p(x), _p(y))
        return y

    def transpose(self):
        t = self.scipy().T.tocsr()
        t.sort_indices()
        return CSR(self.ncols, self.nrows, t.indptr.astype(np.int64), t.indices.astype(np.int32),
                   t.data.astype(np.float64))


def csr_from_scipy(a):
    a = a.tocsr()
    a.sort_indices()
    return CSR(a.shape[0], a.shape[1], a.indptr.astype(np.int64), a.indices.astype(np.int32),
               a.data.astype(np.float64))


def lower_solve(L, b, diag=None):
    """Forward substitution with lower-triangular CSR L (unit diagonal if diag is None)."""
    b = _c(b, np.float64)
    x = np.empty(L.nrows)
    d = None if diag is None else _c(diag, np.float64)
    bad = _load().orc_lower_solve(L.nrows, _p(L.rowptr), _p(L.col), _p(L.val), _p(d), _p(b), _p(x))
    if bad:
        raise ValueError("matrix is not strictly lower triangular at row %d" % (bad - 1))
    return x


def upper_solve(U, b, diag=None):
    """Back substitution with upper-triangular CSR U (unit diagonal if diag is None)."""
    b = _c(b, np.float64)
    x = np.empty(U.nrows)
    d = None if diag is None else _c(diag, np.float64)
    bad = _load().orc_upper_solve(U.nrows, _p(U.rowptr), _p(U.col), _p(U.val), _p(d), _p(b), _p(x))
    if bad:
        raise ValueError("matrix is not strictly upper triangular at row %d" % (bad - 1))
    return x


def dot(a, b):
    """(a, b): the correctly rounded sum (math.fsum) of the rounded products a_i b_i. It does
    not depend on the order of the terms, and its error is below that of any summation
    order a GPU reduction may take. Non-finite products or an overflowing sum give the
    plain sum (inf or nan), as an IEEE summation would."""
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    assert a.shape == b.shape
    with np.errstate(over="ignore", invalid="ignore"):
        p = a * b
    if not np.all(np.isfinite(p)):
        return float(np.sum(p))  # inf or nan: the caller's breakdown test sees it
    try:
        return math.fsum(p)
    except OverflowError:  # the exact sum leaves the double range
        return float(np.sum(p))


def explicit_Y(L1, L2, tauY):
    """Section 3.2: Y~ = L2 L1^{-1} as a sparse matrix. Row i solves y L1 = (row i of L2)
    by back substitution with a sparse right-hand side (oracle_core.c, orc_explicit_y); a
    final entry that is zero or below tauY in magnitude is dropped and not propagated
    (tauY = 0 keeps every nonzero: the exact Y~ up to rounding)."""
    k, n = L2.nrows, L1.nrows
    yptr = np.zeros(k + 1, dtype=np.int64)
    cap = max(16, 4 * L2.nnz)
    ycol = np.empty(cap, dtype=np.int32)
    yval = np.empty(cap)
    row = 0
    while row < k:
        done = _load().orc_explicit_y(row, k, n, _p(L2.rowptr), _p(L2.col), _p(L2.val), _p(L1.rowptr),
                                      _p(L1.col), _p(L1.val), float(tauY), cap, _p(yptr), _p(ycol), _p(yval))
        if done < 0:
            raise MemoryError("orc_explicit_y")
        row = int(done)
        if row < k:
            cap *= 2
            ycol = np.resize(ycol, cap)
            yval = np.resize(yval, cap)
    nnz = int(yptr[-1])
    return CSR(k, n, yptr, ycol[:nnz].copy(), yval[:nnz].copy())


# ----------------------------------------------------------------------------
# Section 5.1 and the problem statement (1.1)


def validate(m, n, rowptr, col, val, appended=False):
    """Check CSR input of A (m x n, m >= n; or, appended, m >= 1 rows of n columns to add)
    and strip explicit zeros."""
    rowptr = _c(rowptr, np.int64)
    col = _c(col, np.int64)
    val = _c(val, np.float64)
    if n < 1 or (m < 1 if appended else m < n):
        raise ValueError("need m >= n >= 1" if not appended else "need at least one row")
    if rowptr.shape != (m + 1,) or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("bad row pointer")
    nnz = int(rowptr[-1])
    if col.shape != (nnz,) or val.shape != (nnz,):
        raise ValueError("bad array lengths")
    if nnz and (col.min() < 0 or col.max() >= n):
        raise ValueError("column index out of range")
    if not np.all(np.isfinite(val)):
        raise ValueError("non-finite value")
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    if nnz > 1:
        same_row = rows[1:] == rows[:-1]
        if np.any(same_row & (col[1:] <= col[:-1])):
            raise ValueError("column indices must be sorted and unique within a row")
    keep = val != 0.0
    rows, col, val = rows[keep], col[keep], val[keep]
    newptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=newptr[1:])
    return newptr, col.astype(np.int32), val


def to_csc(m, n, rowptr, col, val):
    """Column-compressed copy with ascending row indices in each column."""
    a = sp.csr_matrix((val, col, rowptr), shape=(m, n)).tocsc()
    a.sort_indices()
    return a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data.astype(np.float64)


def prescale(n, colptr, rowind, val):
    """Section 5.1: every column of A scaled to unit 2-norm. Returns (scaled values, norms)."""
    sval = np.empty_like(val)
    nrm = np.empty(n)
    _load().orc_prescale(n, _p(colptr), _p(rowind), _p(val), _p(sval), _p(nrm))
    return sval, nrm


# ----------------------------------------------------------------------------
# Algorithms 4-6


def ilup(m, n, colptr, rowind, val, p=10, tau=1e-2, mu=0.1, small=1e-10):
    """Rectangular ILUP(p, tau) of the (prescaled) CSC matrix. See oracle_core.c."""
    colptr = _c(colptr, np.int64)
    rowind = _c(rowind, np.int32)
    val = _c(val, np.float64)
    pe = int(min(p, m))
    lcap = max(1, n * min(pe, m))
    ucap = n * (min(pe, n) + 1)
    perm = np.empty(m, dtype=np.int32)
    lptr = np.empty(n + 1, dtype=np.int64)
    lrow = np.empty(lcap, dtype=np.int32)
    lval = np.empty(lcap)
    uptr = np.empty(n + 1, dtype=np.int64)
    ustep = np.empty(ucap, dtype=np.int32)
    uval = np.empty(ucap)
    nmod = ctypes.c_int64(0)
    rc = _load().orc_ilup(m, n, _p(colptr), _p(rowind), _p(val), pe, float(tau), float(mu), float(small),
                          _p(perm), _p(lptr), _p(lrow), _p(lval), lcap, _p(uptr), _p(ustep), _p(uval), ucap,
                          ctypes.byref(nmod))
    if rc != 0:
        raise RuntimeError("orc_ilup failed with code %d" % rc)
    lnz, unz = int(lptr[-1]), int(uptr[-1])
    return dict(perm=perm, lptr=lptr, lrow=lrow[:lnz].copy(), lval=lval[:lnz].copy(), uptr=uptr,
                ustep=ustep[:unz].copy(), uval=uval[:unz].copy(), nmod=int(nmod.value))


def level_sets(level):
    """(level_ptr, level_rows): rows grouped by level, ascending inside a level."""
    level = np.asarray(level, dtype=np.int64)
    nlev = int(level.max()) + 1 if level.size else 0
    rows = np.argsort(level, kind="stable").astype(np.int32)
    ptr = np.zeros(nlev + 1, dtype=np.int32)
    np.cumsum(np.bincount(level, minlength=nlev), out=ptr[1:])
    return ptr, rows


def levels(T, forward):
    """Depth of each row of triangular CSR T in its dependency DAG."""
    lv = np.empty(T.nrows, dtype=np.int32)
    _load().orc_levels(T.nrows, _p(T.rowptr), _p(T.col), 1 if forward else 0, _p(lv))
    return lv


@dataclass
class Factors:
    m: int
    n: int
    perm: np.ndarray  # int32[m], perm[k] = original row at position k
    colnorm: np.ndarray  # float64[n], A_hat = P A diag(1/colnorm)
    A: CSR  # user's A (validated)
    Ahat: CSR  # rows in pivot order, prescaled columns
    AhatT: CSR
    L1: CSR  # n x n strictly lower (unit diagonal implicit), by position
    L1T: CSR
    L2: CSR  # (m-n) x n
    L2T: CSR
    U: CSR  # n x n strictly upper part of U~
    Udiag: np.ndarray
    UT: CSR
    nmod: int
    smode: str
    S_chol: np.ndarray = field(default=None)  # lower Cholesky factor of S~ (dense mode)
    R: "CSR" = None  # removed rows of A_hat that were in A1 (Section 3.4), or None
    W_chol: np.ndarray = field(default=None)  # lower Cholesky factor of I - R M^{-1} R^T
    cg_steps: int = 2  # CG steps on S~ (cg mode)
    cg_jacobi: bool = False  # the CG steps preconditioned by the diagonal of S~ (explicit Y~)
    S_diag: object = None  # diag(S~) = 1 + the squared row norms of Y~ (cg_jacobi)
    lev: dict = field(default_factory=dict)
    Y: "CSR" = None  # explicit Y~ = L2 L1^{-1} (Section 3.2), or None: applied implicitly
    YT: "CSR" = None
    ytau: float = 0.0  # drop tolerance of the explicit Y~
    cheb_b: float = 1.0  # Chebyshev M_b: upper end of the interval [1, b] (cheb mode)
    cheb_degree: int = 0  # its number of steps
    cheb_omega: float = 1.0  # scale of its input (cheb_scale)
    poly_degree: int = 0  # the requested degree (0: from poly_delta)
    poly_delta: float = 0.9

    @property
    def psize(self):
        """Stored entries used by Algorithm 3: nnz(L1) + nnz(L2) + nnz(U) (diagonal of U
        counted, unit diagonal of L1 not), plus the packed S~ factor in dense mode."""
        s = self.L1.nnz + self.L2.nnz + self.U.nnz + self.n
        if self.smode == "dense":
            k = self.m - self.n
            s += k * (k + 1) // 2
        return s


def extract(m, n, res):
    """Split L~ into L1 (rows at positions < n) and L2 (positions >= n) and build U by rows."""
    perm = res["perm"].astype(np.int64)
    pos = np.empty(m, dtype=np.int64)
    pos[perm] = np.arange(m)
    lcol = np.repeat(np.arange(n), np.diff(res["lptr"]))
    lposn = pos[res["lrow"]]
    in1 = lposn < n
    L1 = csr_from_scipy(sp.coo_matrix((res["lval"][in1], (lposn[in1], lcol[in1])), shape=(n, n)))
    L2 = csr_from_scipy(sp.coo_matrix((res["lval"][~in1], (lposn[~in1] - n, lcol[~in1])), shape=(m - n, n)))
    ucol = np.repeat(np.arange(n), np.diff(res["uptr"]))
    ustep = res["ustep"].astype(np.int64)
    isdiag = ustep == ucol
    Udiag = np.zeros(n)
    Udiag[ucol[isdiag]] = res["uval"][isdiag]
    U = csr_from_scipy(sp.coo_matrix((res["uval"][~isdiag], (ustep[~isdiag], ucol[~isdiag])), shape=(n, n)))
    return L1, L2, U, Udiag


def dense_S(L1, L2):
    """S~ = I + Y~ Y~^T with Y~^T = L1^{-T} L2^T (dense), and its Cholesky factor (Section 3.2)."""
    n = L1.nrows
    L1d = L1.dense() + np.eye(n)
    YT = sla.solve_triangular(L1d.T, L2.dense().T, lower=False, unit_diagonal=True)
    S = np.eye(L2.nrows) + YT.T @ YT
    return S, np.linalg.cholesky(S)


def factor(m, n, rowptr, col, val, p=10, tau=1e-2, mu=0.1, small=1e-10, colscale=True, smode="identity",
           cg_steps=2, ystore=False, ytau=0.0, poly_degree=0, poly_delta=0.9, cg_jacobi=False):
    """Setup: validate, prescale, ILUP, splitting, transposes, level sets, S~, with ystore
    the explicit Y~ (drop tolerance ytau), and in cheb mode the Chebyshev interval and
    degree (poly_degree = 0: chosen by cheb_plan from poly_delta); cg_jacobi (cg mode with
    the explicit Y~) preconditions the CG steps by diag(S~)."""
    rowptr, col, val = validate(m, n, rowptr, col, val)
    A = CSR(m, n, rowptr, col, val)
    colptr, rowind, cval = to_csc(m, n, rowptr, col, val)
    if colscale:
        sval, nrm = prescale(n, colptr, rowind, cval)
    else:
        sval, nrm = cval, np.ones(n)
    res = ilup(m, n, colptr, rowind, sval, p=p, tau=tau, mu=mu, small=small)
    perm = res["perm"]
    L1, L2, U, Udiag = extract(m, n, res)
    scaled = sp.csc_matrix((sval, rowind, colptr), shape=(m, n)).tocsr()
    Ahat = csr_from_scipy(scaled[perm.astype(np.int64), :])
    F = Factors(m=m, n=n, perm=perm, colnorm=nrm, A=A, Ahat=Ahat, AhatT=Ahat.transpose(), L1=L1,
                L1T=L1.transpose(), L2=L2, L2T=L2.transpose(), U=U, Udiag=Udiag, UT=U.transpose(),
                nmod=res["nmod"], smode=smode, cg_steps=cg_steps)
    F.lev = {
        "L1": level_sets(levels(F.L1, True)),
        "L1T": level_sets(levels(F.L1T, False)),
        "U": level_sets(levels(F.U, False)),
        "UT": level_sets(levels(F.UT, True)),
    }
    if smode == "dense":
        if ystore:
            raise ValueError("the explicit Y~ is used with S^ = I, CG or none")
        _, F.S_chol = dense_S(L1, L2)
    elif smode not in ("identity", "none", "cg", "cheb"):
        raise ValueError(smode)
    if ystore:
        F.ytau = float(ytau)
        F.Y = explicit_Y(L1, L2, F.ytau)
        F.YT = F.Y.transpose()
    F.poly_degree, F.poly_delta = int(poly_degree), float(poly_delta)
    if smode == "cheb" and m > n:
        _plan_chebyshev(F)
    if cg_jacobi:
        if smode != "cg" or not ystore:
            raise ValueError("Jacobi-preconditioned CG needs cg mode and the explicit Y~")
        F.cg_jacobi = True
        F.S_diag = S_diagonal(F.Y)
    return F


def S_diagonal(Y):
    """diag(S~) = 1 + (Y~ Y~^T)_ii = 1 + the sum of the squared entries of row i of Y~, each
    sum correctly rounded (math.fsum of the rounded squares)."""
    d = np.ones(Y.nrows)
    for i in range(Y.nrows):
        v = Y.val[Y.rowptr[i]:Y.rowptr[i + 1]]
        if v.size:
            d[i] = 1.0 + math.fsum(v * v)
    return d


def _plan_chebyshev(F):
    F.cheb_b, F.cheb_degree = cheb_plan(lambda_max_S(F), F.poly_delta, F.poly_degree)
    F.cheb_omega = cheb_scale(F.cheb_b, F.cheb_degree, F.poly_delta)


def factor_problem(prob, **kw):
    return factor(prob.m, prob.n, prob.rowptr, prob.col, prob.val, **kw)


def add_rows(F, rowptr, col, val, tau=1e-2):
    """Section 3.4, adding rows: the factorization of A is kept (L1, U, the pivot order of
    A1) and each new row a, prescaled with the setup's column norms (a_hat = a D), becomes
    a row of A2 at the end of the row order with the L2 row l that solves (U)^T l^T =
    a_hat^T by forward substitution; entries with |l_j| < tau (or zero) are dropped, as in
    the ILUP's dropping of L. Dense S~ is recomputed, the explicit Y~ too, and so is W after
    earlier removals.
    Returns new Factors."""
    import dataclasses

    count = len(rowptr) - 1
    rowptr, col, val = validate(count, F.n, rowptr, col, val, appended=True)
    n, m0 = F.n, F.m
    new = sp.csr_matrix((val, col, rowptr), shape=(count, n))
    A = csr_from_scipy(sp.vstack([F.A.scipy(), new]).tocsr())
    scaled = sp.csr_matrix((val / F.colnorm[col], col, rowptr), shape=(count, n))
    Ahat = csr_from_scipy(sp.vstack([F.Ahat.scipy(), scaled]).tocsr())
    rows, cols, vals = [], [], []
    for i in range(count):
        ahat = np.zeros(n)
        e0, e1 = int(rowptr[i]), int(rowptr[i + 1])
        ahat[col[e0:e1]] = val[e0:e1] / F.colnorm[col[e0:e1]]
        l = lower_solve(F.UT, ahat, F.Udiag)  # U^T l^T = a_hat^T
        keep = np.nonzero((l != 0.0) & (np.abs(l) >= tau))[0]
        rows.append(np.full(keep.size, F.L2.nrows + i))
        cols.append(keep)
        vals.append(l[keep])
    L2 = csr_from_scipy(sp.vstack([F.L2.scipy(), sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows) - F.L2.nrows, np.concatenate(cols))),
        shape=(count, n))]).tocsr())
    perm = np.concatenate([F.perm, np.arange(m0, m0 + count, dtype=F.perm.dtype)])
    G = dataclasses.replace(F, m=m0 + count, perm=perm, A=A, Ahat=Ahat, AhatT=Ahat.transpose(), L2=L2,
                            L2T=L2.transpose())
    if F.smode == "dense":
        _, G.S_chol = dense_S(F.L1, L2)
    if F.Y is not None:
        G.Y = explicit_Y(F.L1, L2, F.ytau)
        G.YT = G.Y.transpose()
    if F.smode == "cheb":
        _plan_chebyshev(G)  # S~ changed with the rows
    if F.cg_jacobi:
        G.S_diag = S_diagonal(G.Y)
    if F.R is not None:
        G.W_chol = _woodbury_chol(G)
    return G


# ----------------------------------------------------------------------------
# Algorithm 3 and Algorithm 1


def S_product(F, d):
    """S~ d = d + Y~ Y~^T d (Section 3.2): with the explicit Y~ two sparse products,
    otherwise Y~ = L2 L1^{-1} applied implicitly."""
    if F.Y is not None:
        return d + F.Y.matvec(F.YT.matvec(d))
    return d + F.L2.matvec(lower_solve(F.L1, upper_solve(F.L1T, F.L2T.matvec(d))))


def cg_S(F, u):
    """F.cg_steps steps of unpreconditioned conjugate gradients on S~ w = u from
    w = 0 (Section 3.2; Table 3(a) takes two); stops early on a zero residual. With
    F.cg_jacobi, preconditioned conjugate gradients with diag(S~) instead."""
    if F.cg_jacobi:
        return pcg_S(F, u)
    w = np.zeros_like(u)
    res = u.copy()
    p = u.copy()
    rr = dot(res, res)
    for i in range(F.cg_steps):
        if not rr > 0.0:
            break
        q = S_product(F, p)
        pq = dot(p, q)
        if not (pq > 0.0 and math.isfinite(pq)):
            break
        alpha = rr / pq
        w = w + alpha * p
        res = res - alpha * q
        if i + 1 < F.cg_steps:
            rr_new = dot(res, res)
            p = res + (rr_new / rr) * p
            rr = rr_new
    return w


def pcg_S(F, u):
    """F.cg_steps steps of conjugate gradients on S~ w = u preconditioned by D = diag(S~),
    from w = 0: z = D^{-1} res, alpha = (res, z) / (p, S~ p), w += alpha p, res -= alpha S~ p,
    z = D^{-1} res, beta = (res, z)_new / (res, z), p = z + beta p (the textbook method, as for
    cg_S); stops early on a zero (res, z)."""
    D = F.S_diag
    w = np.zeros_like(u)
    res = u.copy()
    z = res / D
    p = z.copy()
    rz = dot(res, z)
    for i in range(F.cg_steps):
        if not rz > 0.0:
            break
        q = S_product(F, p)
        pq = dot(p, q)
        if not (pq > 0.0 and math.isfinite(pq)):
            break
        alpha = rz / pq
        w = w + alpha * p
        res = res - alpha * q
        if i + 1 < F.cg_steps:
            z = res / D
            rz_new = dot(res, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
    return w


def lambda_max_S(F, steps=50):
    """Estimate of the largest eigenvalue of S~ = I + Y~ Y~^T: `steps` power iterations from
    the all-ones vector, v <- S~ v / ||S~ v||, returning the last Rayleigh quotient
    (v, S~ v) with ||v|| = 1 (a lower bound of lambda_max)."""
    k = F.m - F.n
    v = np.ones(k) / math.sqrt(k)
    lam = 1.0
    for _ in range(steps):
        w = S_product(F, v)
        lam = dot(v, w)
        nw = math.sqrt(dot(w, w))
        v = w / nw
    return lam


def cheb_plan(lam, delta, degree=0):
    """Interval and degree of the Chebyshev polynomial that stands for S~^{-1}.

    The spectrum of S~ lies in [1, lambda_max]; the iteration uses [1, b] with
    b = 1.05 lam. After K steps from w = 0 the residual is r_K(S~) u with
    r_K(t) = T_K((b + 1 - 2t) / (b - 1)) / T_K((b + 1) / (b - 1)), so |r_K| <= eps_K =
    1 / T_K((b + 1) / (b - 1)) on [1, b]. The Algorithm 2 operator with this M_b^{-1}
    has, on an eigenvector of Y~^T Y~ with eigenvalue t - 1, the factor
    1 + (t - 1) r_K(t) in place of the exact 1 (up to the congruence with L1 U), which
    is positive for every t in [1, b] when (b - 1) eps_K < 1, and for every t > b when
    K is even (T_K is then positive left of -1). The default degree is the smallest
    even K with (b - 1) eps_K <= delta (at most 512). Returns (b, K); K = 0 when
    S~ = I (lam <= 1), meaning w = u."""
    if not lam > 1.0:
        return 1.0, 0
    b = 1.05 * lam
    sigma = (b + 1.0) / (b - 1.0)
    if degree > 0:
        return b, int(degree)
    K = 2
    while K < 512 and (b - 1.0) / math.cosh(K * math.acosh(sigma)) > delta:
        K += 2
    return b, K


def cheb_scale(b, K, delta):
    """Scale omega of the Chebyshev M_b^{-1} = omega p_K(S~). When (b - 1) eps_K <= delta
    (cheb_plan's bound; always so for the default degree below 512) omega = 1. Otherwise (a
    degree fixed too low for the interval, or the cap of 512) the unscaled operator can be
    indefinite, and omega = 1 / (1 + eps_K): on [1, b] the factor of cheb_plan becomes
    1 - omega (t - 1) p_K(t) with (t - 1) p_K(t) = (t - 1)(1 - r_K(t)) / t < 1 + eps_K, so it
    stays above 1 / t > 0; right of b an even K keeps r_K > 0 and p_K(t) < 1 / t."""
    if K == 0 or not b > 1.0:
        return 1.0
    eps = 1.0 / math.cosh(K * math.acosh((b + 1.0) / (b - 1.0)))
    return 1.0 if (b - 1.0) * eps <= delta else 1.0 / (1.0 + eps)


def cheb_S(F, u):
    """M_b^{-1} u by the Chebyshev iteration on S~ w = u over [1, F.cheb_b] with F.cheb_degree
    steps from w = 0 (the classical three-term form: theta = (b + 1)/2, delta = (b - 1)/2,
    sigma = theta/delta, rho_0 = 1/sigma, d_0 = u/theta; each step w += d, r -= S~ d,
    rho' = 1/(2 sigma - rho), d = rho' rho d + (2 rho'/delta) r), started from omega u
    (cheb_scale; omega = 1 unless the degree is too low for the interval). A fixed polynomial
    in S~: linear in u and symmetric positive definite (cheb_plan, cheb_scale). Degree 0:
    w = u (S~ = I)."""
    K, b = F.cheb_degree, F.cheb_b
    if K == 0:
        return u.copy()
    theta, half = (b + 1.0) / 2.0, (b - 1.0) / 2.0
    sigma = theta / half
    rho = 1.0 / sigma
    w = np.zeros_like(u)
    r = F.cheb_omega * u
    d = r / theta
    for _ in range(K):
        w = w + d
        r = r - S_product(F, d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = (rho_new * rho) * d + (2.0 * rho_new / half) * r
        rho = rho_new
    return w


def Mb_solve(F, u):
    """Step 3 of Algorithm 2 / step 2 of Algorithm 3 with S^ = CG or Chebyshev on S~, or I."""
    if F.smode == "cg":
        return cg_S(F, u)
    if F.smode == "cheb":
        return cheb_S(F, u)
    return u


def apply_alg3(F, r):
    """Algorithm 3 on the residual r (pivot order): h from (r1, r2).

    u = r2 - Y~ r1 with Y~ r1 = L2 (L1^{-1} r1); solve S^ w = u (S^ = I or the
    dense S~); y = r1 + Y~^T w with Y~^T w = L1^{-T} (L2^T w); L1 v = y; U h = v.
    """
    n = F.n
    r1, r2 = r[:n], r[n:]
    if F.smode == "none" or F.m == n:
        # no correction (w = 0): y = r1
        return upper_solve(F.U, lower_solve(F.L1, r1), F.Udiag)
    if F.Y is not None:
        # explicit Y~ (Section 3.2): u = r2 - Y~ r1, S^ w = u, y = r1 + Y~^T w
        u = r2 - F.Y.matvec(r1)
        w = Mb_solve(F, u)
        y = r1 + F.YT.matvec(w)
        return upper_solve(F.U, lower_solve(F.L1, y), F.Udiag)
    t = lower_solve(F.L1, r1)
    u = r2 - F.L2.matvec(t)
    if F.smode == "dense":
        w = sla.cho_solve((F.S_chol, True), u)
    else:
        w = Mb_solve(F, u)
    g = F.L2T.matvec(w)
    y = r1 + upper_solve(F.L1T, g)
    v = lower_solve(F.L1, y)
    return upper_solve(F.U, v, F.Udiag)


def _ma_solve(F, v):
    """M_a^{-1} v for M_a = (L1 U)^T (L1 U): U^T s = v, L1^T t = s, L1 w = t, U h = w."""
    s = lower_solve(F.UT, v, F.Udiag)
    t = upper_solve(F.L1T, s)
    w = lower_solve(F.L1, t)
    return upper_solve(F.U, w, F.Udiag)


def apply_alg2(F, z):
    """Algorithm 2 with k = n on z = A_hat^T r (pivot-order coordinates).

    Step 1 solves M_a u_a = z; step 2 forms w_b = A2 u_a; step 3 solves
    M_b v_b = w_b; step 4 forms w_a = z - A2^T v_b (the paper's printed
    "u_a - A2^T v_b" contradicts (3.1)-(3.3); z is what the Woodbury form
    needs); step 5 solves M_a h = w_a. Here M_a = (L1 U)^T (L1 U), A2 is
    represented by L2 U (its image under the incomplete factorization, so
    that A2 M_a^{-1} A2^T = Y~ Y~^T), and M_b is S~ (dense mode), I
    (identity mode) or absent (none mode: v_b = 0, h = u_a). With the explicit Y~
    (F.Y), A2 = L2 U = Y~ L1 U is applied through Y~ and S~ products are Y~ Y~^T
    products.
    """
    if F.R is not None:
        return _apply_removed(F, z)
    ua = _ma_solve(F, z)
    if F.smode == "none" or F.m == F.n:
        return ua
    Uua = F.U.matvec(ua) + F.Udiag * ua
    if F.Y is not None:
        # explicit Y~: A2 = L2 U = Y~ L1 U, so w_b = Y~ (L1 U u_a) and A2^T v_b = U^T L1^T Y~^T v_b
        wb = F.Y.matvec(F.L1.matvec(Uua) + Uua)
        vb = Mb_solve(F, wb)
        g = F.YT.matvec(vb)
        g = F.L1T.matvec(g) + g
        wa = z - (F.UT.matvec(g) + F.Udiag * g)
        return _ma_solve(F, wa)
    wb = F.L2.matvec(Uua)
    if F.smode == "dense":
        vb = sla.cho_solve((F.S_chol, True), wb)
    else:
        vb = Mb_solve(F, wb)
    s = F.L2T.matvec(vb)
    wa = z - (F.UT.matvec(s) + F.Udiag * s)
    return _ma_solve(F, wa)


def _woodbury_chol(G):
    """Cholesky factor of W = I - R M^{-1} R^T with the kept operator M^{-1} of G."""
    import dataclasses

    base = dataclasses.replace(G, R=None, W_chol=None)
    Rd = G.R.dense()
    MRt = np.column_stack([apply_alg2(base, Rd[i]) for i in range(G.R.nrows)])
    W = np.eye(G.R.nrows) - Rd @ MRt
    return np.linalg.cholesky(0.5 * (W + W.T))


def _apply_removed(F, z):
    """Section 3.4, removing rows R (Woodbury): C1^{-1} = C^{-1} + C^{-1} R^T (I - R C^{-1} R^T)^{-1}
    R C^{-1}, with C^{-1} the Algorithm 2 operator of the kept factorization."""
    import dataclasses

    base = dataclasses.replace(F, R=None, W_chol=None)
    g = apply_alg2(base, z)
    w = sla.cho_solve((F.W_chol, True), F.R.matvec(g))
    return g + apply_alg2(base, F.R.transpose().matvec(w))


def remove_rows(F, rows):
    """Section 3.4, removing rows (original row indices, unique). The factorization is kept.
    Removed rows of A2 leave L2 (S~ is refactored); removed rows of A1 (now absent from A_hat)
    enter R, and the preconditioner becomes the Woodbury update of the Algorithm 2 operator
    M^{-1} for C1 = C - R^T R: M^{-1} + M^{-1} R^T W^{-1} R M^{-1}, W = I - R M^{-1} R^T (with
    the refactored S~ and every A1 row removed so far in R). Requires the dense S~ (the only
    mode in which M approximates A^T A and not only its A1 part). The remaining rows are
    renumbered in their order. Returns new Factors."""
    import dataclasses

    if F.smode != "dense":
        raise ValueError("removing rows needs the dense S~")
    rows = np.asarray(rows, dtype=np.int64)
    if rows.size == 0 or np.unique(rows).size != rows.size or rows.min() < 0 or rows.max() >= F.m:
        raise ValueError("bad row list")
    if F.m - rows.size < F.n:
        raise ValueError("fewer rows than columns would remain")
    m, n = F.m, F.n
    perm = F.perm.astype(np.int64)
    pos = np.empty(m, dtype=np.int64)
    pos[perm] = np.arange(m)
    gone = np.zeros(m, dtype=bool)
    gone[pos[rows]] = True  # by position
    a1 = np.nonzero(gone[:n])[0]
    keep2 = ~gone[n:]
    Ahs = F.Ahat.scipy()
    Rnew = csr_from_scipy(Ahs[a1])
    R = Rnew if F.R is None else csr_from_scipy(sp.vstack([F.R.scipy(), Rnew.scipy()]).tocsr())
    L2 = csr_from_scipy(F.L2.scipy()[np.nonzero(keep2)[0]])
    renum = np.cumsum(~np.isin(np.arange(m), rows)) - 1  # new index of a kept original row
    keep_pos = np.nonzero(~gone)[0]
    kept_rows = np.setdiff1d(np.arange(m), rows)
    G = dataclasses.replace(F, m=m - rows.size, perm=renum[perm[keep_pos]].astype(F.perm.dtype),
                            A=csr_from_scipy(F.A.scipy()[kept_rows]), Ahat=csr_from_scipy(Ahs[keep_pos]),
                            L2=L2, L2T=L2.transpose(), R=None, W_chol=None)
    G.AhatT = G.Ahat.transpose()
    if G.m > n:
        _, G.S_chol = dense_S(G.L1, G.L2)
    else:
        G.S_chol = None
    if R.nrows:
        G.R = R
        G.W_chol = _woodbury_chol(G)
    return G


def lsqr_m(F, b, tol=1e-8, maxit=2000, trace=False):
    """LSQR on min || P b - A_hat N y ||, x_hat = N y, with N N^T = M^{-1} the SPD operator
    of Algorithm 2 (apply_alg2; modes "none", "dense" and "cheb"), in the M-inner-product form:
    v = N v_hat, M v = N^{-T} v_hat, so only M^{-1} is ever applied.

    Init: beta1 = ||P b||, u = P b / beta1, s = A_hat^T u, v' = M^{-1} s,
    alpha = sqrt(s . v'), v = v'/alpha, Mv = s/alpha, w = v, phibar = beta1,
    rhobar = alpha. Step: t = A_hat v - alpha u, beta = ||t||, u = t/beta;
    s = A_hat^T u - beta Mv, v' = M^{-1} s, alpha = sqrt(s . v'), v = v'/alpha,
    Mv = s/alpha; rho = sqrt(rhobar^2 + beta^2), c = rhobar/rho, sn = beta/rho,
    theta = sn alpha, rhobar = -c alpha, phi = c phibar, phibar = sn phibar;
    x_hat += (phi/rho) w, w = v - (theta/rho) w.
    Since A_hat^T r = phibar c s (up to sign) after a step, the stop test is
    |phibar c| ||D^{-1} s|| <= tol ||A^T b|| with ||A^T b|| = beta1 ||D^{-1} s_1||.
    Breakdown: s . v' <= 0 or a non-finite scalar.
    """
    if F.smode not in ("none", "dense", "cheb") and F.m > F.n:
        raise ValueError("LSQR needs a symmetric positive definite M^{-1}")
    b = _c(b, np.float64)
    n = F.n
    r = b[F.perm.astype(np.int64)].copy()
    xh = np.zeros(n)
    beta1 = math.sqrt(dot(r, r))
    status = "not_converged"
    iters = 0
    hist = []
    if beta1 == 0.0:
        status = "ok"
    else:
        u = r / beta1
        s = F.AhatT.matvec(u)
        s1 = math.sqrt(dot(F.colnorm * s, F.colnorm * s))
        nb = beta1 * s1
        hist.append(nb)
        vp = apply_alg2(F, s)
        sv = dot(s, vp)
        if not (sv > 0.0 and math.isfinite(sv)):
            status = "breakdown" if nb > 0.0 else "ok"
        else:
            alpha = math.sqrt(sv)
            v = vp / alpha
            Mv = s / alpha
            w = v.copy()
            phibar, rhobar = beta1, alpha
            for it in range(1, maxit + 1):
                t = F.Ahat.matvec(v) - alpha * u
                beta = math.sqrt(dot(t, t))
                if not math.isfinite(beta):
                    status = "breakdown"
                    break
                u = t / beta if beta > 0.0 else t
                s = F.AhatT.matvec(u) - beta * Mv
                sn_ = math.sqrt(dot(F.colnorm * s, F.colnorm * s))
                vp = apply_alg2(F, s)
                sv = dot(s, vp)
                alpha = math.sqrt(sv) if sv > 0.0 else 0.0
                rho = math.sqrt(rhobar * rhobar + beta * beta)
                c, sn = rhobar / rho, beta / rho
                theta = sn * alpha
                rhobar = -c * alpha
                phi = c * phibar
                phibar = sn * phibar
                xh = xh + (phi / rho) * w
                iters = it
                est = abs(phibar * c) * sn_
                hist.append(est)
                if alpha > 0.0:
                    v = vp / alpha
                    Mv = s / alpha
                    w = v - (theta / rho) * w
                if est <= tol * nb:
                    status = "ok"
                    break
                if alpha == 0.0 or not math.isfinite(sv):
                    status = "breakdown" if sv < 0.0 or not math.isfinite(sv) else "ok"
                    break
    x = xh / F.colnorm
    atr, rel = true_residual(F.A, b, x)
    return SolveResult(x=x, iters=iters, status=status, atr_norm=atr, atr_rel=rel, hist=hist)


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    status: str  # "ok", "not_converged", "breakdown"
    atr_norm: float  # true ||A^T (b - A x)||
    atr_rel: float  # atr_norm / ||A^T b||
    hist: list = field(default_factory=list)  # recurrence ||A^T r|| per iteration
    rnorm: list = field(default_factory=list)  # ||r|| per iteration (with trace=True)
    orth: list = field(default_factory=list)  # (p_prev, z_new)/(p_prev, z_old) (with trace=True)


def true_residual(A, b, x):
    """||A^T (b - A x)|| and its ratio to ||A^T b|| on the user's A."""
    r = b - A.matvec(x)
    AT = A.transpose()
    atr = float(np.linalg.norm(AT.matvec(r)))
    atb = float(np.linalg.norm(AT.matvec(np.asarray(b, dtype=np.float64))))
    return atr, (atr / atb if atb > 0 else 0.0)


def pcgls(F, b, tol=1e-8, maxit=2000, apply=None, trace=False, form="alg3"):
    """Algorithm 1 on A_hat x_hat ~ P b with h = B(r) from Algorithm 3
    (form "alg3"), or h = M^{-1} z from Algorithm 2 (form "alg2").

    Initialisation: x0 = 0, r0 = P b, z0 = A_hat^T r0, h0 = B(r0),
    rho0 = (z0, h0), p0 = h0. Iteration i: q = A_hat p, alpha = rho/(q,q),
    x += alpha p, r -= alpha q, z = A_hat^T r; stop when ||D^{-1} z|| <=
    tol ||D^{-1} z0|| (this is ||A^T r|| <= tol ||A^T b|| on the user's A);
    else h = B(r), rho' = (z,h), beta = rho'/rho, p = h + beta p.
    Breakdown: (q,q) = 0, rho' = 0 or a non-finite scalar.
    """
    if apply is None:
        if form == "alg2":
            def apply(F_, r_, z_):
                return apply_alg2(F_, z_)
        elif form == "alg3":
            def apply(F_, r_, z_):
                return apply_alg3(F_, r_)
        else:
            raise ValueError(form)
    b = _c(b, np.float64)
    n = F.n
    r = b[F.perm.astype(np.int64)].copy()
    xh = np.zeros(n)
    z = F.AhatT.matvec(r)
    nb = math.sqrt(dot(F.colnorm * z, F.colnorm * z))
    hist = [nb]
    rn, orth = [float(np.linalg.norm(r))], []
    status = "not_converged"
    iters = 0
    if nb == 0.0:
        status = "ok"
    else:
        h = apply(F, r, z)
        rho = dot(z, h)
        p = h.copy()
        if rho == 0.0 or not math.isfinite(rho):
            status = "breakdown"
        else:
            for it in range(1, maxit + 1):
                q = F.Ahat.matvec(p)
                delta = dot(q, q)
                if delta == 0.0 or not math.isfinite(delta):
                    status = "breakdown"
                    break
                alpha = rho / delta
                xh += alpha * p
                r -= alpha * q
                z = F.AhatT.matvec(r)
                zn = math.sqrt(dot(F.colnorm * z, F.colnorm * z))
                hist.append(zn)
                if trace:
                    rn.append(float(np.linalg.norm(r)))
                    orth.append(dot(p, z) / rho)
                iters = it
                if zn <= tol * nb:
                    status = "ok"
                    break
                if it == maxit:
                    break
                h = apply(F, r, z)
                rho_new = dot(z, h)
                if rho_new == 0.0 or not math.isfinite(rho_new):
                    status = "breakdown"
                    break
                beta = rho_new / rho
                rho = rho_new
                p = h + beta * p
    x = xh / F.colnorm
    atr, rel = true_residual(F.A, b, x)
    return SolveResult(x=x, iters=iters, status=status, atr_norm=atr, atr_rel=rel, hist=hist, rnorm=rn, orth=orth)
