"""Seeded synthetic sparse least-squares problems min ||b - A x||, A m x n, m > n.

The paper measures on matrices from the SuiteSparse collection and the CUTEst
LP set (Section 5.1, Table 1). Those are not available here; the generators
below stand in for them with matrices of the same shapes and structure
(quasi-square, tall, sparse-dense). Every generator is a pure function of its
arguments and seed (numpy ``default_rng``), returns CSR with sorted, unique
column indices per row and no explicit zeros, and guarantees structural full
column rank through a transversal (row i holds column i before the rows are
shuffled).

Nothing here implements any step of the method.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    m: int
    n: int
    rowptr: np.ndarray  # int64[m+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    b: np.ndarray  # float64[m]
    x_true: np.ndarray = field(default=None)  # float64[n] or None

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.rowptr))
        a[rows, self.col] = self.val
        return a

    def scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.m, self.n))


# ----------------------------------------------------------------------------
# assembly helpers (structure only)


def _csr_from_rows(m, n, row_of, col_of, val_of):
    """CSR from COO triplets; rows sorted, columns sorted within a row."""
    row_of = np.asarray(row_of, dtype=np.int64)
    col_of = np.asarray(col_of, dtype=np.int64)
    val_of = np.asarray(val_of, dtype=np.float64)
    keep = val_of != 0.0
    row_of, col_of, val_of = row_of[keep], col_of[keep], val_of[keep]
    order = np.lexsort((col_of, row_of))
    row_of, col_of, val_of = row_of[order], col_of[order], val_of[order]
    if len(row_of) > 1:
        dup = (row_of[1:] == row_of[:-1]) & (col_of[1:] == col_of[:-1])
        if dup.any():
            raise ValueError("generator produced a duplicated (row, col)")
    counts = np.bincount(row_of, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    assert col_of.size == 0 or (col_of.min() >= 0 and col_of.max() < n)
    return rowptr, col_of.astype(np.int32), val_of


def _shuffle_rows(rng, m, rowptr, col, val):
    perm = rng.permutation(m)
    counts = np.diff(rowptr)[perm]
    new_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=new_ptr[1:])
    starts = rowptr[perm]
    idx = np.repeat(starts - new_ptr[:-1], counts) + np.arange(new_ptr[-1])
    return new_ptr, col[idx], val[idx]


def _distinct_cols(rng, nrows, ncols, k, exclude=None):
    """(nrows, k) distinct column indices per row, none equal to exclude[row]."""
    if k == 0:
        return np.zeros((nrows, 0), dtype=np.int64)
    if k + (exclude is not None) > ncols:
        raise ValueError("more distinct columns requested than exist")
    if 4 * (k + 1) > ncols:  # dense-ish rows: draw a permutation per row
        out = np.empty((nrows, k), dtype=np.int64)
        for r in range(nrows):
            pool = np.arange(ncols)
            if exclude is not None:
                pool = pool[pool != exclude[r]]
            out[r] = rng.choice(pool, size=k, replace=False)
        return out
    out = rng.integers(0, ncols, size=(nrows, k))

    def bad_rows(a, ex):
        s = np.sort(a, axis=1)
        bad = (s[:, 1:] == s[:, :-1]).any(axis=1)
        if ex is not None:
            bad |= (a == ex[:, None]).any(axis=1)
        return bad

    bad = bad_rows(out, exclude)
    while bad.any():
        idx = np.nonzero(bad)[0]
        out[idx] = rng.integers(0, ncols, size=(idx.size, k))
        sub = bad_rows(out[idx], None if exclude is None else exclude[idx])
        bad = np.zeros(nrows, dtype=bool)
        bad[idx[sub]] = True
    return out


def _finish(name, rng, m, n, rows, cols, vals, rhs="model", shuffle=True):
    rowptr, col, val = _csr_from_rows(m, n, rows, cols, vals)
    if shuffle:
        rowptr, col, val = _shuffle_rows(rng, m, rowptr, col, val)
    x_true = rng.standard_normal(n)
    if rhs == "model":
        # b = A x_true + 1e-3 * N(0, 1)
        r_of = np.repeat(np.arange(m), np.diff(rowptr))
        ax = np.zeros(m)
        np.add.at(ax, r_of, val * x_true[col])
        b = ax + 1e-3 * rng.standard_normal(m)
    elif rhs == "uniform":
        # entries of b uniform in [-1, 1] (Section 5.1)
        b = rng.uniform(-1.0, 1.0, size=m)
        x_true = None
    else:
        raise ValueError(rhs)
    return Problem(name, m, n, rowptr, col, val, b, x_true)


# ----------------------------------------------------------------------------
# the three FP64 workloads


def tiny_c1(m=2000, n=1000, seed=1):
    """Quasi-square tiny case: A = row-shuffle([B; R]).

    B (n x n): diagonal g + 4 sign(g), g ~ N(0,1), and 4 distinct random
    off-diagonal columns per row with N(0,1) values. R ((m-n) x n): 5 distinct
    random columns per row with N(0,1) values. b = A x_true + 1e-3 N(0,1).
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n)
    diag = g + 4.0 * np.sign(g)
    off = _distinct_cols(rng, n, n, 4, exclude=np.arange(n))
    offv = rng.standard_normal((n, 4))
    rr = _distinct_cols(rng, m - n, n, 5)
    rv = rng.standard_normal((m - n, 5))
    rows = np.concatenate([np.arange(n), np.repeat(np.arange(n), 4), n + np.repeat(np.arange(m - n), 5)])
    cols = np.concatenate([np.arange(n), off.ravel(), rr.ravel()])
    vals = np.concatenate([diag, offv.ravel(), rv.ravel()])
    return _finish(f"tiny m={m} n={n}", rng, m, n, rows, cols, vals)


def grid_c2(n=400_000, m=600_000, gw=633, seed=2):
    """Grid-like tall case (633 x 633 grid of columns for n = 400,000).

    Column c is grid cell (c // gw, c % gw); cells >= n are unused. Row i < n is
    centred on column i (the transversal); the other m - n rows are centred
    uniformly. A row holds k ~ U{2..7} entries: its centre and k - 1 distinct
    neighbours drawn from the 7-point set {+-1, +-gw, +(gw+1), -(gw+1)} that lie
    in the grid (fewer if the cell has fewer). Values N(0,1); each column is then
    scaled by 10^U(-3,3) so that A^T A is ill-conditioned.
    """
    rng = np.random.default_rng(seed)
    centre = np.concatenate([np.arange(n), rng.integers(0, n, size=m - n)])
    k = rng.integers(2, 8, size=m)
    gx, gy = np.divmod(centre, gw)
    dx = np.array([0, 0, 1, -1, 1, -1])
    dy = np.array([1, -1, 0, 0, 1, -1])
    nx = gx[:, None] + dx[None, :]
    ny = gy[:, None] + dy[None, :]
    nb = nx * gw + ny
    valid = (nx >= 0) & (nx < gw) & (ny >= 0) & (ny < gw) & (nb < n)
    keys = rng.random((m, 6))
    keys[~valid] = 2.0
    order = np.argsort(keys, axis=1)
    nb_sorted = np.take_along_axis(nb, order, axis=1)
    valid_sorted = np.take_along_axis(valid, order, axis=1)
    take = (np.arange(6)[None, :] < (k - 1)[:, None]) & valid_sorted
    rows = np.concatenate([np.arange(m), np.repeat(np.arange(m), 6)[take.ravel()]])
    cols = np.concatenate([centre, nb_sorted.ravel()[take.ravel()]])
    vals = rng.standard_normal(rows.size)
    scale = 10.0 ** rng.uniform(-3.0, 3.0, size=n)
    vals = vals * scale[cols]
    return _finish(f"grid m={m} n={n}", rng, m, n, rows, cols, vals)


def sparse_dense_c3(n=400_000, m_sparse=450_000, n_dense=64, dense_frac=0.3, k=6, seed=3):
    """Sparse-dense case: m_sparse sparse rows plus n_dense dense rows.

    Sparse rows hold k distinct random columns (row i < n includes column i);
    dense rows hold exactly round(dense_frac * n) distinct random columns.
    Values N(0,1).
    """
    rng = np.random.default_rng(seed)
    first = _distinct_cols(rng, n, n, k - 1, exclude=np.arange(n))
    rest = _distinct_cols(rng, m_sparse - n, n, k)
    nd = int(round(dense_frac * n))
    dense_cols = [np.sort(rng.choice(n, size=nd, replace=False)) for _ in range(n_dense)]
    rows = np.concatenate(
        [
            np.arange(n),
            np.repeat(np.arange(n), k - 1),
            n + np.repeat(np.arange(m_sparse - n), k),
            m_sparse + np.repeat(np.arange(n_dense), nd),
        ]
    )
    cols = np.concatenate([np.arange(n), first.ravel(), rest.ravel()] + dense_cols)
    vals = rng.standard_normal(rows.size)
    m = m_sparse + n_dense
    return _finish(f"sparse-dense m={m} n={n}", rng, m, n, rows, cols, vals)


# ----------------------------------------------------------------------------
# served requests (a stream of independent problems of uneven size)


def served_request(n, m, seed, n_dense=0, dense_frac=0.3):
    """One request of the served stream: the tiny-case recipe at size m x n with
    4-8 entries per row (B: diagonal g + 4 sign(g) and 3-7 off-diagonals; R:
    4-8 random columns), plus n_dense rows holding round(dense_frac * n)
    random columns. Values N(0,1); b = A x_true + 1e-3 N(0,1).
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n)
    diag = g + 4.0 * np.sign(g)
    kb = rng.integers(3, 8, size=n)  # off-diagonals of B rows
    off = _distinct_cols(rng, n, n, 7, exclude=np.arange(n))
    take_b = np.arange(7)[None, :] < kb[:, None]
    nr = m - n - n_dense
    kr = rng.integers(4, 9, size=nr)
    rr = _distinct_cols(rng, nr, n, 8)
    take_r = np.arange(8)[None, :] < kr[:, None]
    nd = int(round(dense_frac * n))
    dense_cols = [np.sort(rng.choice(n, size=nd, replace=False)) for _ in range(n_dense)]
    rows = np.concatenate([np.arange(n), np.repeat(np.arange(n), 7)[take_b.ravel()],
                           n + np.repeat(np.arange(nr), 8)[take_r.ravel()]] +
                          [np.full(nd, n + nr + d) for d in range(n_dense)])
    cols = np.concatenate([np.arange(n), off.ravel()[take_b.ravel()], rr.ravel()[take_r.ravel()]] + dense_cols)
    vals = np.concatenate([diag, rng.standard_normal(rows.size - n)])
    return _finish(f"served m={m} n={n} dense={n_dense}", rng, m, n, rows, cols, vals)


def served_stream(count=512, seed=5, n_lo=2000, n_hi=200_000, dense_share=0.1):
    """Sizes of the served stream: n log-uniform in [n_lo, n_hi], m = round(n U(1.1, 2.0)),
    a share of requests with U{8..32} dense rows. Returns (n, m, seed, n_dense) tuples."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        m = int(round(n * rng.uniform(1.1, 2.0)))
        nd = int(rng.integers(8, 33)) if rng.random() < dense_share else 0
        out.append((n, m, seed * 100003 + i, nd))
    return out


# ----------------------------------------------------------------------------
# small generic cases for tests


def random_sparse(m, n, k=4, seed=0, n_dense=0, dense_len=None, transversal=True, rhs="model", shuffle=True):
    """Random sparse m x n: k distinct columns per row (row i < n includes i).

    n_dense extra rows hold dense_len distinct random columns each.
    """
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    if transversal:
        rows.append(np.arange(n))
        cols.append(np.arange(n))
        if k > 1:
            oth = _distinct_cols(rng, n, n, min(k - 1, n - 1), exclude=np.arange(n))
            rows.append(np.repeat(np.arange(n), oth.shape[1]))
            cols.append(oth.ravel())
        first_free = n
    else:
        first_free = 0
    nr = m - first_free - n_dense
    if nr > 0:
        kk = min(k, n)
        oth = _distinct_cols(rng, nr, n, kk)
        rows.append(first_free + np.repeat(np.arange(nr), kk))
        cols.append(oth.ravel())
    if n_dense:
        dl = dense_len or max(1, n // 3)
        for d in range(n_dense):
            rows.append(np.full(dl, m - n_dense + d))
            cols.append(np.sort(rng.choice(n, size=dl, replace=False)))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.standard_normal(rows.size)
    return _finish(f"random m={m} n={n} k={k}", rng, m, n, rows, cols, vals, rhs=rhs, shuffle=shuffle)


# Shapes of test problems of Table 1: (paper problem number, m, n, nz, lmax)
PAPER_SHAPES = {
    "quasi-square": (1, 17516, 17443, 68779, 46),
    "dense-ish": (3, 2511, 2456, 171214, 829),
    "mid": (10, 14318, 11028, 57376, 18),
    "tall": (24, 25067, 1118, 144812, 6),
    "heavy-dense-rows": (22, 15904, 3159, 2872265, 2500),
}


def paper_shape(key, seed=0, scale=1.0):
    """Random matrix with the m, n, nz and longest row of a Table 1 problem.

    Most rows get the average length; a few rows of length between lmax/2 and
    lmax carry the rest when the problem has long rows. b ~ U[-1, 1] as in
    Section 5.1. ``scale`` < 1 shrinks m, n and nz proportionally.
    """
    _, m, n, nz, lmax = PAPER_SHAPES[key]
    m = max(int(round(m * scale)), 4)
    n = max(int(round(n * scale)), 3)
    if m <= n:
        m = n + 1
    nz = int(round(nz * scale))
    lmax = max(2, min(lmax, n))
    rng = np.random.default_rng(seed)
    avg = nz / m
    if lmax > 3 * max(avg, 1):
        n_long = max(1, int(0.5 * nz / (0.75 * lmax)) if avg > 20 else max(1, m // 2000))
        n_long = min(n_long, m - n, max(1, m // 4))
    else:
        n_long = 0
    long_len = rng.integers(max(2, lmax // 2), lmax + 1, size=n_long)
    short_nz = max(nz - int(long_len.sum()), m)
    k_short = max(1, min(int(round(short_nz / (m - n_long))), max(1, lmax - 1), n))
    rows, cols = [np.arange(n)], [np.arange(n)]
    if k_short > 1:
        oth = _distinct_cols(rng, n, n, min(k_short - 1, n - 1), exclude=np.arange(n))
        rows.append(np.repeat(np.arange(n), oth.shape[1]))
        cols.append(oth.ravel())
    nr = m - n - n_long
    if nr > 0:
        oth = _distinct_cols(rng, nr, n, min(k_short, n))
        rows.append(n + np.repeat(np.arange(nr), oth.shape[1]))
        cols.append(oth.ravel())
    for d in range(n_long):
        rows.append(np.full(long_len[d], m - n_long + d))
        cols.append(np.sort(rng.choice(n, size=long_len[d], replace=False)))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.standard_normal(rows.size)
    return _finish(f"paper-shape {key} m={m} n={n}", rng, m, n, rows, cols, vals, rhs="uniform")


def by_name(name):
    """Named workloads used by the bench and the tests."""
    if name == "c1":
        return tiny_c1()
    if name == "c2":
        return grid_c2()
    if name.startswith("c2-seed"):
        # the same recipe and size with another seed (a second draw of the workload)
        return grid_c2(seed=int(name[len("c2-seed"):]))
    if name == "c3":
        return sparse_dense_c3()
    if name == "c4":
        return grid_c2(n=1_000_000, m=1_500_000, gw=1000, seed=4)
    if name == "c2-small":
        return grid_c2(n=20_000, m=30_000, gw=142, seed=12)
    if name == "c3-40k":
        # the sparse-dense recipe at the largest size whose host setup stays near a minute
        # (the elimination's reach grows with the column index on this recipe)
        return sparse_dense_c3(n=40_000, m_sparse=45_000, n_dense=64, dense_frac=0.3, k=6, seed=3)
    if name == "c3-mini":
        return sparse_dense_c3(n=2000, m_sparse=2250, n_dense=8, dense_frac=0.3, k=6, seed=13)
    raise KeyError(name)
