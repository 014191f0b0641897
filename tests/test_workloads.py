"""The seeded generators: shapes, structure and determinism of the synthetic inputs."""

import numpy as np
import pytest

import gen


def _check_csr(p):
    assert p.rowptr.dtype == np.int64 and p.col.dtype == np.int32 and p.val.dtype == np.float64
    assert p.rowptr[0] == 0 and p.rowptr[-1] == p.col.size == p.val.size
    assert np.all(np.diff(p.rowptr) >= 0)
    rows = np.repeat(np.arange(p.m), np.diff(p.rowptr))
    same = rows[1:] == rows[:-1]
    assert np.all(p.col[1:][same] > p.col[:-1][same])
    assert p.col.min() >= 0 and p.col.max() < p.n
    assert np.all(p.val != 0) and np.all(np.isfinite(p.val))
    # structural full column rank: every column is hit
    assert np.unique(p.col).size == p.n


def test_tiny_shape_and_determinism():
    a, b = gen.tiny_c1(), gen.tiny_c1()
    _check_csr(a)
    assert (a.m, a.n, a.nnz) == (2000, 1000, 10000)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val) and np.array_equal(a.b, b.b)
    assert np.diff(a.rowptr).max() == 5


def test_grid_small():
    p = gen.by_name("c2-small")
    _check_csr(p)
    lens = np.diff(p.rowptr)
    assert lens.min() >= 2 and lens.max() <= 7
    scales = np.abs(p.val)
    assert scales.max() / scales.min() > 1e4  # column scaling spreads magnitudes


def test_sparse_dense_mini():
    p = gen.by_name("c3-mini")
    _check_csr(p)
    lens = np.sort(np.diff(p.rowptr))
    assert np.all(lens[-8:] == 600) and np.all(lens[:-8] == 6)


@pytest.mark.slow
def test_full_sizes():
    p = gen.grid_c2()
    assert (p.m, p.n) == (600_000, 400_000) and 2_600_000 < p.nnz < 2_800_000
    p = gen.sparse_dense_c3()
    assert (p.m, p.n, p.nnz) == (450_064, 400_000, 450_000 * 6 + 64 * 120_000)


@pytest.mark.parametrize("key", list(gen.PAPER_SHAPES))
def test_paper_shapes(key):
    p = gen.paper_shape(key, scale=0.2)
    _check_csr(p)
    assert p.m > p.n
    assert np.all(np.abs(p.b) <= 1.0)
