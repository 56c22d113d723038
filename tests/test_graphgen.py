"""The threaded R-MAT builder gives exactly the numpy generator's graph."""
import numpy as np
import pytest

import graphgen as gg


@pytest.fixture(scope="module", autouse=True)
def native():
    gg.build_native(force=False)


@pytest.mark.parametrize("scale,ef,seed", [(3, 3, 9), (10, 16, 2), (12, 8, 5), (15, 16, 1011)])
def test_native_rmat_equals_numpy(scale, ef, seed):
    a = gg.rmat_numpy(scale, ef, seed)
    b = gg.rmat_native(scale, ef, seed, threads=3)
    assert a.n == b.n
    assert np.array_equal(a.row_ptr, b.row_ptr)
    assert np.array_equal(a.col_idx, b.col_idx)


def test_native_rmat_is_a_valid_csr():
    g = gg.rmat_native(13, 16, 77, threads=4)
    deg = np.diff(g.row_ptr)
    assert deg.min() >= 1
    src = np.repeat(np.arange(g.n), deg)
    assert np.all(src != g.col_idx)                       # no loops
    for v in range(0, g.n, 97):                             # sorted, no duplicates
        row = g.neighbors(v)
        assert np.all(np.diff(row) > 0)
    key = src.astype(np.int64) * g.n + g.col_idx
    rev = g.col_idx.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(key), np.sort(rev))       # symmetric
