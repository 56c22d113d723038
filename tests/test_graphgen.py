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


def test_hyperbolic_graph_shape():
    """The hyperbolic builder's graph: symmetric CSR with sorted rows, no
    loops or duplicates, connected (largest component kept), average degree
    near the requested one, and a heavy degree tail (power law, exponent
    about 3: the complementary CDF falls by about 4x per doubling)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    g = gg.hyperbolic(15, 40.0, 3)
    n = g.n
    deg = np.diff(g.row_ptr)
    assert n > 0.9 * (1 << 15)
    assert 0.85 * 40 <= deg.mean() <= 1.15 * 40
    rows = np.repeat(np.arange(n), deg)
    assert np.all(g.col_idx != rows)
    for v in range(0, n, 97):
        r = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
        assert np.all(np.diff(r) > 0)
    a = sp.csr_matrix((np.ones(len(rows)), (rows, g.col_idx)), shape=(n, n))
    assert (a != a.T).nnz == 0
    assert connected_components(a, directed=False)[0] == 1
    # tail: P(deg >= 2k) / P(deg >= k) near 2^-(gamma - 1) = 1/4 for k well above the mean
    k = 4 * 40
    ratio = (deg >= 2 * k).mean() / (deg >= k).mean()
    assert 0.12 <= ratio <= 0.45, ratio
    assert deg.max() > 10 * deg.mean()
