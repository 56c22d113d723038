"""Pins of the oracle's sample step: distances, path counts, uniformity.

Independent references: scipy's BFS distances, networkx's enumeration of
all shortest paths, closed forms (grid corner to corner: a binomial;
hypercube antipodes: k!), Python big integers for path counts that
overflow 64 bits, and Brandes' exact betweenness for unbiasedness.
"""
import math
from collections import Counter

import networkx as nx
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path
from scipy.stats import chisquare

import graphgen as gg


def to_nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for u in g.neighbors(v):
            if u > v:
                G.add_edge(v, int(u))
    return G


def dist_matrix(g):
    a = csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    return shortest_path(a, unweighted=True, directed=False)


def assert_shortest_path(g, path, d, s, t):
    assert len(path) == d + 1
    assert path[0] == s and path[-1] == t
    for a, b in zip(path[:-1], path[1:]):
        assert b in set(g.neighbors(a).tolist())
    assert len(set(path.tolist())) == len(path)


SMALL = [
    lambda: gg.gnm(300, 900, 5),
    lambda: gg.rmat(10, 8, 7),
    lambda: gg.grid_graph(12, 15),
    lambda: gg.road_grid(24, 11),
    lambda: gg.hypercube_graph(6),
    lambda: gg.random_connected(200, 60, 4),
]


@pytest.mark.parametrize("make", SMALL)
@pytest.mark.parametrize("mode", [0, 1])
def test_distance_and_path_validity(oracle, make, mode):
    g = make()
    D = dist_matrix(g)
    S = oracle.Sampler(g, seed=11, sigma_mode=mode)
    for i in range(300):
        path, info = S.sample(i)
        assert info.d == D[info.s, info.t]
        assert_shortest_path(g, path, info.d, info.s, info.t)
        assert info.w in set(path.tolist())


@pytest.mark.parametrize("make", SMALL[:3] + SMALL[5:])
def test_int_sigma_is_the_number_of_shortest_paths(oracle, make):
    g = make()
    G = to_nx(g)
    S = oracle.Sampler(g, seed=2)
    for i in range(60):
        _, info = S.sample(i)
        assert info.fp_mode == 0
        want = sum(1 for _ in nx.all_shortest_paths(G, info.s, info.t))
        assert info.sigma_st_int == want


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (8, 8), (20, 13)])
def test_grid_corner_sigma_is_binomial(oracle, a, b):
    g = gg.grid_graph(a, b)
    S = oracle.Sampler(g, seed=1)
    _, info = S.sample_fixed(0, 0, a * b - 1)
    assert info.d == a + b - 2
    assert info.sigma_st_int == math.comb(a + b - 2, a - 1)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 7])
def test_hypercube_antipodes_sigma_is_factorial(oracle, k):
    g = gg.hypercube_graph(k)
    S = oracle.Sampler(g, seed=1)
    _, info = S.sample_fixed(0, 0, (1 << k) - 1)
    assert info.d == k
    assert info.sigma_st_int == math.factorial(k)


@pytest.mark.parametrize("a", [40, 120, 450])
def test_fp_sigma_matches_big_integers(oracle, a):
    """Corner to corner on an a x a grid: C(2a-2, a-1) overflows uint64 for
    a >= 35; each side of the search grows about a layers, and a layer's
    largest count exceeds 2^400 once a side passes about 410 layers, so at
    a = 450 both sides rescale."""
    g = gg.grid_graph(a, a)
    S = oracle.Sampler(g, seed=1)
    _, info = S.sample_fixed(0, 0, a * a - 1)
    assert info.fp_mode == 1
    exact = math.comb(2 * a - 2, a - 1)
    # compare log2 of the scaled FP value with log2 of the exact count
    got = math.log2(info.sigma_st) + info.sigma_exp
    want = math.log2(exact)
    layers = 2 * a
    assert abs(got - want) <= layers * 8 * 2.0**-53 * 4 / math.log(2) + 1e-12
    if a >= 430:
        assert info.sigma_exp >= 800


def test_forced_fp_matches_int_below_2_53(oracle):
    g = gg.gnm(300, 900, 5)
    Si = oracle.Sampler(g, seed=3, sigma_mode=0)
    Sf = oracle.Sampler(g, seed=3, sigma_mode=1)
    for i in range(200):
        _, a = Si.sample(i)
        _, b = Sf.sample(i)
        assert b.fp_mode == 1 and a.fp_mode == 0
        assert b.sigma_exp == 0 and b.sigma_st == float(a.sigma_st_int)


def _path_chi2(oracle, g, s, t, mode, N=6000):
    G = to_nx(g)
    paths = [tuple(p) for p in nx.all_shortest_paths(G, s, t)]
    S = oracle.Sampler(g, seed=5, sigma_mode=mode)
    cnt = Counter()
    for i in range(N):
        p, _ = S.sample_fixed(i, s, t)
        cnt[tuple(int(x) for x in p)] += 1
    assert set(cnt) <= set(paths)
    obs = np.array([cnt[p] for p in paths], dtype=float)
    return chisquare(obs).pvalue, len(paths)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", ["hypercube", "grid", "random", "ladder"])
def test_paths_are_uniform(oracle, mode, case):
    if case == "hypercube":
        g, s, t = gg.hypercube_graph(4), 0, 15
    elif case == "grid":
        g, s, t = gg.grid_graph(4, 5), 0, 19
    elif case == "random":
        g = gg.random_connected(40, 70, 9)
        D = dist_matrix(g)
        G = to_nx(g)
        best = max(((a, b) for a in range(g.n) for b in range(g.n) if a != b and D[a, b] >= 3),
                   key=lambda p: (sum(1 for _ in nx.all_shortest_paths(G, *p)), -p[0], -p[1]))
        s, t = best
    else:  # two hubs joined by many 2-paths plus a tail: unequal meet weights
        u = [0] * 6 + list(range(1, 7)) + [7, 8, 8]
        v = list(range(1, 7)) + [7] * 6 + [8, 9, 10]
        g = gg.from_edges(11, np.array(u), np.array(v))
        s, t = 0, 9
    p, k = _path_chi2(oracle, g, s, t, mode)
    assert k >= 2
    assert p > 1e-4


def test_overflowing_grid_paths_cross_the_antidiagonal_hypergeometrically(oracle):
    """On an m x m grid of steps (m = 36, C(72, 36) > 2^64) a uniform corner
    to corner path crosses anti-diagonal i + j = k at row i with probability
    C(k, i) C(2m - k, m - i) / C(2m, m)."""
    m = 36
    g = gg.grid_graph(m + 1, m + 1)
    S = oracle.Sampler(g, seed=8)
    k = m
    hits = Counter()
    N = 4000
    for it in range(N):
        p, info = S.sample_fixed(it, 0, (m + 1) * (m + 1) - 1)
        assert info.fp_mode == 1
        v = int(p[k])
        r, c = divmod(v, m + 1)
        assert r + c == k
        hits[r] += 1
    probs = np.array([math.comb(k, i) * math.comb(2 * m - k, m - i) for i in range(k + 1)], dtype=float)
    probs /= probs.sum()
    keep = probs * N >= 5
    obs = np.array([hits[i] for i in range(k + 1)], dtype=float)
    exp = probs * N
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    assert chisquare(o, e).pvalue > 1e-4


def test_counts_are_unbiased_for_betweenness(oracle):
    g = gg.random_connected(30, 25, 21)
    bc = oracle.brandes(g)
    N = 200000
    c, _ = oracle.count(g, 13, 0, 0, N)
    bt = c / N
    se = np.sqrt(np.maximum(bc * (1 - bc), 1e-12) / N)
    assert np.all(np.abs(bt - bc) <= 5 * se + 1e-12)


def test_adjacent_pair_has_no_interior(oracle):
    g = gg.path_graph(2)
    S = oracle.Sampler(g)
    p, info = S.sample(0)
    assert info.d == 1 and len(p) == 2


def test_disconnected_pair_is_an_error(oracle):
    g = gg.from_edges(4, np.array([0, 2]), np.array([1, 3]))
    S = oracle.Sampler(g)
    with pytest.raises(RuntimeError):
        S.sample_fixed(0, 0, 3)
