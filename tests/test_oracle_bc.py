"""Pins of the exact betweenness reference (Brandes) and of the (eps, delta) guarantee.

Betweenness here is the paper's normalisation (Sec. I): ordered pairs,
divided by n(n-1).  networkx normalises undirected graphs by
(n-1)(n-2)/2 over unordered pairs, so b = b_nx * (n-2)/n.
"""
import networkx as nx
import numpy as np
import pytest

import graphgen as gg


def nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for u in g.neighbors(v):
            G.add_edge(v, int(u))
    return G


@pytest.mark.parametrize("make", [lambda: gg.gnm(120, 300, 1), lambda: gg.rmat(8, 8, 3),
                                  lambda: gg.road_grid(12, 2), lambda: gg.hypercube_graph(5)])
def test_brandes_matches_networkx(oracle, make):
    g = make()
    bc = oracle.brandes(g)
    ref = nx.betweenness_centrality(nx_graph(g), normalized=True)
    want = np.array([ref[v] for v in range(g.n)]) * (g.n - 2) / g.n
    assert np.allclose(bc, want, rtol=1e-12, atol=1e-15)


def test_closed_forms(oracle):
    n = 9
    bc = oracle.brandes(gg.path_graph(n))
    i = np.arange(n)
    assert np.allclose(bc, 2 * i * (n - 1 - i) / (n * (n - 1)))
    assert abs(oracle.brandes(gg.path_graph(5))[2] - 0.4) < 1e-15
    bc = oracle.brandes(gg.star_graph(n))
    assert abs(bc[0] - (n - 2) / n) < 1e-15 and np.all(bc[1:] == 0)
    assert np.all(oracle.brandes(gg.complete_graph(7)) == 0)
    bc = oracle.brandes(gg.cycle_graph(10))
    assert np.allclose(bc, bc[0])


def _guarantee_failures(oracle, g, seeds, eps=0.01, delta=0.1):
    bc = oracle.brandes(g)
    lo, hi = oracle.vd_bracket(g)
    omega = oracle.omega_bracket(lo, hi, eps, delta)
    fails, errs = 0, []
    for seed in seeds:
        cal = oracle.calibrate(g, seed=seed, omega_=omega, delta=delta)
        r = oracle.run(g, seed=seed, eps=eps, omega_=omega, epoch=1024, LL=cal["LL"], LU=cal["LU"])
        err = np.abs(r["c"] / r["tau"] - bc).max()
        errs.append(err)
        fails += err > eps
    return fails, max(errs)


def test_guarantee_on_er_workload(oracle):
    fails, worst = _guarantee_failures(oracle, gg.workload("er2048"), range(1, 21))
    assert fails <= 2, (fails, worst)


def test_guarantee_on_small_rmat(oracle):
    fails, worst = _guarantee_failures(oracle, gg.rmat(11, 16, 5), range(1, 21))
    assert fails <= 2, (fails, worst)
