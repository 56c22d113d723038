"""Exact vertex diameter on the device (iFUB with multi-source BFS) against
the oracle: the definition (a BFS from every vertex) on small graph
families, and on the 2048 x 2048 perturbed grid, whose three-sweep bracket
is wide, a single value inside the bracket whose witness vertex has the
claimed eccentricity (an oracle BFS).  A sampler asked for the exact
diameter takes omega from it."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

K = None

FAMILIES = {
    "er400": lambda: gg.gnm(400, 900, 3),
    "rmat10": lambda: gg.rmat(10, 8, 2),
    "rmat12": lambda: gg.rmat(12, 16, 9),
    "road40": lambda: gg.road_grid(40, 5),
    "road64": lambda: gg.road_grid(64, 8),
    "grid30x47": lambda: gg.grid_graph(30, 47),
    "path300": lambda: gg.path_graph(300),
    "star50": lambda: gg.star_graph(50),
    "complete30": lambda: gg.complete_graph(30),
    "cycle101": lambda: gg.cycle_graph(101),
    "hypercube8": lambda: gg.hypercube_graph(8),
    "rc500": lambda: gg.random_connected(500, 100, 4),
    "two": lambda: gg.path_graph(2),
}


@pytest.fixture(scope="module")
def ctx():
    global K
    from paper_1910_11039_amd import kadabra as KK
    K = KK
    c = K.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name", list(FAMILIES))
def test_exact_vd_matches_oracle(ctx, oracle, name):
    g = FAMILIES[name]()
    G = K.Graph(ctx, g, validate=True)
    vd, wit, runs = K.kad_exact_vd(ctx.h, G.h)
    assert vd == oracle.exact_vd(g)
    assert oracle.eccentricity(g, wit) == vd - 1
    lo, hi = oracle.vd_bracket(g)
    assert lo <= vd <= hi


def test_exact_diameter_sampler_takes_omega_from_it(ctx, oracle):
    g = gg.rmat(12, 16, 9)
    G = K.Graph(ctx, g)
    S = K.Sampler(G, seed=1, epsilon=0.02, delta=0.1, exact_diameter=1)
    r = S.result()
    assert r.omega == oracle.omega(oracle.exact_vd(g), 0.02, 0.1)
    assert r.vd_lo <= oracle.exact_vd(g) <= r.vd_hi


@pytest.mark.parametrize("name", ["grid2048", "rmat20"])
def test_exact_vd_at_full_size(ctx, oracle, name):
    """The grid's bracket [3216, 5335] collapses to one value; R-MAT 20's
    [9, 11] too.  The witness's eccentricity is checked by the oracle."""
    import time
    g = gg.workload(name)
    G = K.Graph(ctx, g)
    t0 = time.perf_counter()
    vd, wit, runs = K.kad_exact_vd(ctx.h, G.h)
    dt = time.perf_counter() - t0
    lo, hi = oracle.vd_bracket(g)
    print(f"{name}: VD={vd} in [{lo}, {hi}], witness {wit}, {runs} BFS runs, {dt * 1e3:.1f} ms", flush=True)
    assert lo <= vd <= hi
    assert oracle.eccentricity(g, wit) == vd - 1
