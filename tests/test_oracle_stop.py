"""Pins of the stop rule, omega, the calibration and the epoch loop.

* f and g are the positive roots of the Bernstein-type quadratics
  tau^2 x^2 - 2 L (tau/3 -/+ omega) x - 2 L omega b~ = 0 (residual check, a
  characterisation independent of the closed form), with the closed form
  at b~ = 0 and a 50-digit mpmath evaluation of the roots as pins.
* omega: the worked value for the Erdos-Renyi workload (vertex diameter 6,
  eps = 0.01, delta = 0.1) and the vertex diameter from networkx.
* calibration: sum of delta_L + delta_U below delta / 2 in 50-digit
  arithmetic, and the bisection constant minimal.
* epochs: every epoch before the stop fails the rule, tau is a multiple of
  E or ceil(omega), and a paused-and-resumed run equals an uninterrupted one.
"""
import math

import mpmath as mp
import networkx as nx
import numpy as np
import pytest

import graphgen as gg

rng = np.random.default_rng(1234)


def quad_root(tau, L, omega, b, sign):
    """Positive root of tau^2 x^2 - 2 L (tau/3 + sign*omega) x - 2 L omega b = 0 (mpmath)."""
    mp.mp.dps = 50
    tau, L, omega, b = map(mp.mpf, (tau, L, omega, b))
    A = tau**2
    B = -2 * L * (tau / 3 + sign * omega)
    Cc = -2 * L * omega * b
    return (-B + mp.sqrt(B * B - 4 * A * Cc)) / (2 * A)


@pytest.mark.parametrize("i", range(40))
def test_f_g_are_quadratic_roots(oracle, i):
    r = np.random.default_rng(i)
    omega = float(r.uniform(1e3, 1e6))
    tau = float(r.uniform(0.05, 1.0) * omega)
    L = float(r.uniform(1.0, 40.0))
    b = float(r.uniform(0, 0.3))
    f = oracle.f(b, L, omega, tau)
    g = oracle.g(b, L, omega, tau)
    fr = quad_root(tau, L, omega, b, -1)
    gr = quad_root(tau, L, omega, b, +1)
    # the clamps min(f, b~), min(g, 1 - b~)
    fr = min(fr, mp.mpf(b))
    gr = min(gr, 1 - mp.mpf(b))
    assert abs(f - float(fr)) <= 1e-12 * max(abs(float(fr)), 1e-300) + 1e-300
    assert abs(g - float(gr)) <= 1e-12 * max(abs(float(gr)), 1e-300)


def test_f_g_at_zero_count(oracle):
    for (L, omega, tau) in [(18.22, 29978.66, 10000.0), (5.0, 1e5, 3e4), (30.0, 2e4, 2e4)]:
        assert oracle.f(0.0, L, omega, tau) == 0.0
        g = oracle.g(0.0, L, omega, tau)
        want = 2 * L / tau * (1 / 3 + omega / tau)
        assert abs(g - want) <= 1e-14 * want


def test_floor_delta_forbids_early_stop_on_er(oracle):
    """With the floor allocation delta = beta*delta/(4n) on the Erdos-Renyi
    workload, g(0) < 0.01 needs tau > 11077: a vertex never hit keeps the
    run going until then."""
    n, beta, delta, omega = 2048, 1e-3, 0.1, oracle.omega(6, 0.01, 0.1)
    L = math.log(4 * n / (beta * delta))
    assert oracle.g(0.0, L, omega, 11077.0) > 0.01
    assert oracle.g(0.0, L, omega, 11078.0) < 0.01


def test_omega_worked_value(oracle):
    assert abs(oracle.omega(6, 0.01, 0.1) - 29978.66136776995) < 1e-8
    # the log term vanishes for VD - 2 < 1 and is constant on [2^k + 2, 2^(k+1) + 1]
    assert oracle.omega(2, 0.01, 0.1) == oracle.omega(3, 0.01, 0.1) != oracle.omega(4, 0.01, 0.1)
    assert oracle.omega(6, 0.01, 0.1) == oracle.omega(9, 0.01, 0.1)
    assert oracle.omega(10, 0.01, 0.1) > oracle.omega(9, 0.01, 0.1)


@pytest.mark.parametrize("make", [lambda: gg.gnm(400, 900, 3), lambda: gg.rmat(9, 8, 2),
                                  lambda: gg.road_grid(20, 5), lambda: gg.path_graph(17),
                                  lambda: gg.cycle_graph(12), lambda: gg.star_graph(9)])
def test_vd_bracket_contains_networkx_diameter(oracle, make):
    g = make()
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for u in g.neighbors(v):
            G.add_edge(v, int(u))
    vd = nx.diameter(G) + 1
    lo, hi = oracle.vd_bracket(g)
    assert lo <= vd <= hi
    assert oracle.exact_vd(g) == vd
    om = oracle.omega_bracket(lo, hi, 0.01, 0.1)
    assert om >= oracle.omega(vd, 0.01, 0.1)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_calibration_keeps_delta_budget(oracle, seed):
    g = gg.rmat(10, 8, seed)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), 0.01, 0.1)
    cal = oracle.calibrate(g, seed=seed, omega_=omega, delta=0.1)
    mp.mp.dps = 50
    total = mp.fsum(2 * mp.e ** (-mp.mpf(x)) for x in cal["LL"])
    assert total <= mp.mpf(0.1) / 2
    assert np.all(np.isfinite(cal["LL"])) and np.all(cal["LL"] > 0)
    # vertices never hit get exactly the floor beta * delta / (4 n)
    floor = -math.log(1e-3 * 0.1 / (4 * g.n))
    assert np.allclose(cal["LL"][cal["cprime"] == 0], floor, rtol=0, atol=1e-12)
    # the constant is (nearly) the smallest admissible one
    prior = cal["cprime"] / cal["tau0"]
    Cc = cal["C"]
    target = 0.25 * 0.1 * (1 - 1e-9)
    s_at = mp.fsum(mp.e ** (-mp.mpf(Cc) / mp.mpf(p)) for p in prior if p > 0)
    s_below = mp.fsum(mp.e ** (-mp.mpf(Cc * (1 - 1e-9)) / mp.mpf(p)) for p in prior if p > 0)
    assert s_at <= target * (1 + 1e-12)
    assert s_below > target


def test_calibration_without_hits_is_the_floor(oracle):
    g = gg.complete_graph(12)      # every pair adjacent: no interior vertex
    cal = oracle.calibrate(g, seed=1, omega_=1000.0, delta=0.1)
    assert cal["C"] == 0.0 and np.all(cal["cprime"] == 0)


def test_epoch_invariants_and_resume(oracle):
    g = gg.workload("er2048")
    omega = oracle.omega(6, 0.01, 0.1)
    cal = oracle.calibrate(g, seed=1, omega_=omega)
    full = oracle.run(g, omega_=omega, epoch=1024, LL=cal["LL"], LU=cal["LU"])
    assert full["reason"] == oracle.STOP_COND
    E = 1024
    assert full["tau"] % E == 0 or full["tau"] == math.ceil(omega)
    assert full["tau"] == full["epochs"] * E
    worst = np.maximum(full["max_f"], full["max_g"])
    assert np.all(worst[:-1] >= 0.01) and worst[-1] < 0.01
    # pause after 5 epochs, resume from the counters
    part = oracle.run(g, omega_=omega, epoch=1024, LL=cal["LL"], LU=cal["LU"], stop_after_epochs=5)
    assert part["reason"] == oracle.STOP_PAUSED and part["epochs"] == 5
    rest = oracle.run(g, omega_=omega, epoch=1024, LL=cal["LL"], LU=cal["LU"], start_epoch=5,
                      c_init=part["c"])
    assert rest["tau"] == full["tau"] and rest["epochs"] == full["epochs"]
    assert np.array_equal(rest["c"], full["c"])


def test_omega_cap_truncates_last_epoch(oracle):
    g = gg.gnm(200, 600, 4)
    L, U = oracle.uniform_delta(g.n, 0.1)
    omega = 2500.5            # never satisfied before the cap at this eps
    r = oracle.run(g, eps=1e-4, omega_=omega, epoch=1000, LL=L, LU=U)
    assert r["reason"] == oracle.STOP_OMEGA
    assert r["tau"] == 2501 and r["epochs"] == 3
    c_direct, _ = oracle.count(g, 1, 0, 0, 2501)
    assert np.array_equal(r["c"], c_direct)


def test_eccentricity_matches_networkx(oracle):
    g = gg.rmat(9, 8, 3)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for u in g.neighbors(v):
            G.add_edge(v, int(u))
    ecc = nx.eccentricity(G)
    for v in range(0, g.n, 17):
        assert oracle.eccentricity(g, v) == ecc[v]
    assert oracle.exact_vd(g) == max(ecc.values()) + 1
