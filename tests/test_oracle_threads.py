"""Pins of the oracle's threaded runner, its -ln(delta) and its check margin.

* The threaded runner (every epoch split over threads, thread-local state
  frames summed at the boundary) must give the single-threaded run's
  counters, tau, stop epoch and per-epoch f/g bit for bit: integer sums and
  max/min/AND do not depend on the order.  Checked on three graph families,
  both sigma modes, thread counts that do and do not divide the epoch, and
  a paused-and-resumed run.
* -ln(delta): against 50-digit mpmath logarithms, within one ulp.
* The check's smallest margin |eps - max(f, g)|: with every count zero,
  f = 0 and g is the closed form (2L/tau)(1/3 + omega/tau), so the margin is
  |eps - g(0)| at the vertex with the largest L.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import graphgen as gg

CASES = {
    "rmat12": lambda: gg.rmat(12, 16, 4),
    "er": lambda: gg.gnm(1500, 6000, 2),
    "road40": lambda: gg.road_grid(40, 5),
}


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("threads", [2, 3, 8])
@pytest.mark.parametrize("case", list(CASES))
def test_threaded_run_equals_single_thread(oracle, case, threads, mode):
    g = oracle.Graph(CASES[case]())
    L, U = oracle.uniform_delta(g.n, 0.1)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), 0.03, 0.1)
    a = oracle.run(g, seed=3, eps=0.03, omega_=omega, epoch=333, LL=L, LU=U, sigma_mode=mode)
    b = oracle.run(g, seed=3, eps=0.03, omega_=omega, epoch=333, LL=L, LU=U, sigma_mode=mode,
                   threads=threads)
    assert (a["tau"], a["epochs"], a["reason"], a["edges"]) == (b["tau"], b["epochs"], b["reason"], b["edges"])
    assert np.array_equal(a["c"], b["c"])
    for k in ("max_f", "max_g", "min_margin"):
        assert np.array_equal(a[k], b[k]), k


def test_threaded_count_equals_single_thread(oracle):
    g = oracle.Graph(gg.rmat(13, 16, 8))
    for first, cnt, threads in [(0, 2000, 5), (12345, 777, 16), (7, 3, 8)]:
        c1, e1 = oracle.count(g, 2, 1, first, cnt)
        c2, e2 = oracle.count(g, 2, 1, first, cnt, threads=threads)
        assert np.array_equal(c1, c2) and e1 == e2


def test_threaded_pause_and_resume(oracle):
    g = oracle.Graph(gg.rmat(12, 16, 9))
    L, U = oracle.uniform_delta(g.n, 0.1)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), 0.03, 0.1)
    full = oracle.run(g, seed=5, eps=0.03, omega_=omega, epoch=256, LL=L, LU=U)
    part = oracle.run(g, seed=5, eps=0.03, omega_=omega, epoch=256, LL=L, LU=U, stop_after_epochs=3,
                      threads=4)
    assert part["reason"] == oracle.STOP_PAUSED and part["epochs"] == 3
    rest = oracle.run(g, seed=5, eps=0.03, omega_=omega, epoch=256, LL=L, LU=U, start_epoch=3,
                      c_init=part["c"], threads=6)
    assert (rest["tau"], rest["epochs"]) == (full["tau"], full["epochs"])
    assert np.array_equal(rest["c"], full["c"])


def test_threaded_calibration_equals_single_thread(oracle):
    g = oracle.Graph(gg.rmat(12, 16, 2))
    om = oracle.omega_bracket(*oracle.vd_bracket(g), 0.01, 0.1)
    a = oracle.calibrate(g, seed=1, omega_=om)
    b = oracle.calibrate(g, seed=1, omega_=om, threads=5)
    assert np.array_equal(a["cprime"], b["cprime"]) and a["C"] == b["C"]
    assert np.array_equal(a["LL"], b["LL"])


def test_neglog_within_one_ulp_of_mpmath(oracle):
    mp.mp.dps = 50
    r = np.random.default_rng(17)
    d = np.concatenate([r.uniform(1e-12, 1.0, 300), 10.0 ** r.uniform(-300, -1, 300),
                        [1e-308, 0.5, 0.999999999, 1.0 - 2.0 ** -52]])
    L = oracle.neglog(d)
    for x, l in zip(d, L):
        want = -mp.log(mp.mpf(float(x)))
        assert abs(mp.mpf(float(l)) - want) <= mp.mpf(math.ulp(float(want))), (x, l)


def test_check_margin_closed_form_at_zero_counts(oracle):
    n = 50
    r = np.random.default_rng(3)
    LL = r.uniform(5.0, 20.0, n)
    LU = r.uniform(5.0, 20.0, n)
    c = np.zeros(n, dtype=np.uint32)
    for tau, omega, eps in [(10000, 29978.66, 0.01), (50000, 60000.0, 0.01), (2000, 2500.0, 0.05)]:
        ok, ci = oracle.check(c, tau, omega, eps, LL, LU)
        g0 = 2 * LU.max() / tau * (1 / 3 + omega / tau)
        assert ci.max_f == 0.0
        assert abs(ci.max_g - g0) <= 1e-14 * g0
        # every vertex's margin is |eps - g(0)| at its own L; g(0) grows with L
        margins = np.abs(eps - 2 * LU / tau * (1 / 3 + omega / tau))
        assert abs(ci.min_abs_margin - margins.min()) <= 1e-14 * max(margins.min(), 1e-300) + 1e-17
        assert ok == (g0 < eps)
