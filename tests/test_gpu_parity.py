"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Integer and index results (pairs, paths, counters, tau, stop epoch, the
calibration counters) must match bit for bit; FP64 values (f, g, the
allocation constant) within 1e-12 relative (|d| <= 1e-12 * max(|x|, eps)).
"""
import math

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

K = None


@pytest.fixture(scope="module")
def ctx():
    global K
    from paper_1910_11039_amd import kadabra as KK
    K = KK
    c = K.Context(0)
    yield c
    c.close()


def upload(ctx, g):
    return K.Graph(ctx, g, validate=True)


def explicit_sampler(G, g, oracle, eps=0.01, omega=None, epoch=1024, seed=1, **kw):
    if omega is None:
        omega = oracle.omega_bracket(*oracle.vd_bracket(g), eps, 0.1)
    L, _ = oracle.uniform_delta(g.n, 0.1)
    S = K.Sampler(G, seed=seed, epsilon=eps, delta=0.1, epoch_size=epoch, omega_override=omega,
                  alloc_mode=K.KAD_ALLOC_EXPLICIT, **kw)
    d = np.exp(-L)
    S.set_delta(d, d)
    return S, omega


def test_philox_draws_match_oracle(ctx, oracle):
    for seed, stream, first in [(1, 0, 0), (42, 1, 12345), (2**63 + 5, 3, 2**40)]:
        got = K.kad_philox(ctx.h, seed, stream, first, 64, 11)
        for i in range(0, 64, 7):
            for j in range(11):
                assert int(got[i, j]) == oracle.draw(seed, stream, first + i, j)


@pytest.mark.parametrize("make", [lambda: gg.gnm(400, 900, 3), lambda: gg.rmat(10, 8, 2),
                                  lambda: gg.road_grid(40, 5), lambda: gg.path_graph(300),
                                  lambda: gg.star_graph(50), lambda: gg.complete_graph(30)])
def test_vd_bracket_matches_oracle(ctx, oracle, make):
    g = make()
    G = upload(ctx, g)
    assert K.kad_vd_bracket(ctx.h, G.h) == oracle.vd_bracket(g)


PATH_CASES = {
    "er300": lambda: gg.gnm(300, 900, 5),
    "rmat10": lambda: gg.rmat(10, 8, 7),
    "rmat12": lambda: gg.rmat(12, 16, 9),
    "grid12x15": lambda: gg.grid_graph(12, 15),
    "grid64": lambda: gg.grid_graph(64, 64),          # corner-ish pairs overflow uint64
    "road48": lambda: gg.road_grid(48, 11),
    "hypercube8": lambda: gg.hypercube_graph(8),
    "rc200": lambda: gg.random_connected(200, 60, 4),
    "path300": lambda: gg.path_graph(300),
    "star40": lambda: gg.star_graph(40),
    "complete20": lambda: gg.complete_graph(20),
    "two": lambda: gg.path_graph(2),
}


def compare_paths(ctx, oracle, g, mode, count=300, seed=11, stream=0, first=0, **kw):
    G = upload(ctx, g)
    S, _ = explicit_sampler(G, g, oracle, seed=seed, sigma_mode=mode, **kw)
    try:
        return _compare_paths(S, g, oracle, mode, count, seed, stream, first)
    finally:
        S.close()
        G.close()


def _compare_paths(S, g, oracle, mode, count, seed, stream, first):
    max_len = g.n + 1
    paths, info = S.sample_paths(stream, first, count, max_len)
    O = oracle.Sampler(g, seed=seed, stream=stream, sigma_mode=mode)
    for i in range(count):
        p, inf = O.sample(first + i)
        d = inf.d
        got = paths[i, : d + 1]
        assert np.array_equal(got, p), (i, got, p)
        assert np.all(paths[i, d + 1:] == -1)
        want = [inf.s, inf.t, inf.d, inf.w, inf.fp_mode, inf.meet_size, inf.steps, inf.edges]
        assert list(info[i, :8]) == want, (i, list(info[i, :8]), want)
        assert info[i, 9] == (2 if (inf.fp_mode and mode == 0) else 1)
    return info


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", list(PATH_CASES))
def test_sample_paths_match_oracle(ctx, oracle, case, mode):
    compare_paths(ctx, oracle, PATH_CASES[case](), mode)


def test_grid_overflow_switches_to_fp(ctx, oracle):
    info = compare_paths(ctx, oracle, gg.grid_graph(80, 80), 0, count=200)
    assert info[:, 4].sum() > 0          # some samples needed FP path counts


@pytest.mark.parametrize("mode", [0, 1])
def test_meet_sets_beyond_lds_capacity(ctx, oracle, mode):
    """Complete bipartite K_{1100,1100}: a same-side pair meets on all 1100
    vertices of the other side (above the 1024 ranked in LDS)."""
    k = 1100
    a, b = np.meshgrid(np.arange(k), np.arange(k, 2 * k))
    g = gg.from_edges(2 * k, a.ravel(), b.ravel())
    info = compare_paths(ctx, oracle, g, mode, count=60 if mode else 200)
    assert info[:, 5].max() == k


@pytest.mark.parametrize("block,slots", [(64, 7), (128, 50), (256, 0), (512, 13), (1024, 0), (1024, 3)])
def test_launch_shapes_give_identical_counts(ctx, oracle, block, slots):
    g = gg.rmat(12, 16, 3)
    G = upload(ctx, g)
    S, _ = explicit_sampler(G, g, oracle, block_size=block, slots=slots)
    c = S.count_samples(0, 100, 3000)
    want, _ = oracle.count(g, 1, 0, 100, 3000)
    assert np.array_equal(c, want)


@pytest.mark.parametrize("block", [64, 128])
def test_reached_filter_aliasing_gives_identical_counts(ctx, oracle, block):
    """More vertices than the small shapes' LDS filter has bits (32 768), so
    distinct vertices share bits and probe scans must fall back to reading
    their records."""
    g = gg.rmat(16, 16, 21)
    assert g.n > 32768
    G = upload(ctx, g)
    S, _ = explicit_sampler(G, g, oracle, block_size=block)
    c = S.count_samples(0, 0, 1500)
    want, _ = oracle.count(g, 1, 0, 0, 1500)
    assert np.array_equal(c, want)


def oracle_threads(oracle):
    return oracle.host_threads()


def _run_and_compare(S, g, oracle, omega, eps, epoch, LL, LU, seed=1, exact_L=True):
    """Runs the sampler to its stop and compares it with the oracle's run on
    the oracle's own L = ln(1/delta) arrays.  The device's L must equal them
    (bit for bit when both are libm logarithms of the caller's delta,
    within 1e-12 relative when the device allocated delta itself).  When a
    stop decision lies within 1e-12 eps of eps (a near tie that rounding
    may decide either way) the run comparison is reported as xfail."""
    r = S.run_to_stop()
    c, tau = S.counts()
    dLL, dLU = S.delta_logs()
    if exact_L:
        assert np.array_equal(dLL, LL) and np.array_equal(dLU, LU)
    else:
        assert np.allclose(dLL, LL, rtol=1e-12, atol=0) and np.allclose(dLU, LU, rtol=1e-12, atol=0)
    ref = oracle.run(g, seed=seed, eps=eps, omega_=omega, epoch=epoch, LL=LL, LU=LU,
                     threads=oracle_threads(oracle))
    margin = float(ref["min_margin"].min())
    if margin < 1e-12 * eps:
        pytest.xfail(f"near tie: smallest |eps - max(f, g)| = {margin:.3e} up to the stop epoch")
    assert (tau, r.epochs, r.stop_reason) == (ref["tau"], ref["epochs"], ref["reason"])
    assert np.array_equal(c, ref["c"])
    hist = S.history(r.epochs)
    tol = lambda x: 1e-12 * np.maximum(np.abs(x), eps)
    assert np.all(np.abs(hist[:, 0] - ref["max_f"]) <= tol(ref["max_f"]))
    assert np.all(np.abs(hist[:, 1] - ref["max_g"]) <= tol(ref["max_g"]))
    f, gv = S.fg()
    fo, go = oracle.fg_arrays(c, tau, omega, LL, LU)
    assert np.all(np.abs(f - fo) <= tol(fo)) and np.all(np.abs(gv - go) <= tol(go))
    return r, ref


def _explicit_run(ctx, oracle, g, eps, epoch, seed=1, **kw):
    """EXPLICIT allocation with delta_L = delta_U = 0.999 delta / (4n): the
    oracle takes its own -ln of the same delta arrays."""
    G = upload(ctx, g)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), eps, 0.1)
    L0, _ = oracle.uniform_delta(g.n, 0.1)
    d = np.exp(-L0)
    S = K.Sampler(G, seed=seed, epsilon=eps, delta=0.1, epoch_size=epoch, omega_override=omega,
                  alloc_mode=K.KAD_ALLOC_EXPLICIT, **kw)
    S.set_delta(d, d)
    L = oracle.neglog(d)
    return _run_and_compare(S, g, oracle, omega, eps, epoch, L, L.copy(), seed=seed)


def test_er_workload_explicit_delta_run_matches_oracle(ctx, oracle):
    """Erdos-Renyi G(2048, 16384), eps = 0.01, delta = 0.1, seed 1, E = 1024,
    with the oracle's calibrated delta passed explicitly."""
    g = gg.workload("er2048")
    G = upload(ctx, g)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), 0.01, 0.1)
    cal = oracle.calibrate(g, seed=1, omega_=omega)
    S = K.Sampler(G, seed=1, epsilon=0.01, delta=0.1, epoch_size=1024, omega_override=omega,
                  alloc_mode=K.KAD_ALLOC_EXPLICIT)
    d = np.exp(-cal["LL"])
    S.set_delta(d, d)
    L = oracle.neglog(d)
    r, ref = _run_and_compare(S, g, oracle, omega, 0.01, 1024, L, L.copy())
    assert r.stop_reason == K.KAD_STOP_COND
    # the run's estimate is within eps of exact betweenness
    bc = oracle.brandes(g)
    assert np.abs(S.btilde() - bc).max() <= 0.01


def _plain_run_matches_oracle(S, g, oracle, eps, seed=1):
    """PLAIN allocation end to end as the library runs it: omega from the
    device bracket, calibration counters bit-exact, constant C within
    1e-12, the device's L within 1e-12 of the oracle's, then the adaptive
    phase (on the oracle's own L) bit-exact."""
    r = S.run_to_stop()
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), eps, 0.1)
    assert r.omega == omega
    cal = oracle.calibrate(g, seed=seed, omega_=omega, threads=oracle_threads(oracle))
    cp, tau0, Cc = S.calibration()
    assert tau0 == cal["tau0"] == r.tau0
    assert np.array_equal(cp, cal["cprime"])
    assert abs(Cc - cal["C"]) <= 1e-12 * abs(cal["C"])
    dLL, dLU = S.delta_logs()
    assert np.allclose(dLL, cal["LL"], rtol=1e-12, atol=0)
    assert np.allclose(dLU, cal["LU"], rtol=1e-12, atol=0)
    c, tau = S.counts()
    ref = oracle.run(g, seed=seed, eps=eps, omega_=omega, epoch=r.epoch_size, LL=cal["LL"], LU=cal["LU"],
                     threads=oracle_threads(oracle))
    margin = float(ref["min_margin"].min())
    if margin < 1e-12 * eps:
        pytest.xfail(f"near tie: smallest |eps - max(f, g)| = {margin:.3e} up to the stop epoch")
    assert (tau, r.epochs, r.stop_reason) == (ref["tau"], ref["epochs"], ref["reason"])
    assert np.array_equal(c, ref["c"])
    return r, ref


def test_er_workload_plain_run_matches_oracle(ctx, oracle):
    """Plain allocation on ER(2048, 16384), E = 1024."""
    g = gg.workload("er2048")
    G = upload(ctx, g)
    S = K.Sampler(G, seed=1, epsilon=0.01, delta=0.1, epoch_size=1024)
    _plain_run_matches_oracle(S, g, oracle, 0.01)


def test_rmat20_benched_plain_run_matches_oracle(ctx, oracle):
    """R-MAT scale 20 at eps = 0.005 exactly as the benchmark launches it:
    autotuned epoch size and workgroup shape, every slot pool, the
    calibration beside the first epochs, timing on; the whole run to its
    stop equals the oracle's (counters, tau, stop epoch)."""
    g = gg.workload("rmat20")
    G = K.Graph(ctx, g)
    S = K.Sampler(G, seed=1, epsilon=0.005, delta=0.1, timing=1)
    r, ref = _plain_run_matches_oracle(S, g, oracle, 0.005)
    print(f"rmat20 benched shape: E={r.epoch_size} block={r.block_size} slots={r.slots} pools={r.pools} "
          f"tau={r.tau} epochs={r.epochs}", flush=True)
    assert r.pools >= 2 and r.epoch_size >= 4096


def test_road_grid_fp_mode_run_matches_oracle(ctx, oracle):
    """FP path counts (forced) for a whole run to the stop on a perturbed
    256 x 256 grid: thousands of samples with hundreds of layers each."""
    g = gg.road_grid(256, 7)
    r, ref = _explicit_run(ctx, oracle, g, 0.02, 768, sigma_mode=K.KAD_SIGMA_FP)
    assert r.fp_samples == r.samples_run


def test_step_epoch_and_omega_cap(ctx, oracle):
    g = gg.gnm(200, 600, 4)
    G = upload(ctx, g)
    S, omega = explicit_sampler(G, g, oracle, eps=1e-4, omega=2500.5, epoch=1000)
    stops = [S.step_epoch() for _ in range(3)]
    assert stops == [False, False, True]
    c, tau = S.counts()
    assert tau == 2501
    want, _ = oracle.count(g, 1, 0, 0, 2501)
    assert np.array_equal(c, want)
    assert S.result().stop_reason in (0, K.KAD_STOP_OMEGA)


@pytest.mark.parametrize("pools", [1, 2, 4])
def test_graph_run_matches_oracle(ctx, oracle, pools):
    """The pooled epoch schedule replayed from a captured hipGraph (epochs
    dealt to 1, 2 or 4 pools and streams, each pool's epoch read on the
    device), timing on, twice in a row: both runs give the oracle's run
    (counters, tau, stop epoch)."""
    g = gg.rmat(12, 16, 5)
    G = upload(ctx, g)
    omega = oracle.omega_bracket(*oracle.vd_bracket(g), 0.02, 0.1)
    L0, _ = oracle.uniform_delta(g.n, 0.1)
    d = np.exp(-L0)
    S = K.Sampler(G, seed=1, epsilon=0.02, delta=0.1, epoch_size=512, omega_override=omega,
                  alloc_mode=K.KAD_ALLOC_EXPLICIT, use_graphs=1, pools=pools, slots=40, timing=1)
    S.set_delta(d, d)
    L = oracle.neglog(d)
    for seed in (1, 2):
        S.reset(seed)
        r, _ = _run_and_compare(S, g, oracle, omega, 0.02, 512, L, L.copy(), seed=seed)
        assert r.pools == pools


@pytest.mark.parametrize("pools", [1, 2, 4])
def test_overlapped_pools_give_the_oracle_run(ctx, oracle, pools):
    """Epochs overlapped across 1, 2 or 4 slot pools and streams: the stop
    epoch, tau and every counter equal the oracle's sequential run."""
    r, _ = _explicit_run(ctx, oracle, gg.rmat(12, 16, 6), 0.02, 256, pools=pools, slots=40)
    assert r.pools == pools


def test_rejects_bad_inputs(ctx, oracle):
    g = gg.from_edges(4, np.array([0, 2]), np.array([1, 3]))
    with pytest.raises(K.KadError) as ei:
        K.Graph(ctx, g, validate=True)
    assert ei.value.status == -4
    g = gg.gnm(100, 300, 1)
    G = upload(ctx, g)
    S = K.Sampler(G, epsilon=0.01, delta=0.1, alloc_mode=K.KAD_ALLOC_EXPLICIT, omega_override=1000.0)
    big = np.full(g.n, 0.1)
    with pytest.raises(K.KadError):
        S.set_delta(big, big)
    with pytest.raises(K.KadError):
        S.run_to_stop()          # EXPLICIT without arrays
    with pytest.raises(K.KadError):
        K.Sampler(G, epsilon=0.0, delta=0.1)
    with pytest.raises(K.KadError) as ei:
        K.Sampler(G, epsilon=0.01, delta=0.1, pools=5)
    assert ei.value.status == -1


def test_rmat20_sampled_paths_at_full_size(ctx, oracle):
    """R-MAT scale 20 (the benchmark graph): 1500 samples spread over the index
    range, every path and its statistics equal to the oracle's."""
    g = gg.workload("rmat20")
    for first in (0, 70000, 139000):
        compare_paths(ctx, oracle, g, 0, count=500, seed=1, first=first)


def test_grid2048_sampled_paths_at_full_size(ctx, oracle):
    """2048 x 2048 perturbed grid: 24 samples (FP path counts), paths equal."""
    g = gg.workload("grid2048")
    info = compare_paths(ctx, oracle, g, 0, count=24, seed=1, first=5000)
    assert info[:, 4].sum() >= 20


@pytest.mark.parametrize("name", ["rmat20", "grid2048"])
def test_vd_bracket_at_full_size(ctx, oracle, name):
    """The bracket's three sweeps on the benchmark graphs: R-MAT's wide
    levels take the bottom-up steps, the grid's thousands of narrow levels
    the single-workgroup and top-down ones; both equal the oracle's."""
    g = gg.workload(name)
    G = K.Graph(ctx, g)
    assert K.kad_vd_bracket(ctx.h, G.h) == oracle.vd_bracket(g)
