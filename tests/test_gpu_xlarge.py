"""R-MAT scale 26, edge factor 16 (n = 32.8 M, nnz = 2.1 G, about 8.4 GB of
column indices): the batched sampler at full size, as launched by the
benchmark, against the oracle.

Builds the graph once with the threaded generator (about a minute).  The
sampled paths are compared one by one; the plain arm (eps = 0.01, delta =
0.1, autotuned launch shape, every slot pool, timing on) is compared with
the oracle's threaded run over its calibration and first four epochs: the
oracle needs minutes of host time per epoch of this graph, so the run to
the stop is compared on the smaller graphs.
"""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def say(request, msg):
    """A progress line that reaches the log even while pytest captures the
    tests' output: these tests take minutes (graph build, oracle passes)."""
    capman = request.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)


@pytest.fixture(scope="module")
def big(request):
    from paper_1910_11039_amd import kadabra as K
    say(request, "building R-MAT 26")
    g = gg.workload("rmat26")
    say(request, f"n={g.n} nnz={g.nnz}")
    ctx = K.Context(0)
    G = K.Graph(ctx, g)
    say(request, "graph uploaded")
    yield K, ctx, G, g
    ctx.close()


def test_rmat26_sampled_paths_at_full_size(big, oracle, request):
    K, ctx, G, g = big
    L, _ = oracle.uniform_delta(g.n, 0.1)
    d = np.exp(-L)
    S = K.Sampler(G, seed=1, epsilon=0.01, delta=0.1, omega_override=35000.0,
                  alloc_mode=K.KAD_ALLOC_EXPLICIT, epoch_size=2048)
    S.set_delta(d, d)
    O = oracle.Sampler(g, seed=1, stream=0)
    say(request, "oracle sampler ready")
    for first in (0, 123_456_789):
        paths, info = S.sample_paths(0, first, 16, 64)
        for i in range(16):
            p, inf = O.sample(first + i)
            assert np.array_equal(paths[i, : inf.d + 1], p), (first + i, paths[i], p)
            want = [inf.s, inf.t, inf.d, inf.w, inf.fp_mode, inf.meet_size, inf.steps, inf.edges]
            assert list(info[i, :8]) == want, (first + i, list(info[i, :8]), want)
            say(request, f"sample {first + i} equal")
    S.close()


def test_rmat26_first_epochs_match_oracle(big, oracle, request):
    """The plain arm in the benchmark's launch shape (autotuned epoch size
    and workgroups, every slot pool, timing on): omega, the calibration and
    the allocation, then the first four epochs' counters, tau and per-epoch
    f/g maxima equal the oracle's threaded run, epoch by epoch."""
    K, ctx, G, g = big
    S = K.Sampler(G, seed=1, epsilon=0.01, delta=0.1, timing=1)
    stops = [S.step_epoch() for _ in range(4)]
    r = S.result()
    c, tau = S.counts()
    say(request, f"device: E={r.epoch_size} block={r.block_size} slots={r.slots} pools={r.pools} tau={tau} "
                f"stopped={stops}")
    threads = oracle.host_threads()
    og = oracle.Graph(g)
    say(request, "oracle graph ready")
    omega = oracle.omega_bracket(*oracle.vd_bracket(og), 0.01, 0.1)
    assert r.omega == omega
    say(request, f"oracle bracket done, omega={omega}")
    cal = oracle.calibrate(og, seed=1, omega_=omega, threads=threads)
    cp, tau0, Cc = S.calibration()
    assert tau0 == cal["tau0"]
    assert np.array_equal(cp, cal["cprime"])
    assert abs(Cc - cal["C"]) <= 1e-12 * abs(cal["C"])
    dLL, dLU = S.delta_logs()
    assert np.allclose(dLL, cal["LL"], rtol=1e-12, atol=0)
    assert np.allclose(dLU, cal["LU"], rtol=1e-12, atol=0)
    say(request, f"calibration equal (tau0={tau0}); oracle epochs on {threads} threads")
    co = None
    maxf, maxg = [], []
    for k in range(4):
        ref = oracle.run(og, seed=1, eps=0.01, omega_=omega, epoch=r.epoch_size, LL=cal["LL"], LU=cal["LU"],
                         threads=threads, start_epoch=k, stop_after_epochs=1, c_init=co)
        co = ref["c"]
        maxf.append(ref["max_f"][-1])
        maxg.append(ref["max_g"][-1])
        say(request, f"oracle epoch {k} done: tau={ref['tau']} reason={ref['reason']}")
    assert not any(stops[:3])
    assert tau == ref["tau"]
    assert np.array_equal(c, co)
    hist = S.history(4)
    tol = lambda x: 1e-12 * np.maximum(np.abs(x), 0.01)
    assert np.all(np.abs(hist[:, 0] - np.array(maxf)) <= tol(np.array(maxf)))
    assert np.all(np.abs(hist[:, 1] - np.array(maxg)) <= tol(np.array(maxg)))
    S.close()
