"""kad_count_samples_noalloc (the entry point for callers that cannot
allocate) against kad_count_samples and the oracle: the same counters, bit
for bit, on two calls in a row, the second on a smaller graph with fewer
samples (the scratch keeps the first call's contents); a graph whose one
slot does not fit the scratch is refused with KAD_EOVERFLOW."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _noalloc_counts(K, ctx, G, n, seed, stream, first, count, mode):
    d = K.kad_device_alloc(ctx.h, 4 * n)
    try:
        K.kad_memcpy_h2d(ctx.h, d, np.zeros(n, dtype=np.uint32))
        K.kad_count_samples_noalloc(ctx.h, G.h, seed, stream, first, count, mode, d)
        out = np.zeros(n, dtype=np.uint32)
        K.kad_memcpy_d2h(ctx.h, out, d)
    finally:
        K.kad_device_free(ctx.h, d)
    return out


def test_noalloc_counts_equal_count_samples(oracle):
    from paper_1910_11039_amd import kadabra as K
    ctx = K.Context(0)
    try:
        cases = [(gg.rmat(13, 16, 3), 2, 0, 100, 4000, 0),     # n ~ 7k: about 200 slots fit
                 (gg.gnm(300, 900, 5), 5, 1, 7, 500, 1)]        # smaller graph, fewer samples, FP mode
        for g, seed, stream, first, count, mode in cases:
            G = K.Graph(ctx, g, validate=True)
            S = K.Sampler(G, seed=seed, epsilon=0.02, delta=0.1, omega_override=1000.0,
                          alloc_mode=K.KAD_ALLOC_EXPLICIT, sigma_mode=mode)
            want = S.count_samples(stream, first, count)
            S.close()
            got = _noalloc_counts(K, ctx, G, g.n, seed, stream, first, count, mode)
            assert np.array_equal(got, want), (g.name, int(np.abs(got.astype(np.int64) - want).sum()))
            ref, _ = oracle.count(g, seed, stream, first, count, sigma_mode=mode)
            assert np.array_equal(got, ref)
            print(f"{g.name}: n={g.n} {count} samples equal", flush=True)
            G.close()
    finally:
        ctx.close()


def test_noalloc_refuses_a_graph_beyond_the_scratch():
    from paper_1910_11039_amd import kadabra as K
    ctx = K.Context(0)
    try:
        g = gg.path_graph(3_000_000)       # one slot needs about 72 MB
        G = K.Graph(ctx, g)
        d = K.kad_device_alloc(ctx.h, 4 * g.n)
        with pytest.raises(K.KadError) as ei:
            K.kad_count_samples_noalloc(ctx.h, G.h, 1, 0, 0, 10, 0, d)
        assert ei.value.status == -6
        K.kad_device_free(ctx.h, d)
        G.close()
    finally:
        ctx.close()
