"""R-MAT scale 26, edge factor 16 (n = 32.8 M, nnz = 2.1 G, about 8.4 GB of
column indices): the batched sampler at full size, as launched by the
runs, against the oracle on sampled outputs.

Builds the graph with the threaded generator (about a minute); the
oracle then walks the same samples one by one.
"""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def test_rmat26_sampled_paths_at_full_size(oracle):
    from paper_1910_11039_amd import kadabra as K
    print("building R-MAT 26", flush=True)
    g = gg.workload("rmat26")
    print(f"n={g.n} nnz={g.nnz}", flush=True)
    ctx = K.Context(0)
    try:
        G = K.Graph(ctx, g)
        L, _ = oracle.uniform_delta(g.n, 0.1)
        d = np.exp(-L)
        S = K.Sampler(G, seed=1, epsilon=0.01, delta=0.1, omega_override=35000.0,
                      alloc_mode=K.KAD_ALLOC_EXPLICIT, epoch_size=2048)
        S.set_delta(d, d)
        O = oracle.Sampler(g, seed=1, stream=0)
        for first in (0, 123_456_789):
            paths, info = S.sample_paths(0, first, 16, 64)
            for i in range(16):
                p, inf = O.sample(first + i)
                assert np.array_equal(paths[i, : inf.d + 1], p), (first + i, paths[i], p)
                want = [inf.s, inf.t, inf.d, inf.w, inf.fp_mode, inf.meet_size, inf.steps, inf.edges]
                assert list(info[i, :8]) == want, (first + i, list(info[i, :8]), want)
            print(f"samples {first}..{first + 15} equal", flush=True)
        S.close()
        G.close()
    finally:
        ctx.close()
