"""Learned prior for the delta_L / delta_U allocation.

The paper's calibration phase (Sec. III-A, phase 2) spends a few
non-adaptive samples to choose the per-vertex failure probabilities; any
choice whose sum stays below delta is valid and only changes how soon the
stop rule holds.  Here a small network predicts a betweenness prior from
three cheap per-vertex features instead, and the same allocation rule
turns that prior into delta_L = delta_U.  The plain allocation remains the
fallback (the library uses it whenever the learned one is not finite or
breaks the budget).

Everything numeric runs in the library's HIP kernels (features, targets,
standardisation, initialisation, batches, forward, backward, Adam, all
behind kad_mlp_train); this module only orchestrates: it runs the plain
method on seeded graphs and stores the weights.
"""
from __future__ import annotations

import math
import os

import numpy as np

from . import kadabra as K

N_PARAMS = 4481
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "mlp_prior.npz")
INIT_STREAM = 2   # Philox stream of the initialisation and the shuffles


def _rng(seed: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[(seed + salt) & (2**64 - 1), INIT_STREAM]))


def init_params(seed: int = 7) -> np.ndarray:
    """Random weights in the law of the initialisation (uniform within
    sqrt(6 / fan_in), biases zero; layout W1[64][3], b1[64], W2[64][64],
    b2[64], W3[64], b3) from a host stream: fixed weights for checking the
    network kernels.  Training draws its own on the device."""
    r = _rng(seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[0:192] = r.uniform(-1, 1, 192) * math.sqrt(6 / 3)
    p[256:4352] = r.uniform(-1, 1, 4096) * math.sqrt(6 / 64)
    p[4416:4480] = r.uniform(-1, 1, 64) * math.sqrt(6 / 64)
    return p


def plain_run(ctx: K.Context, g, eps: float = 0.01, delta: float = 0.1, seed: int = 1):
    """Plain KADABRA on the GPU; returns (resident graph, b~, omega, result)."""
    G = K.Graph(ctx, g)
    S = K.Sampler(G, seed=seed, epsilon=eps, delta=delta)
    r = S.run_to_stop()
    b = S.btilde()
    S.close()
    return G, b, r.omega, r


def build_training_set(ctx: K.Context, graphs, eps: float = 0.01, seed: int = 1, log=None):
    """Plain runs on the training graphs: the graphs stay resident, with
    their estimates b~ and omegas (the targets are formed on the device)."""
    Gs, bts, oms = [], [], []
    for g in graphs:
        G, b, omega, r = plain_run(ctx, g, eps=eps, seed=seed)
        Gs.append(G)
        bts.append(b)
        oms.append(omega)
        if log:
            log(f"{g.name}: n={g.n} tau={r.tau} tau0={r.tau0} time={r.t_total_ms:.1f} ms")
    return Gs, bts, oms


def train(ctx: K.Context, Gs, btildes, omegas, epochs: int = 8, batch: int = 4096, lr: float = 2e-3,
          halve_every: int = 3, seed: int = 7):
    """kad_mlp_train: features, targets ln(b~ + 1/omega), standardisation,
    initialisation and Adam on the mean squared error, in the library's
    kernels.  Returns (params, norm, per-epoch losses)."""
    return K.kad_mlp_train(ctx.h, [G.h for G in Gs], btildes, omegas, epochs, batch, lr, halve_every, seed)


def save(path: str, params: np.ndarray, norm: np.ndarray, **meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), norm=norm.astype(np.float32),
             **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str = DEFAULT_WEIGHTS):
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), z["norm"].astype(np.float32)


def main():
    import argparse
    import sys
    import time

    ROOT = os.path.dirname(HERE)
    sys.path.insert(0, ROOT)
    import graphgen as gg

    ap = argparse.ArgumentParser(description="train the learned delta-allocation prior")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--graphs", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--eps", type=float, default=0.01)
    args = ap.parse_args()

    def log(s):
        print(s, flush=True)

    t0 = time.time()
    graphs = gg.training_graphs(args.graphs)
    log(f"graphs ready in {time.time() - t0:.1f} s")
    ctx = K.Context(0)
    Gs, bts, oms = build_training_set(ctx, graphs, eps=args.eps, log=log)
    rows = sum(len(b) for b in bts)
    log(f"training rows: {rows}")
    t1 = time.time()
    params, norm, losses = train(ctx, Gs, bts, oms, epochs=args.epochs)
    log(f"trained in {time.time() - t1:.1f} s; mse per epoch {np.round(losses, 5).tolist()}")
    save(args.out, params, norm, losses=np.array(losses), graph_seeds=np.arange(101, 101 + args.graphs),
         eps=args.eps, rows=rows)
    log(f"saved {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()
