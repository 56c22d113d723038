"""Pins of the oracle's learned-prior pieces (features, MLP, Adam).

References: central finite differences of the oracle's own loss, PyTorch
CPU autograd in float64 (an independent implementation of the same
network), torch.optim.Adam in float64, and features recomputed from a
networkx graph.
"""
import math

import networkx as nx
import numpy as np
import pytest
import torch

import graphgen as gg

NP = 4481


def random_params(seed, scale=0.3):
    r = np.random.default_rng(seed)
    return r.normal(0, scale, NP)


def torch_net(p):
    t = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    W1 = t[:192].view(64, 3)
    b1 = t[192:256]
    W2 = t[256:4352].view(64, 64)
    b2 = t[4352:4416]
    W3 = t[4416:4480].view(1, 64)
    b3 = t[4480:4481]

    def fwd(x):
        h = torch.relu(x @ W1.T + b1)
        h = torch.relu(h @ W2.T + b2)
        return (h @ W3.T + b3).squeeze(-1)
    return t, fwd


def test_forward_matches_torch(oracle):
    p = random_params(1)
    x = np.random.default_rng(2).normal(size=(257, 3))
    y = oracle.mlp_forward(p, x)
    _, fwd = torch_net(p)
    want = fwd(torch.tensor(x)).detach().numpy()
    assert np.allclose(y, want, rtol=1e-12, atol=1e-12)


def test_gradient_matches_torch_autograd(oracle):
    p = random_params(3)
    r = np.random.default_rng(4)
    x = r.normal(size=(300, 3))
    tgt = r.normal(size=300)
    loss, grad = oracle.mlp_loss_grad(p, x, tgt)
    t, fwd = torch_net(p)
    L = ((fwd(torch.tensor(x)) - torch.tensor(tgt)) ** 2).mean()
    L.backward()
    assert abs(loss - L.item()) <= 1e-12 * abs(loss)
    assert np.allclose(grad, t.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_gradient_matches_finite_differences(oracle):
    p = random_params(5)
    r = np.random.default_rng(6)
    x = r.normal(size=(40, 3))
    tgt = r.normal(size=40)
    _, grad = oracle.mlp_loss_grad(p, x, tgt)
    idx = np.concatenate([np.arange(0, 256, 7), np.arange(256, 4481, 97), [4480]])
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (oracle.mlp_loss_grad(pp, x, tgt)[0] - oracle.mlp_loss_grad(pm, x, tgt)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), i


def test_adam_matches_torch(oracle):
    p = random_params(7)
    r = np.random.default_rng(8)
    t = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(NP)
    v = np.zeros(NP)
    q = p.copy()
    for step in range(1, 6):
        g = r.normal(size=NP)
        oracle.adam_step(q, g, m, v, step)
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(q, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_match_networkx(oracle):
    g = gg.rmat(9, 8, 4)
    x = oracle.features(g)
    G = nx.Graph()
    for v in range(g.n):
        for u in g.neighbors(v):
            G.add_edge(v, int(u))
    for v in range(0, g.n, 13):
        nb = list(G.neighbors(v))
        dv = len(nb)
        want = [math.log1p(dv), sum(math.log1p(G.degree(u)) for u in nb) / dv,
                math.log1p(sum(G.degree(u) for u in nb))]
        assert np.allclose(x[v], want, rtol=1e-13)
