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


def test_prior_from_output_inverts_the_target(oracle):
    """The target is y = ln(b + 1/omega); the prior inverts it on [0, 1]
    and clamps outside: y = ln(1/omega) gives 0, anything below gives 0,
    y = ln(1 + 1/omega) gives 1, anything above gives 1."""
    omega = 35000.0
    b = np.array([0.0, 1e-6, 0.003, 0.25, 0.999, 1.0])
    y = np.log(b + 1.0 / omega)
    pr = oracle.prior_from_output(y, omega)
    assert np.allclose(pr, b, rtol=1e-9, atol=1e-15)
    pr = oracle.prior_from_output(np.array([-50.0, np.log(0.5 / omega), 3.0, 40.0]), omega)
    assert list(pr) == [0.0, 0.0, 1.0, 1.0]


def test_init_is_he_uniform(oracle):
    """Weights uniform within +-sqrt(6 / fan_in) (mean and variance of the
    uniform law within 5 standard errors), biases zero."""
    p = oracle.mlp_init(7)
    assert np.all(p[192:256] == 0) and np.all(p[4352:4416] == 0) and p[4480] == 0
    for sl, fan in ((slice(0, 192), 3), (slice(256, 4352), 64), (slice(4416, 4480), 64)):
        w = p[sl]
        b = math.sqrt(6 / fan)
        assert np.all(np.abs(w) < b)
        n = len(w)
        assert abs(w.mean()) <= 5 * b / math.sqrt(3 * n)
        # variance of U(-b, b) is b^2/3; the sample variance's sd is about b^2 sqrt(4/45/n)
        assert abs(w.var() - b * b / 3) <= 5 * b * b * math.sqrt(4 / 45 / n)
    assert not np.array_equal(oracle.mlp_init(7), oracle.mlp_init(8))


def test_batch_rows_are_uniform(oracle):
    """Rows drawn for the Adam steps: chi-square over 20 rows, 2000 steps."""
    from scipy import stats
    rows = 20
    cnt = np.zeros(rows)
    for j in range(2000):
        r = oracle.batch_rows(3, j, 50, rows)
        assert r.min() >= 0 and r.max() < rows
        cnt += np.bincount(r, minlength=rows)
    chi2 = ((cnt - cnt.mean()) ** 2 / cnt.mean()).sum()
    assert stats.chi2.sf(chi2, rows - 1) > 1e-4


def test_training_loop_equals_torch_adam_on_the_same_batches(oracle):
    """The oracle's loop (init, batches, Adam, step-size halving, per-epoch
    loss) against torch autograd + torch.optim.Adam in float64 fed the
    oracle's batches: same parameters and loss curve."""
    r = np.random.default_rng(4)
    rows, batch, epochs, lr, halve = 300, 64, 3, 3e-3, 2
    x = r.normal(size=(rows, 3))
    y = np.sin(x[:, 0]) + 0.3 * x[:, 1]
    p, losses = oracle.mlp_train(x, y, epochs=epochs, batch=batch, lr=lr, halve_every=halve, seed=11)
    t, fwd = torch_net(oracle.mlp_init(11))
    opt = torch.optim.Adam([t], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    X = torch.tensor(x)
    Y = torch.tensor(y)
    steps = (rows + batch - 1) // batch
    j = 0
    tl = []
    for e in range(epochs):
        for g in opt.param_groups:
            g["lr"] = lr * 0.5 ** (e // halve)
        s = 0.0
        for _ in range(steps):
            idx = torch.tensor(oracle.batch_rows(11, j, batch, rows))
            opt.zero_grad()
            loss = ((fwd(X[idx]) - Y[idx]) ** 2).mean()
            loss.backward()
            opt.step()
            s += loss.item()
            j += 1
        tl.append(s / steps)
    assert np.allclose(p, t.detach().numpy(), rtol=1e-9, atol=1e-12)
    assert np.allclose(losses, tl, rtol=1e-12)
