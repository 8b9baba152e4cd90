"""Pins of the float64 learned-combiner reference: central finite differences,
torch autograd and torch's Adam on the CPU (library routines)."""
import numpy as np
import torch

import tn_inputs as T
from oracle import mlp


def _batch(N, seed):
    g = T.rng(seed)
    x = g.normal(size=(N, 16))
    y = g.normal(size=N)
    return x, y


def test_gradient_matches_central_differences():
    p = T.mlp_init(1).astype(np.float64)
    x, y = _batch(37, 2)
    gr = mlp.grad(p, x, y)
    g = T.rng(3)
    idx = g.choice(p.shape[0], 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, y) - mlp.loss(p - e, x, y)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(fd)), i


def _torch_model(p):
    layers = mlp.unpack(p)
    mods = []
    for i, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if i < len(layers) - 1:
            mods.append(torch.nn.ReLU())
    return torch.nn.Sequential(*mods)


def test_gradient_and_adam_match_torch():
    p = T.mlp_init(4).astype(np.float64)
    x, y = _batch(64, 5)
    model = _torch_model(p)
    opt = torch.optim.Adam(model.parameters(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    cur = p.copy()
    for step in range(1, 4):
        opt.zero_grad()
        out = model(torch.from_numpy(x))[:, 0]
        loss = torch.mean((out - torch.from_numpy(y)) ** 2)
        loss.backward()
        tg = np.concatenate([torch.cat([mod.weight.grad.ravel(), mod.bias.grad])
                             .numpy() for mod in model if isinstance(mod, torch.nn.Linear)])
        g = mlp.grad(cur, x, y)
        assert np.allclose(g, tg, rtol=1e-10, atol=1e-12)
        assert abs(mlp.loss(cur, x, y) - loss.item()) < 1e-12
        opt.step()
        cur, m, v = mlp.adam_step(cur, m, v, g, step)
        tp = np.concatenate([torch.cat([mod.weight.detach().ravel(), mod.bias.detach()])
                             .numpy() for mod in model if isinstance(mod, torch.nn.Linear)])
        assert np.allclose(cur, tp, rtol=1e-10, atol=1e-12)


def test_first_adam_step_is_lr_times_sign():
    p = T.mlp_init(6).astype(np.float64)
    x, y = _batch(50, 7)
    g = mlp.grad(p, x, y)
    q, _, _ = mlp.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, 1, lr=1e-3)
    big = np.abs(g) > 1e-4
    assert np.allclose((p - q)[big], 1e-3 * np.sign(g[big]), rtol=1e-3)
