"""Pins of the float64 learned-combiner reference: central finite differences,
torch autograd and torch's Adam on the CPU (library routines)."""
import os

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


def test_splitmix64_known_answer():
    # the published first outputs of SplitMix64 for one seed (golden file)
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    lines = [ln.split("#", 1)[0].strip() for ln in open(path)]
    lines = [ln for ln in lines if ln]
    seed = int(lines[0].split()[1])
    want = [int(v) for v in lines[1:]]
    assert mlp.splitmix64(seed, len(want)) == want


def test_init_bounds_biases_and_moments():
    # He-uniform: weights of layer i uniform on (-sqrt(6/fan_in), sqrt(6/fan_in)),
    # biases zero; mean 0 and variance bound^2 / 3 within sampling error
    p = mlp.init(11).astype(np.float64)
    for W, b in mlp.unpack(p):
        bound = np.sqrt(6.0 / W.shape[1])
        assert (np.abs(W) <= bound).all() and (b == 0).all()
        k = W.size
        assert abs(W.mean()) < 5 * bound / np.sqrt(3 * k)
        var = W.var()
        # variance of the sample variance of a uniform: (bound^4)(1/5 - 1/9) / k
        assert abs(var - bound ** 2 / 3) < 5 * bound ** 2 * np.sqrt((1 / 5 - 1 / 9) / k)
        # the draws fill the whole interval
        assert W.min() < -0.9 * bound and W.max() > 0.9 * bound
    assert (mlp.init(11) == mlp.init(11)).all()
    assert (mlp.init(11) != mlp.init(12)).mean() > 0.9
