"""The training step that allocates nothing (tn_mlp_train_step_noalloc)
against the allocating step (tn_mlp_train_step), through the C ABI: two calls
in a row, the second smaller, bit for bit."""
import numpy as np
import pytest
import torch

import tn_inputs as T

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_step_equals_the_allocating_step():
    g = T.rng(5)
    state = {}
    for call, (N, rows) in enumerate(((4096, 4096), (1000, 3000))):
        x = _dev(g.normal(size=(rows, 16)).astype(np.float32))
        y = _dev(g.normal(size=rows).astype(np.float32))
        idx = None if call == 0 else _dev(g.permutation(rows)[:N].astype(np.int32))
        if not state:
            p0 = tn.mlp_init(11)
            state = {"a": [p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)],
                     "b": [p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)]}
        for step in (2 * call + 1, 2 * call + 2):
            pa, ma, va = state["a"]
            pb, mb, vb = state["b"]
            la, ga = tn.mlp_train_step(pa, ma, va, step, x, y, idx=idx, lr=1e-3, want_grad=True)
            lb = torch.full((1,), -1.0, device="cuda")
            gb = torch.full((tn.MLP_PARAMS,), -1.0, device="cuda")
            tn.mlp_train_step_noalloc(pb, mb, vb, step, x, y, idx=idx, lr=1e-3, loss=lb, grad=gb)
            torch.cuda.synchronize()
            assert torch.equal(la, lb) and torch.equal(ga, gb), (call, step)
            for u, v in zip(state["a"], state["b"]):
                assert torch.equal(u, v), (call, step)
            assert bool(torch.isfinite(la).all()) and float(la[0]) > 0


def test_noalloc_step_rejects_more_samples_than_its_array():
    p = tn.mlp_init(3)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    x = torch.zeros((16385, 16), dtype=torch.float32, device="cuda")
    y = torch.zeros(16385, dtype=torch.float32, device="cuda")
    before = p.clone()
    with pytest.raises(tn.TNError) as e:
        tn.mlp_train_step_noalloc(p, m, v, 1, x, y)
    assert e.value.code == -6
    torch.cuda.synchronize()
    assert torch.equal(p, before) and not m.any() and not v.any()
