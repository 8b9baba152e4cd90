"""End to end on the GPU: the learned combiner, trained on exact sizes from the
component-matrix path, against the fusion estimator it refines (Sec. 4.2)."""
import numpy as np
import pytest
import torch

import tn_inputs as T

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")
from paper_2307_04890_amd import combiner as cb  # noqa: E402


def dataset(specs, H, K, seed):
    xs, ys, ests, exacts, ns = [], [], [], [], []
    for i, (n, m, Tm, s_) in enumerate(specs):
        s, d, t = T.activity_driven(n, m, Tm, seed=s_)
        f = cb.hashed_features(n, s, d, t, T.hash_coefficients(H, seed=seed + i), K)
        exact = cb.exact_out_sizes(n, s, d, t)
        xs.append(f["x"])
        ys.append(torch.log(exact.float() / n))
        ests.append(f["est"])
        exacts.append(exact)
        ns.append(n)
    return xs, ys, ests, exacts, ns


def test_combiner_gains_over_fusion_estimate():
    H, K = 16, 256
    train = [(3000, 3600, 3000, 100 + i) for i in range(10)]
    held = [(6000, 7200, 6000, 900 + i) for i in range(2)]
    xs, ys, _, _, _ = dataset(train, H, K, 10)
    X = torch.cat(xs).contiguous()
    Y = torch.cat(ys).contiguous()
    comb = cb.Combiner(seed=1)
    g = T.rng(2)
    losses = comb.fit(X, Y, [g.permutation(X.shape[0]) for _ in range(60)], batch=2048, lr=2e-3)
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    hx, _, hest, hexact, hn = dataset(held, H, K, 50)
    mlp_err, est_err = [], []
    for x, est, exact, n in zip(hx, hest, hexact, hn):
        pred = comb.predict(x, n, est=est).cpu().numpy()
        e = exact.cpu().numpy()
        mlp_err.append(cb.relative_errors(pred, e))
        est_err.append(cb.relative_errors(est.cpu().numpy(), e))
        assert (pred <= est.cpu().numpy() + 1e-3).all() and (pred >= 1).all()
    m_mlp = np.mean([r["mean"] for r in mlp_err])
    m_est = np.mean([r["mean"] for r in est_err])
    print(f"held-out mean relative error: combiner {m_mlp:.4f}, fusion estimate {m_est:.4f}")
    assert m_mlp < m_est
