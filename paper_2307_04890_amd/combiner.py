"""Learned combiner on top of the hashing framework.

The fusion estimator of Sec. 4.2 returns a superset of each out-component,
so its size overestimates.  The combiner is a 16 -> 64 -> 64 -> 1 ReLU
network (FP32, trained and evaluated by the library's own kernels) that maps
the H = 16 per-hash lifted sizes |h_j^{-1}(OC_j(h_j(u)))| of a node, as
ln(size / n), to ln(|OC(u)| / n).  It is trained on exact sizes from the
component-matrix path; at inference its estimate is clamped to [1, fusion
estimate], since the fusion estimate is an upper bound.

Everything here is orchestration of C-ABI calls: features, exact sizes,
training steps and predictions all run in libtn's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def hashed_features(n, src, dst, t, coeffs, K, flags=0, ctx=None):
    """Hash, build the H proxies (streamed, all H per batched launch), fuse.
    Returns a dict with the MLP features x (n, H), the fusion estimate est
    (n,), the lifted sizes (H, n), and the proxies P (H, K, ldK)."""
    ctx = ctx or api.get_context()
    bucket, count, P, _ = api.hash_build_proxies(n, src, dst, t, coeffs, K, flags=flags, ctx=ctx)
    est, lifted = api.recombine(P, bucket, count, n, ctx=ctx)
    x = api.mlp_features(lifted, n, ctx=ctx)
    return {"x": x, "est": est, "lifted": lifted, "P": P, "bucket": bucket, "count": count}


def exact_out_sizes(n, src, dst, t, flags=0, ctx=None):
    """Exact maximum out-component sizes (row popcounts of the component matrix)."""
    C = api.build_component_matrix(n, src, dst, t, flags=flags, ctx=ctx)
    out, _ = api.component_sizes(C, n, inn=False, ctx=ctx)
    del C
    return out


def exact_out_sizes_batched(nets, flags=0, ctx=None):
    """Exact out-sizes of many networks built in one persistent launch."""
    b = api.Batch(nets, flags=flags, ctx=ctx)
    Cs = b.execute()
    outs = [api.component_sizes(C, n, inn=False, ctx=ctx)[0] for C, (n, *_rest) in zip(Cs, nets)]
    b.close()
    return outs


class Combiner:
    """The trainable network: parameters and Adam moments live on the device."""

    def __init__(self, seed: int = 1, init_params: np.ndarray | None = None,
                 device: int | None = None):
        """Parameters from tn_mlp_init(seed) on the device, or copied from
        ``init_params`` when given."""
        if device is None:
            device = torch.cuda.current_device()
        if init_params is None:
            self.params = api.mlp_init(seed)
        else:
            p = np.ascontiguousarray(init_params, dtype=np.float32)
            if p.shape != (api.MLP_PARAMS,):
                raise ValueError(f"expected {api.MLP_PARAMS} parameters")
            self.params = torch.from_numpy(p).to(f"cuda:{device}")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def fit(self, x: torch.Tensor, y: torch.Tensor, orders, batch: int = 4096, lr: float = 1e-3):
        """One epoch per permutation in ``orders`` (host int arrays over the rows
        of x); returns the loss of every step."""
        losses = []
        for order in orders:
            order = torch.from_numpy(np.ascontiguousarray(order, dtype=np.int32)).to(x.device)
            N = order.shape[0]
            for lo in range(0, N, batch):
                self.step += 1
                loss, _ = api.mlp_train_step(self.params, self.m, self.v, self.step, x, y,
                                             idx=order[lo:lo + batch], lr=lr)
                losses.append(loss)
        return [float(v) for v in torch.cat(losses).cpu()] if losses else []

    def predict(self, x: torch.Tensor, n: int, est: torch.Tensor | None = None) -> torch.Tensor:
        return api.mlp_predict(self.params, x, n, est=est)


def relative_errors(estimate, exact) -> dict:
    """Mean, median, p90 and p99 of |estimate - exact| / exact."""
    e = np.asarray(estimate, dtype=np.float64)
    s = np.asarray(exact, dtype=np.float64)
    r = np.abs(e - s) / s
    return {"mean": float(r.mean()), "median": float(np.median(r)),
            "p90": float(np.percentile(r, 90)), "p99": float(np.percentile(r, 99))}
