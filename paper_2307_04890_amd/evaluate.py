"""Accuracy criteria of the hashing framework (Sec. 4.4, host side).

The paper compares the exact distribution of out-component sizes with the
one the hashing framework infers through the Earth-Mover (Wasserstein-1)
distance.  Between two one-dimensional empirical distributions it has a
closed form: the integral over x of |F(x) - G(x)|, F and G the two
empirical CDFs.  These helpers run on host arrays of sizes that the
library's kernels produced.
"""
from __future__ import annotations

import numpy as np


def emd_1d(a, b) -> float:
    """Wasserstein-1 distance between the empirical distributions of the
    samples a and b (any lengths): sum over the gaps of the merged sorted
    values of gap * |F_a - F_b| on that gap."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    b = np.sort(np.asarray(b, dtype=np.float64).ravel())
    if a.size == 0 or b.size == 0:
        raise ValueError("both samples must be non-empty")
    allv = np.sort(np.concatenate([a, b]))
    gaps = np.diff(allv)
    Fa = np.searchsorted(a, allv[:-1], side="right") / a.size
    Fb = np.searchsorted(b, allv[:-1], side="right") / b.size
    return float(np.sum(np.abs(Fa - Fb) * gaps))


def relative_memory(n: int, K: int, H: int) -> float:
    """Bytes of the H proxy matrices over the bytes of the exact matrix,
    both as bit matrices with rows padded to 64-bit words."""
    return H * K * ((K + 63) // 64) / (n * ((n + 63) // 64))
