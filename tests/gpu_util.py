"""Helpers of the GPU tests (no oracle arithmetic)."""
import numpy as np
import torch


def host(C):
    """A device bit matrix (..., rows, ld) as uint64 host words, trimmed to
    ceil(rows / 64) words per row after checking that every padding word the
    library wrote is 0 (the layout contract of every matrix output)."""
    torch.cuda.synchronize()
    a = C.cpu().numpy().view(np.uint64)
    nw = (a.shape[-2] + 63) // 64
    assert not a[..., nw:].any(), "padding words are not 0"
    return a[..., :nw]
