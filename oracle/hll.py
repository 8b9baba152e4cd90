"""HyperLogLog variant of the reverse-time stream (Sec. 3.4, last paragraph;
HyperLogLog itself, Sec. 2.2): plain numpy, slow, obviously correct.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every node starts with the HLL structure of the set {node}; for each time
step, in reverse time order (forward order for in-components), every node
touched at that step merges the structures of the nodes it receives from,
computed from the structures as they were before the step (Sec. 2.1: events
of one time step are not adjacent).  Merging two HLL structures is the
register-wise maximum, and it equals the structure of the union of the two
sets, which pins the stream (the registers of u must equal the registers of
u's exact out-component built from scratch).

The HLL structure follows Flajolet, Fusy, Gandouet and Meunier (2007):
s = 2^b registers; an element with 64-bit hash x goes to register j, the top
b bits of x, and that register keeps the maximum of rho, the 1-based position
of the leftmost 1 in the remaining 64 - b bits (64 - b + 1 if they are all
zero).  The raw estimate is alpha_s s^2 / sum_j 2^-M[j] with alpha_16 =
0.673, alpha_32 = 0.697, alpha_64 = 0.709 and alpha_s = 0.7213 / (1 + 1.079/s)
for s >= 128; when it is at most 5s/2 and V registers are zero, V > 0, the
estimate is s ln(s / V) (linear counting).  With 64-bit hashes no large-range
correction applies.  The element hashes are inputs (one uniform 64-bit word
per node), so no hash function is part of this module.
"""
from __future__ import annotations

import numpy as np


def register_of(x: int, b: int) -> tuple[int, int]:
    """(register index, rho) of one 64-bit hash value."""
    x = int(x) & ((1 << 64) - 1)
    j = x >> (64 - b)
    w = x & ((1 << (64 - b)) - 1)
    width = 64 - b
    if w == 0:
        rho = width + 1
    else:
        rho = width - w.bit_length() + 1  # leading zeros within the width, plus one
    return j, rho


def registers_of_set(hashes, b: int) -> np.ndarray:
    """HLL registers (uint8[2^b]) of the set whose elements hash to `hashes`."""
    M = np.zeros(1 << b, dtype=np.uint8)
    for x in np.asarray(hashes, dtype=np.uint64).tolist():
        j, rho = register_of(x, b)
        if rho > M[j]:
            M[j] = rho
    return M


def alpha(s: int) -> float:
    if s == 16:
        return 0.673
    if s == 32:
        return 0.697
    if s == 64:
        return 0.709
    return 0.7213 / (1.0 + 1.079 / s)


def estimate(M: np.ndarray) -> np.ndarray:
    """HLL size estimates (float64) of each row of registers M (rows x s)."""
    M = np.atleast_2d(np.asarray(M, dtype=np.int64))
    s = M.shape[1]
    Z = np.sum(np.ldexp(1.0, -M), axis=1)
    E = alpha(s) * s * s / Z
    V = np.sum(M == 0, axis=1)
    small = (E <= 2.5 * s) & (V > 0)
    E = E.copy()
    E[small] = s * np.log(s / V[small])
    return E


def stream_registers(n, src, dst, t, node_hash, b, directed=False, sequential=False,
                     forward=False) -> np.ndarray:
    """Registers (n x 2^b uint8) after the HLL stream over the events."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    m = src.shape[0]
    M = np.zeros((n, 1 << b), dtype=np.uint8)
    for u in range(n):
        j, rho = register_of(int(node_hash[u]), b)
        M[u, j] = rho
    # time-step groups [a, b) in processing order
    groups = []
    a = 0
    while a < m:
        e = a + 1
        if not sequential:
            while e < m and t[e] == t[a]:
                e += 1
        groups.append((a, e))
        a = e
    if not forward:
        groups.reverse()
    for a, e in groups:
        new = {}
        for k in range(a, e):
            x, y = int(src[k]), int(dst[k])
            to, frm = (y, x) if forward else (x, y)  # the row that receives
            new.setdefault(to, M[to].copy())
            new[to] = np.maximum(new[to], M[frm])
            if not directed:
                new.setdefault(frm, M[frm].copy())
                new[frm] = np.maximum(new[frm], M[to])
        for x, row in new.items():
            M[x] = row
    return M
