"""CPU oracle: plain, slow, obviously correct reference of what the GPU path computes.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  The library's product path never
imports, links or calls it, and the two share no code: the only common module
is ``tn_inputs``, which draws random inputs and holds none of the method's
arithmetic.

Contents
--------
* ``tn_oracle.c`` (built to ``liboracle.so`` with gcc): the reverse-time
  component matrix (Sec. 3.4 with the adjacency rule of Sec. 2.1), forward
  Algorithm 1 (Sec. 3.1), row / column popcounts (Sec. 3.1, Eq. 1), the hash
  family (Sec. 4.1) and the recombination (Sec. 4.2).
* ``si.py``: deterministic SI simulation from every node (Sec. 1), the brute
  force that pins the matrix.
* ``mlp.py``: float64 forward / backward / Adam of the learned combiner.
* ``hll.py``: the HyperLogLog variant of the stream (Sec. 3.4): registers,
  register-wise max per time step, and the estimator.

Every matrix routine returns ``uint64`` arrays with node ``w`` at bit
``w & 63`` of word ``w >> 6``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MERSENNE61 = (1 << 61) - 1


def build() -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u32, i64, i32, u64 = ctypes.c_uint32, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64
    for name in ("tno_reverse_matrix", "tno_forward_matrix"):
        f = getattr(lib, name)
        f.argtypes = [u32, i64, P, P, P, i32, i32, i64, i64, P]
        f.restype = i32
    lib.tno_row_counts.argtypes = [u32, i64, P, P]
    lib.tno_col_counts.argtypes = [u32, i64, P, P]
    lib.tno_multaddmod.argtypes = [u64, u64, u64]
    lib.tno_multaddmod.restype = u64
    lib.tno_poly.argtypes = [P, i32, u64]
    lib.tno_poly.restype = u64
    lib.tno_hash_raw.argtypes = [P, i32, u64]
    lib.tno_hash_raw.restype = u64
    lib.tno_hash_nodes.argtypes = [u32, u32, P, i32, u32, P]
    lib.tno_recombine.argtypes = [u32, u32, u32, i64, P, P, i64, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def words(n: int) -> int:
    return (n + 63) // 64


def _events(src, dst, t):
    return (np.ascontiguousarray(src, dtype=np.uint32),
            np.ascontiguousarray(dst, dtype=np.uint32),
            np.ascontiguousarray(t, dtype=np.int64))


def _matrix(fn, n, src, dst, t, directed, sequential, w0, nw):
    src, dst, t = _events(src, dst, t)
    if nw is None:
        nw = words(n) - w0
    M = np.empty((n, nw), dtype=np.uint64)
    rc = fn(n, src.shape[0], _ptr(src), _ptr(dst), _ptr(t), int(directed),
            int(sequential), w0, nw, _ptr(M))
    if rc == -2:
        raise ValueError("node id out of range")
    if rc == -3:
        raise ValueError("events are not in chronological order")
    if rc != 0:
        raise RuntimeError(f"oracle failed: {rc}")
    return M


def reverse_matrix(n, src, dst, t, directed=False, sequential=False, w0=0, nw=None):
    """Reverse-time component matrix C (row u = out-component of u), words [w0, w0+nw)."""
    return _matrix(_load().tno_reverse_matrix, n, src, dst, t, directed, sequential, w0, nw)


def forward_matrix(n, src, dst, t, directed=False, sequential=False, w0=0, nw=None):
    """Algorithm 1's matrix S (row x = in-component of x), words [w0, w0+nw)."""
    return _matrix(_load().tno_forward_matrix, n, src, dst, t, directed, sequential, w0, nw)


def row_counts(M: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.uint64)
    out = np.empty(M.shape[0], dtype=np.int64)
    _load().tno_row_counts(M.shape[0], M.shape[1], _ptr(M), _ptr(out))
    return out


def col_counts(M: np.ndarray, n_cols: int | None = None) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.uint64)
    col = np.empty(64 * M.shape[1], dtype=np.int64)
    _load().tno_col_counts(M.shape[0], M.shape[1], _ptr(M), _ptr(col))
    return col if n_cols is None else col[:n_cols]


def sizes(M: np.ndarray, n: int):
    """(out, in) component sizes of a full reverse-time matrix (Sec. 3.1)."""
    return row_counts(M), col_counts(M, n)


def to_dense(M: np.ndarray, n: int) -> np.ndarray:
    """Unpack bit rows into a bool n x n array (column b = node b)."""
    bits = np.unpackbits(M.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :n].astype(bool)


def from_dense(D: np.ndarray) -> np.ndarray:
    n_rows, n = D.shape
    nw = words(n)
    pad = np.zeros((n_rows, nw * 64), dtype=np.uint8)
    pad[:, :n] = D
    return np.packbits(pad, axis=1, bitorder="little").view(np.uint64).reshape(n_rows, nw)


def multaddmod(x: int, acc: int, a: int) -> int:
    return int(_load().tno_multaddmod(x, acc, a))


def poly(Ai, x: int) -> int:
    Ai = np.ascontiguousarray(Ai, dtype=np.uint64)
    return int(_load().tno_poly(_ptr(Ai), Ai.shape[0], x))


def hash_raw(A, u: int) -> int:
    """Un-reduced hash value of node u for one coefficient table A (3 x order)."""
    A = np.ascontiguousarray(A, dtype=np.uint64)
    return int(_load().tno_hash_raw(_ptr(A), A.shape[1], u))


def hash_nodes(n: int, A, K: int) -> np.ndarray:
    """bucket[j, u] = h_j(u) mod K for the H coefficient tables A (H x 3 x order)."""
    A = np.ascontiguousarray(A, dtype=np.uint64)
    H, _, order = A.shape
    out = np.empty((H, n), dtype=np.uint32)
    _load().tno_hash_nodes(n, H, _ptr(A), order, K, _ptr(out))
    return out


def bucket_counts(bucket: np.ndarray, K: int) -> np.ndarray:
    """count[j, r] = |h_j^{-1}(r)| (Sec. 4.2, inverse of a hash)."""
    H, n = bucket.shape
    out = np.zeros((H, K), dtype=np.int64)
    for j in range(H):
        for u in range(n):
            out[j, bucket[j, u]] += 1
    return out


def proxies(K: int, src, dst, t, bucket: np.ndarray, directed=False, sequential=False):
    """Component matrices of the hashed networks: events (h_j(u), h_j(v), t) on K nodes."""
    src, dst, t = _events(src, dst, t)
    out = []
    for j in range(bucket.shape[0]):
        hs = bucket[j][src]
        hd = bucket[j][dst]
        out.append(reverse_matrix(K, hs, hd, t, directed, sequential))
    return np.stack(out)


def recombine(n: int, P: np.ndarray, bucket: np.ndarray, us=None):
    """|estimated OC(u)| and per-hash lifted sizes for the sources ``us`` (default all)."""
    P = np.ascontiguousarray(P, dtype=np.uint64)
    H, K, ldK = P.shape
    bucket = np.ascontiguousarray(bucket, dtype=np.uint32)
    if us is None:
        us = np.arange(n, dtype=np.uint32)
    us = np.ascontiguousarray(us, dtype=np.uint32)
    est = np.empty(us.shape[0], dtype=np.int64)
    lifted = np.empty((H, us.shape[0]), dtype=np.int64)
    _load().tno_recombine(n, H, K, ldK, _ptr(P), _ptr(bucket), us.shape[0], _ptr(us),
                          _ptr(est), _ptr(lifted))
    return est, lifted
