"""Python binding of the C ABI: host arrays are numpy, device buffers are torch
tensors on a HIP device, the stream is torch's current stream.  Argument
marshalling only; every step of the computation runs in the library."""
from __future__ import annotations

import atexit
import ctypes

import numpy as np
import torch

from ._lib import (DIRECTED, FORWARD, KERNELS, TIES_SEQUENTIAL, PlanStats, StreamStats, TNError,
                   check, lib)

__all__ = ["Context", "Plan", "Online", "FORWARD", "hll_build", "build_component_matrix_streamed",
           "hash_build_proxies", "Batch", "hash_compress", "recombine", "MLP_PARAMS", "mlp_init", "mlp_features", "mlp_forward", "mlp_predict", "mlp_train_step", "mlp_train_step_noalloc", "build_component_matrix_batched", "host_schedule", "DIRECTED", "TIES_SEQUENTIAL", "TNError", "words",
           "build_component_matrix", "component_sizes", "get_context"]


def words(n: int) -> int:
    return (int(n) + 63) // 64


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _dp(t: torch.Tensor | None):
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("device buffer expected")
    if not t.is_contiguous():
        raise ValueError("contiguous device buffer expected")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context on one device, enqueuing on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        check(lib.tn_create(self.device, ctypes.c_void_p(self._stream()), ctypes.byref(h)))
        self.h = h

    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def bind_stream(self):
        """Points the context at torch's current stream (call before enqueuing)."""
        check(lib.tn_set_stream(self.h, ctypes.c_void_p(self._stream())))
        return self.h

    def sync(self):
        check(lib.tn_sync(self.h))

    def profile(self, enable: bool = True):
        """Times every kernel this context launches with HIP events on its stream."""
        check(lib.tn_profile_enable(self.h, int(bool(enable))))

    def saturation(self, enable: bool = True):
        """Skips the row traffic saturated rows make redundant (on by default)."""
        check(lib.tn_set_saturation(self.h, int(bool(enable))))

    def last_traffic(self) -> tuple[int, int]:
        """(row words loaded, row words stored) by the last plan execution (waits)."""
        w = np.zeros(2, dtype=np.uint64)
        check(lib.tn_plan_last_traffic(self.h, _hp(w)))
        return int(w[0]), int(w[1])

    def profile_take(self, cap: int = 1 << 16):
        """[(kernel name, ms)] in launch order since the last take (waits for the stream)."""
        ids = np.zeros(cap, dtype=np.int32)
        ms = np.zeros(cap, dtype=np.float32)
        k = lib.tn_profile_take(self.h, _hp(ids), _hp(ms), cap)
        if k < 0:
            check(k)
        return [(KERNELS.get(int(i), str(int(i))), float(x)) for i, x in zip(ids[:k], ms[:k])]

    def close(self):
        if getattr(self, "h", None):
            lib.tn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def _close_contexts():
    """Destroys every context at interpreter exit, first thing: atexit
    handlers run before modules are torn down, while torch's streams and the
    HIP runtime are still alive (a context's destruction waits for its
    stream and frees its device scratch and pinned host staging)."""
    for c in list(_contexts.values()):
        try:
            c.close()
        except Exception:
            pass
    _contexts.clear()


atexit.register(_close_contexts)


def get_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    c = _contexts.get(device)
    if c is None:
        c = _contexts[device] = Context(device)
    return c


def _events(src, dst, t):
    src, dst, t = _host(src, np.uint32), _host(dst, np.uint32), _host(t, np.int64)
    if not (src.shape == dst.shape == t.shape) or src.ndim != 1:
        raise ValueError("src, dst, t must be 1-D arrays of one length")
    return src, dst, t


def alloc_matrix(n: int, ld: int | None = None, device: int | None = None, rows: int | None = None):
    """An (n, ld) int64 device tensor for a bit matrix of n columns; ld
    defaults to tn_recommended_ld(n) (rows on 128-byte lines)."""
    if device is None:
        device = torch.cuda.current_device()
    if ld is None:
        ld = int(lib.tn_recommended_ld(int(n)))
    return torch.empty((n if rows is None else rows, ld), dtype=torch.int64,
                       device=f"cuda:{device}")


class Plan:
    """The device-resident level schedule of one network (tn_plan_create)."""

    def __init__(self, n: int, src, dst, t, flags: int = 0, ctx: Context | None = None):
        self.ctx = ctx or get_context()
        self.n = int(n)
        src, dst, t = _events(src, dst, t)
        h = ctypes.c_void_p()
        check(lib.tn_plan_create(self.ctx.bind_stream(), self.n, src.shape[0], _hp(src),
                                 _hp(dst), _hp(t), int(flags), ctypes.byref(h)))
        self.h = h

    @property
    def stats(self) -> dict:
        s = PlanStats()
        check(lib.tn_plan_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def hll(self, node_hash, log2s: int, M: torch.Tensor | None = None,
            est: torch.Tensor | None = None):
        """The HyperLogLog stream on this plan's schedule (tn_hll_execute):
        (registers (n, 2^log2s) uint8, estimates (n,) float64), into M and
        est when given (a TN_HLL plan replays its captured level launches
        while M stays the same)."""
        dev = f"cuda:{self.ctx.device}"
        h = torch.as_tensor(np.ascontiguousarray(node_hash, dtype=np.uint64).view(np.int64)).to(dev)
        if h.shape != (self.n,):
            raise ValueError("node_hash must hold one value per node")
        if M is None:
            M = torch.empty((self.n, 1 << log2s), dtype=torch.uint8, device=dev)
        if est is None:
            est = torch.empty(self.n, dtype=torch.float64, device=dev)
        if (M.dtype != torch.uint8 or tuple(M.shape) != (self.n, 1 << log2s)
                or not M.is_contiguous() or M.device != torch.device(dev)):
            raise ValueError("M must be a contiguous uint8 (n, 2^log2s) tensor on the plan's device")
        if est.dtype != torch.float64 or tuple(est.shape) != (self.n,) or est.device != torch.device(dev):
            raise ValueError("est must be a float64 (n,) tensor on the plan's device")
        check(lib.tn_hll_execute(self.ctx.bind_stream(), self.h, int(log2s), _dp(h), _dp(M),
                                 _dp(est)))
        return M, est

    def execute(self, C: torch.Tensor | None = None, slice_words: int = 0) -> torch.Tensor:
        if C is None:
            C = alloc_matrix(self.n, device=self.ctx.device)
        if C.dtype != torch.int64 or C.dim() != 2 or C.shape[0] != self.n:
            raise ValueError("C must be an int64 (n, ld) device tensor")
        check(lib.tn_plan_execute(self.ctx.bind_stream(), self.h, _dp(C), C.stride(0),
                                  int(slice_words)))
        return C

    def execute_sizes(self, C: torch.Tensor | None = None, slice_words: int = 0,
                      out: torch.Tensor | None = None, inn: torch.Tensor | None = None):
        """execute(), then (out_sizes, in_sizes) from the matrix and the slice
        state the execution left: (C, out, inn), int32 device tensors."""
        if C is None:
            C = alloc_matrix(self.n, device=self.ctx.device)
        if C.dtype != torch.int64 or C.dim() != 2 or C.shape[0] != self.n:
            raise ValueError("C must be an int64 (n, ld) device tensor")
        dev = C.device
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=dev)
        if inn is None:
            inn = torch.empty(self.n, dtype=torch.int32, device=dev)
        for a in (out, inn):
            if a.dtype != torch.int32 or a.numel() != self.n or not a.is_contiguous():
                raise ValueError("out and inn must be contiguous int32 tensors of n entries")
        check(lib.tn_plan_execute_sizes(self.ctx.bind_stream(), self.h, _dp(C), C.stride(0),
                                        int(slice_words), _dp(out), _dp(inn)))
        return C, out, inn

    def close(self):
        if getattr(self, "h", None):
            lib.tn_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_component_matrix(n: int, src, dst, t, flags: int = 0, C: torch.Tensor | None = None,
                           ctx: Context | None = None) -> torch.Tensor:
    """Reverse-time component matrix: row u = out-component of u (int64 view of uint64 words)."""
    ctx = ctx or get_context()
    src, dst, t = _events(src, dst, t)
    if C is None:
        C = alloc_matrix(n, device=ctx.device)
    check(lib.tn_build_component_matrix(ctx.bind_stream(), int(n), src.shape[0], _hp(src),
                                        _hp(dst), _hp(t), int(flags), _dp(C), C.stride(0)))
    return C


def build_component_matrix_streamed(n: int, src, dst, t, flags: int = 0,
                                    C: torch.Tensor | None = None, chunk_events: int = 0,
                                    ctx: Context | None = None):
    """Streamed one-shot build (tn_build_component_matrix_streamed): returns
    (C, stats) once C is complete."""
    ctx = ctx or get_context()
    src, dst, t = _events(src, dst, t)
    if C is None:
        C = alloc_matrix(n, device=ctx.device)
    st = StreamStats()
    check(lib.tn_build_component_matrix_streamed(ctx.bind_stream(), int(n), src.shape[0],
                                                 _hp(src), _hp(dst), _hp(t), int(flags), _dp(C),
                                                 C.stride(0), int(chunk_events),
                                                 ctypes.byref(st)))
    return C, st.as_dict()


def hll_build(n: int, src, dst, t, node_hash, log2s: int, flags: int = 0,
              ctx: Context | None = None):
    """HyperLogLog stream (tn_hll_build): returns (registers (n, 2^log2s)
    uint8, estimates (n,) float64) on the device."""
    ctx = ctx or get_context()
    src, dst, t = _events(src, dst, t)
    dev = f"cuda:{ctx.device}"
    h = torch.as_tensor(np.ascontiguousarray(node_hash, dtype=np.uint64).view(np.int64)).to(dev)
    if h.shape != (n,):
        raise ValueError("node_hash must hold one value per node")
    M = torch.empty((n, 1 << log2s), dtype=torch.uint8, device=dev)
    est = torch.empty(n, dtype=torch.float64, device=dev)
    check(lib.tn_hll_build(ctx.bind_stream(), int(n), src.shape[0], _hp(src), _hp(dst), _hp(t),
                           int(flags), int(log2s), _dp(h), _dp(M), _dp(est)))
    return M, est


class Online:
    """A live component matrix that takes batches of events (tn_online_*).
    With FORWARD in flags the batches come in time order and rows are
    in-components; otherwise they come in reverse time order and rows are
    out-components."""

    def __init__(self, n: int, flags: int = 0, C: torch.Tensor | None = None,
                 ctx: Context | None = None):
        self.ctx = ctx or get_context()
        self.n = int(n)
        self.C = C if C is not None else alloc_matrix(self.n, device=self.ctx.device)
        h = ctypes.c_void_p()
        check(lib.tn_online_create(self.ctx.bind_stream(), self.n, int(flags), _dp(self.C),
                                   self.C.stride(0), ctypes.byref(h)))
        self.h = h

    def insert(self, src, dst, t, chunk_events: int = 0) -> dict:
        src, dst, t = _events(src, dst, t)
        st = StreamStats()
        check(lib.tn_online_insert(self.ctx.bind_stream(), self.h, src.shape[0], _hp(src),
                                   _hp(dst), _hp(t), int(chunk_events), ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib.tn_online_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def component_sizes(C: torch.Tensor, n: int, out: bool = True, inn: bool = True,
                    ctx: Context | None = None):
    """(out_sizes, in_sizes) int32 device tensors (None where not asked for)."""
    ctx = ctx or get_context()
    o = torch.empty(n, dtype=torch.int32, device=C.device) if out else None
    i = torch.empty(n, dtype=torch.int32, device=C.device) if inn else None
    check(lib.tn_component_sizes(ctx.bind_stream(), int(n), _dp(C), C.stride(0), _dp(o), _dp(i)))
    return o, i


def host_schedule(n: int, src, dst, t, flags: int = 0, fwd_level_cap: int = 0) -> dict:
    """The level schedule the planner builds (host only, no device), as numpy arrays;
    ``fwd_lvl``/``fwd_ops`` are its forwarded form with levels of at most
    ``fwd_level_cap`` ops (0: 768, the form the kernels run)."""
    src, dst, t = _events(src, dst, t)
    h = ctypes.c_void_p()
    check(lib.tn_schedule_build(int(n), src.shape[0], _hp(src), _hp(dst), _hp(t), int(flags),
                                ctypes.byref(h)))
    try:
        st = PlanStats()
        ptrs = [ctypes.c_void_p() for _ in range(6)]
        check(lib.tn_schedule_arrays(h, ctypes.byref(st), *[ctypes.byref(p) for p in ptrs]))
        L, P, G = st.levels, st.pairs, st.gathers

        def arr(p, k):
            if k == 0 or not p.value:
                return np.zeros(0, dtype=np.uint32)
            return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint32)),
                                         shape=(k,)).copy()
        optr = [ctypes.c_void_p() for _ in range(2)]
        check(lib.tn_schedule_op_arrays(h, ctypes.byref(optr[0]), ctypes.byref(optr[1])))
        Lo, nops = st.op_levels, st.ops
        lvl_pair = arr(ptrs[0], L + 1)
        lvl_gat = arr(ptrs[1], L + 1)
        gat_ptr = arr(ptrs[4], G + 1)
        out = dict(stats=st.as_dict(), lvl_pair=lvl_pair, lvl_gat=lvl_gat,
                   pairs=arr(ptrs[2], 2 * P).reshape(P, 2), gat_tgt=arr(ptrs[3], G),
                   gat_ptr=gat_ptr, gat_src=arr(ptrs[5], int(gat_ptr[-1]) if G else 0),
                   lvl_op=arr(optr[0], Lo + 1), ops=arr(optr[1], 4 * nops).reshape(nops, 4))
        fl = ctypes.c_uint32()
        fptr = [ctypes.c_void_p() for _ in range(2)]
        check(lib.tn_schedule_fwd_arrays(h, int(fwd_level_cap), ctypes.byref(fl),
                                         ctypes.byref(fptr[0]), ctypes.byref(fptr[1])))
        out["fwd_lvl"] = arr(fptr[0], fl.value + 1)
        out["fwd_ops"] = arr(fptr[1], 4 * nops).reshape(nops, 4)
    finally:
        lib.tn_schedule_destroy(h)
    return out


class Batch:
    """Schedules of many networks built in one persistent launch (tn_batch_create).

    ``nets`` is a sequence of (n, src, dst, t).  The first execute() tunes the
    tile shape on the device and captures the launch in a HIP graph."""

    def __init__(self, nets, flags: int = 0, ctx: Context | None = None, _handle=None):
        self.ctx = ctx or get_context()
        if _handle is not None:
            self.h = _handle
            self.ns = [int(x) for x in nets]
            return
        evs = [_events(s, d, t) for (_, s, d, t) in nets]
        self.ns = [int(n) for (n, _, _, _) in nets]
        B = len(nets)
        n_arr = np.asarray(self.ns, dtype=np.uint32)
        m_arr = np.asarray([e[0].shape[0] for e in evs], dtype=np.int64)
        ptr = lambda k: (ctypes.c_void_p * B)(*[e[k].ctypes.data for e in evs])
        self._keep = evs
        h = ctypes.c_void_p()
        check(lib.tn_batch_create(self.ctx.bind_stream(), B, _hp(n_arr), _hp(m_arr), ptr(0),
                                  ptr(1), ptr(2), int(flags), ctypes.byref(h)))
        self._keep = None
        self.h = h

    def __len__(self):
        return len(self.ns)

    def stats(self):
        B = len(self.ns)
        st = (PlanStats * B)()
        tiles = ctypes.c_int64()
        lds = ctypes.c_int64()
        check(lib.tn_batch_get_stats(self.h, st, ctypes.byref(tiles), ctypes.byref(lds)))
        return [s.as_dict() for s in st], int(tiles.value), int(lds.value)

    def shape(self) -> dict:
        """The launch shape (the tuned one after the first execute())."""
        v = (ctypes.c_int64 * 6)()
        check(lib.tn_batch_get_shape(self.h, v))
        keys = ("threads", "lds_bytes", "per_cu", "grid", "halvings", "global_width")
        return dict(zip(keys, (int(x) for x in v)))

    def alloc(self):
        return [alloc_matrix(n, device=self.ctx.device) for n in self.ns]

    def execute(self, Cs=None):
        if Cs is None:
            Cs = self.alloc()
        B = len(self.ns)
        if len(Cs) != B:
            raise ValueError("one matrix per network expected")
        for C, n in zip(Cs, self.ns):
            if C.dtype != torch.int64 or C.dim() != 2 or C.shape[0] != n or not C.is_contiguous():
                raise ValueError("C must be contiguous int64 (n, ld) device tensors")
        cp = (ctypes.c_void_p * B)(*[C.data_ptr() for C in Cs])
        ld = np.asarray([C.stride(0) for C in Cs], dtype=np.int64)
        check(lib.tn_batch_execute(self.ctx.bind_stream(), self.h, cp, _hp(ld)))
        return Cs

    def close(self):
        if getattr(self, "h", None):
            lib.tn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_component_matrix_batched(nets, flags: int = 0, Cs=None, ctx: Context | None = None):
    """One call: plan, tune, build and free a batch; returns the matrices."""
    ctx = ctx or get_context()
    evs = [_events(s, d, t) for (_, s, d, t) in nets]
    ns = [int(n) for (n, _, _, _) in nets]
    B = len(nets)
    if Cs is None:
        Cs = [alloc_matrix(n, device=ctx.device) for n in ns]
    n_arr = np.asarray(ns, dtype=np.uint32)
    m_arr = np.asarray([e[0].shape[0] for e in evs], dtype=np.int64)
    ptr = lambda k: (ctypes.c_void_p * B)(*[e[k].ctypes.data for e in evs])
    cp = (ctypes.c_void_p * B)(*[C.data_ptr() for C in Cs])
    ld = np.asarray([C.stride(0) for C in Cs], dtype=np.int64)
    check(lib.tn_build_component_matrix_batched(ctx.bind_stream(), B, _hp(n_arr), _hp(m_arr),
                                                ptr(0), ptr(1), ptr(2), int(flags), cp, _hp(ld)))
    return Cs


def hash_compress(n: int, src, dst, t, coeffs, K: int, flags: int = 0,
                  ctx: Context | None = None):
    """Network hashing (Sec. 4.1): returns (bucket (H, n) int32 view of uint32,
    count (H, K) int32, proxies Batch of H networks on K super-nodes).
    ``coeffs`` is the (H, 3, order) uint64 random table of the hash family."""
    ctx = ctx or get_context()
    src, dst, t = _events(src, dst, t)
    A = np.ascontiguousarray(coeffs, dtype=np.uint64)
    if A.ndim != 3 or A.shape[1] != 3:
        raise ValueError("coeffs must have shape (H, 3, order)")
    H, _, order = A.shape
    dev = f"cuda:{ctx.device}"
    bucket = torch.empty((H, n), dtype=torch.int32, device=dev)
    count = torch.empty((H, K), dtype=torch.int32, device=dev)
    h = ctypes.c_void_p()
    check(lib.tn_hash_compress(ctx.bind_stream(), int(n), src.shape[0], _hp(src), _hp(dst), _hp(t),
                               int(flags), H, int(K), _hp(A), order, _dp(bucket), _dp(count),
                               ctypes.byref(h)))
    return bucket, count, Batch([K] * H, ctx=ctx, _handle=h)


def hash_build_proxies(n: int, src, dst, t, coeffs, K: int, flags: int = 0,
                       chunk_events: int = 0, P: torch.Tensor | None = None,
                       ctx: Context | None = None):
    """Hashing plus the streamed build of all H proxies (tn_hash_build_proxies):
    returns (bucket (H, n), count (H, K), P (H, K, ldK) int64, stats)."""
    ctx = ctx or get_context()
    src, dst, t = _events(src, dst, t)
    A = np.ascontiguousarray(coeffs, dtype=np.uint64)
    if A.ndim != 3 or A.shape[1] != 3:
        raise ValueError("coeffs must have shape (H, 3, order)")
    H, _, order = A.shape
    dev = f"cuda:{ctx.device}"
    bucket = torch.empty((H, n), dtype=torch.int32, device=dev)
    count = torch.empty((H, K), dtype=torch.int32, device=dev)
    if P is None:
        P = torch.empty((H, K, words(K)), dtype=torch.int64, device=dev)
    if P.dim() != 3 or not P.is_contiguous() or P.shape[0] != H or P.shape[1] != K:
        raise ValueError("P must be a contiguous (H, K, ldK) tensor")
    st = StreamStats()
    check(lib.tn_hash_build_proxies(ctx.bind_stream(), int(n), src.shape[0], _hp(src), _hp(dst),
                                    _hp(t), int(flags), H, int(K), _hp(A), order, _dp(bucket),
                                    _dp(count), _dp(P), P.shape[2], int(chunk_events),
                                    ctypes.byref(st)))
    return bucket, count, P, st.as_dict()


def recombine(P: torch.Tensor, bucket: torch.Tensor, count: torch.Tensor, n: int,
              lifted: bool = True, ctx: Context | None = None):
    """Fusion (Sec. 4.2): |estimated OC(u)| for every node and, optionally, the
    per-hash lifted sizes.  P is (H, K, ldK) int64 on the device."""
    ctx = ctx or get_context()
    if P.dim() != 3 or not P.is_contiguous():
        raise ValueError("P must be a contiguous (H, K, ldK) tensor")
    H, K, ldK = P.shape
    est = torch.empty(n, dtype=torch.int32, device=P.device)
    lif = torch.empty((H, n), dtype=torch.int32, device=P.device) if lifted else None
    check(lib.tn_recombine(ctx.bind_stream(), int(n), H, K, _dp(P), ldK, _dp(bucket), _dp(count),
                           _dp(est), _dp(lif)))
    return est, lif


MLP_PARAMS = 5313


def mlp_init(seed: int, params: torch.Tensor | None = None,
             ctx: Context | None = None) -> torch.Tensor:
    """Seeded He-uniform initial parameters on the device (tn_mlp_init):
    (MLP_PARAMS,) float32."""
    ctx = ctx or get_context()
    if params is None:
        params = torch.empty(MLP_PARAMS, dtype=torch.float32, device=f"cuda:{ctx.device}")
    if params.dtype != torch.float32 or params.numel() != MLP_PARAMS or not params.is_contiguous():
        raise ValueError(f"params must be a contiguous float32 tensor of {MLP_PARAMS} values")
    check(lib.tn_mlp_init(ctx.bind_stream(), int(seed) & ((1 << 64) - 1), _dp(params)))
    return params


def mlp_features(lifted: torch.Tensor, n: int, ctx: Context | None = None) -> torch.Tensor:
    """x[u, j] = ln(lifted[j, u] / n) for H = 16 hashes: (n, 16) float32."""
    ctx = ctx or get_context()
    H = lifted.shape[0]
    x = torch.empty((n, H), dtype=torch.float32, device=lifted.device)
    check(lib.tn_mlp_features(ctx.bind_stream(), int(n), H, _dp(lifted), _dp(x)))
    return x


def mlp_forward(params: torch.Tensor, x: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    ctx = ctx or get_context()
    N = x.shape[0]
    yhat = torch.empty(N, dtype=torch.float32, device=x.device)
    check(lib.tn_mlp_forward(ctx.bind_stream(), _dp(params), _dp(x), N, _dp(yhat)))
    return yhat


def mlp_train_step(params, adam_m, adam_v, step: int, x, y, idx=None, lr: float = 1e-3,
                   want_grad: bool = False, ctx: Context | None = None):
    """One Adam step in place; returns (loss (1,) tensor, gradient or None)."""
    ctx = ctx or get_context()
    N = x.shape[0] if idx is None else idx.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device) if want_grad else None
    check(lib.tn_mlp_train_step(ctx.bind_stream(), _dp(params), _dp(adam_m), _dp(adam_v),
                                int(step), _dp(x), _dp(y), _dp(idx), N, float(lr), _dp(loss),
                                _dp(grad)))
    return loss, grad


def mlp_train_step_noalloc(params, adam_m, adam_v, step: int, x, y, idx=None, lr: float = 1e-3,
                           loss=None, grad=None, ctx: Context | None = None):
    """tn_mlp_train_step_noalloc: the same Adam step with no device allocation
    inside the call (at most 16384 samples); loss and grad, if given, are
    caller-owned outputs.  Returns (loss, grad)."""
    ctx = ctx or get_context()
    N = x.shape[0] if idx is None else idx.shape[0]
    check(lib.tn_mlp_train_step_noalloc(ctx.bind_stream(), _dp(params), _dp(adam_m), _dp(adam_v),
                                        int(step), _dp(x), _dp(y), _dp(idx), N, float(lr),
                                        _dp(loss), _dp(grad)))
    return loss, grad


def mlp_predict(params, x, n: int, est=None, ctx: Context | None = None) -> torch.Tensor:
    """Size estimates n * exp(MLP(x)) clamped to [1, est] (or [1, n])."""
    ctx = ctx or get_context()
    N = x.shape[0]
    sizes = torch.empty(N, dtype=torch.float32, device=x.device)
    check(lib.tn_mlp_predict(ctx.bind_stream(), _dp(params), _dp(x), N, int(n), _dp(est),
                             _dp(sizes)))
    return sizes
