"""Host model of the row-OR kernel's skip rules (no device): replays the
binary-op schedule slice by slice, keeping per row and slice a "row slice is
all ones" flag and a "row slice is all zero" flag, and counts the row words
the kernel must load and store.  A full operand makes the result full without
loads; a zero operand is not loaded; a full result into a full row and a zero
result into a zero row are not stored.  Zero flags start set on every real
row except the slice's own nodes (the identity) and unknown on scratch rows,
and are used in the zero phase (the levels before the one at which the ops
so far reach n), while some real row of the slice is still zero.  A slice stops
at the first level that starts with every real row full and whose index within
its launch (the zero phase is a launch of its own) is a multiple of 3.  The
matrix it ends
with must be the plain recurrence's; the counts are what the kernel's own
counters must report for the same slice width."""
import numpy as np

import oracle

SCR = 0x80000000
NOROW = 0xFFFFFFFF


def replay(n, sch, slice_words, saturation=True, zero=True):
    nw = oracle.words(n)
    ns = (nw + slice_words - 1) // slice_words
    pad = ns * slice_words
    nscr = sch["stats"]["scratch_rows"] + 1
    R = np.zeros((n + nscr, pad), dtype=np.uint64)
    R[:n, :nw] = oracle.from_dense(np.eye(n, dtype=bool))
    full = np.zeros(pad, dtype=np.uint64)
    full[:nw] = np.uint64(0xFFFFFFFFFFFFFFFF)
    if n % 64:
        full[nw - 1] = np.uint64((1 << (n % 64)) - 1)
    valid = np.minimum(slice_words, nw - np.arange(ns) * slice_words)  # words per slice
    flag = np.zeros((n + nscr, ns), dtype=bool)
    if saturation and (n - 1) % (64 * slice_words) == 0:
        flag[n - 1, (n - 1) // (64 * slice_words)] = True  # a one-column slice
    zflag = np.zeros((n + nscr, ns), dtype=bool)
    if saturation and zero:
        zflag[:n] = True
        zflag[np.arange(n), np.arange(n) // (64 * slice_words)] = False
    alive = np.ones(ns, dtype=bool)
    lv, ops = sch["lvl_op"], sch["ops"].astype(np.int64)
    L = sch["stats"]["op_levels"]
    zero_levels = int(np.searchsorted(lv[:L], n, side="left")) if (saturation and zero) else 0
    fullS = full.reshape(ns, slice_words)
    loads = stores = 0

    def idx(x):
        x = x.copy()
        sc = (x & SCR) != 0
        x[sc] = n + (x[sc] & 0x7FFFFFFF)
        return x

    for l in range(sch["stats"]["op_levels"]):
        # a slice stops only at a level that is a multiple of 3 within its
        # launch (the zero phase is a launch of its own)
        rel = l - zero_levels if 0 < zero_levels <= l else l
        if saturation and rel % 3 == 0:
            alive &= ~flag[:n].all(axis=0)
        live = valid * alive
        O = ops[lv[l]:lv[l + 1]]
        a, b = idx(O[:, 0]), idx(O[:, 1])
        zon = zflag[:n].any(axis=0) & (l < zero_levels)  # per slice, fixed for the level
        skip = (flag[a] | flag[b]) if saturation else np.zeros((O.shape[0], ns), bool)
        zx, zy = zflag[a] & zon[None], zflag[b] & zon[None]
        loads += int((live[None, :] * (~skip & ~zx)).sum() + (live[None, :] * (~skip & ~zy)).sum())
        r = (R[a] | R[b]).reshape(-1, ns, slice_words)
        r = np.where(skip[:, :, None], fullS[None], r)
        rf = (r == fullS[None]).all(axis=2)
        rz = (r == 0).all(axis=2) & zon[None]
        writes = []
        for col in (2, 3):
            keep = O[:, col] != NOROW
            d = idx(O[keep, col])
            if saturation:
                st = ~(rf[keep] & flag[d]) & ~(rz[keep] & zflag[d] & zon[None])
            else:
                st = np.ones((d.shape[0], ns), bool)
            stores += int((live[None, :] * st).sum())
            writes.append((d, r[keep], rf[keep], rz[keep]))
        cols = np.repeat(alive, slice_words)
        for d, rr, ff, zz in writes:
            R[np.ix_(d, cols)] = rr.reshape(-1, pad)[:, cols]
            flag[np.ix_(d, alive)] = ff[:, alive]
            upd = alive & zon
            zflag[np.ix_(d, upd)] = zz[:, upd]
    return R[:n, :nw], loads, stores


FWD = 0x40000000


def fwd_traffic(n, sch):
    """Row words the plain kernel loads and stores on the forwarded schedule:
    operands without the forwarding bit are loaded, destinations without the
    no-store bit are stored, each over every word of the row."""
    nw = oracle.words(n)
    fo = sch["fwd_ops"].astype(np.int64)
    cold = int(((fo[:, :2] & FWD) == 0).sum())
    dst = fo[:, 2:]
    stored = int(((dst != NOROW) & ((dst & FWD) == 0)).sum())  # FWD is the no-store bit here
    return cold * nw, stored * nw
