"""Host model of the row-OR kernel's saturation rule (no device): replays the
binary-op schedule slice by slice, keeping one "row slice is all ones" flag per
row and slice, and counts the row words the kernel must load and store.  A
slice stops at the first level that starts with every real row full.  The
matrix it ends with must be the plain recurrence's; the counts are what the
kernel's own counters must report for the same slice width."""
import numpy as np

import oracle

SCR = 0x80000000
NOROW = 0xFFFFFFFF


def replay(n, sch, slice_words, saturation=True):
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
    alive = np.ones(ns, dtype=bool)
    lv, ops = sch["lvl_op"], sch["ops"].astype(np.int64)
    fullS = full.reshape(ns, slice_words)
    loads = stores = 0

    def idx(x):
        x = x.copy()
        sc = (x & SCR) != 0
        x[sc] = n + (x[sc] & 0x7FFFFFFF)
        return x

    for l in range(sch["stats"]["op_levels"]):
        if saturation:
            alive &= ~flag[:n].all(axis=0)
        live = valid * alive
        O = ops[lv[l]:lv[l + 1]]
        a, b = idx(O[:, 0]), idx(O[:, 1])
        skip = (flag[a] | flag[b]) if saturation else np.zeros((O.shape[0], ns), bool)
        loads += int(2 * (live[None, :] * ~skip).sum())
        r = (R[a] | R[b]).reshape(-1, ns, slice_words)
        r = np.where(skip[:, :, None], fullS[None], r)
        rf = (r == fullS[None]).all(axis=2)
        writes = []
        for col in (2, 3):
            keep = O[:, col] != NOROW
            d = idx(O[keep, col])
            st = ~(rf[keep] & flag[d]) if saturation else np.ones((d.shape[0], ns), bool)
            stores += int((live[None, :] * st).sum())
            writes.append((d, r[keep], rf[keep]))
        cols = np.repeat(alive, slice_words)
        for d, rr, ff in writes:
            R[np.ix_(d, cols)] = rr.reshape(-1, pad)[:, cols]
            flag[np.ix_(d, alive)] = ff[:, alive]
    return R[:n, :nw], loads, stores
