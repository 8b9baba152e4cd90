"""Host planner (CPU, no device): the level schedule, replayed by a plain numpy
simulation of the kernels' per-level semantics, must give the oracle's matrix;
the items of every level must touch disjoint rows; bad input is rejected."""
import numpy as np
import pytest

import oracle
import paper_2307_04890_amd as tn
import tn_inputs as T

MASK = np.uint32(0x7FFFFFFF)
DIR = np.uint32(0x80000000)


def simulate(n, sch):
    """Apply a schedule level by level: pairs OR both rows (one for directed),
    gathers read all old rows of their level, then write."""
    nw = oracle.words(n)
    C = oracle.from_dense(np.eye(n, dtype=bool)) if n else np.zeros((0, nw), np.uint64)
    lp, lg = sch["lvl_pair"], sch["lvl_gat"]
    pairs, gt, gp, gs = sch["pairs"], sch["gat_tgt"], sch["gat_ptr"], sch["gat_src"]
    for l in range(sch["stats"]["levels"]):
        P = pairs[lp[l]:lp[l + 1]]
        u = P[:, 0].astype(np.int64)
        v = (P[:, 1] & MASK).astype(np.int64)
        sym = (P[:, 1] & DIR) == 0
        r = C[u] | C[v]
        new = [(int(gt[g]), np.bitwise_or.reduce(C[gs[gp[g]:gp[g + 1]].astype(np.int64)], axis=0))
               for g in range(lg[l], lg[l + 1])]
        C[u] = r
        C[v[sym]] = r[sym]
        for x, row in new:
            C[x] = row
    return C


NOROW = 0xFFFFFFFF
SCR = 0x80000000


def simulate_ops(n, sch):
    """Apply the binary-op form level by level: every op of a level reads
    the rows as they were before the level, then all writes happen."""
    nw = oracle.words(n)
    C = oracle.from_dense(np.eye(n, dtype=bool)) if n else np.zeros((0, nw), np.uint64)
    S = np.zeros((sch["stats"]["scratch_rows"] + 1, nw), dtype=np.uint64)
    lv, ops = sch["lvl_op"], sch["ops"].astype(np.int64)

    def get(ids):
        ids = np.asarray(ids, dtype=np.int64)
        out = np.empty((ids.shape[0], nw), dtype=np.uint64)
        sc = (ids & SCR) != 0
        out[~sc] = C[ids[~sc]]
        out[sc] = S[ids[sc] & 0x7FFFFFFF]
        return out

    def put(ids, vals):
        ids = np.asarray(ids, dtype=np.int64)
        keep = ids != NOROW
        ids, vals = ids[keep], vals[keep]
        sc = (ids & SCR) != 0
        C[ids[~sc]] = vals[~sc]
        S[ids[sc] & 0x7FFFFFFF] = vals[sc]

    for l in range(sch["stats"]["op_levels"]):
        O = ops[lv[l]:lv[l + 1]]
        r = get(O[:, 0]) | get(O[:, 1])
        put(O[:, 2], r)
        put(O[:, 3], r)
    return C


FWD = 0x40000000


def simulate_fwd(n, sch):
    """Apply the forwarded op form level by level as the plain kernel does:
    an operand with the forwarding bit is the result of that op of the level
    before (kept aside, never read from the matrix); any other operand is
    read from the matrix, which holds only the values actually stored; a
    destination with the bit is not stored."""
    nw = oracle.words(n)
    C = oracle.from_dense(np.eye(n, dtype=bool)) if n else np.zeros((0, nw), np.uint64)
    S = np.zeros((sch["stats"]["scratch_rows"] + 1, nw), dtype=np.uint64)
    lv, ops = sch["fwd_lvl"], sch["fwd_ops"].astype(np.int64)
    prev = np.zeros((0, nw), dtype=np.uint64)

    def row(i):
        return S[i & 0x7FFFFFFF] if i & SCR else C[i]

    for l in range(len(lv) - 1):
        O = ops[lv[l]:lv[l + 1]]
        assert O.shape[0] <= 768
        cur = np.empty((O.shape[0], nw), dtype=np.uint64)
        for j, (a, b, d1, d2) in enumerate(O):
            x = prev[a & 0x3FF] if (a & FWD) else row(a)
            y = prev[b & 0x3FF] if (b & FWD) else row(b)
            cur[j] = x | y
        for j, (a, b, d1, d2) in enumerate(O):
            for dd in (d1, d2):
                if dd == NOROW or (dd & FWD):
                    continue
                if dd & SCR:
                    S[dd & 0x7FFFFFFF] = cur[j]
                else:
                    C[dd] = cur[j]
        prev = cur
    return C


def check_ops_independent(sch):
    lv, ops = sch["lvl_op"], sch["ops"].astype(np.int64)
    for l in range(sch["stats"]["op_levels"]):
        O = ops[lv[l]:lv[l + 1]]
        assert 0 < O.shape[0] <= 1024, l
        writer = {}
        for i, (a, b, d1, d2) in enumerate(O):
            for d in (d1, d2):
                if d != NOROW:
                    assert d not in writer, (l, "two writes")
                    writer[d] = i
        for i, (a, b, _, _) in enumerate(O):
            for x in (a, b):
                assert writer.get(x, i) == i, (l, "read of a row another op writes")


def check_disjoint(n, sch):
    lp, lg = sch["lvl_pair"], sch["lvl_gat"]
    pairs, gt, gp, gs = sch["pairs"], sch["gat_tgt"], sch["gat_ptr"], sch["gat_src"]
    for l in range(sch["stats"]["levels"]):
        P = pairs[lp[l]:lp[l + 1]]
        pn = np.concatenate([P[:, 0], P[:, 1] & MASK])
        assert np.unique(pn).shape[0] == pn.shape[0], l
        tg = gt[lg[l]:lg[l + 1]]
        assert np.unique(tg).shape[0] == tg.shape[0], l
        gsrc = gs[gp[lg[l]]:gp[lg[l + 1]]] if lg[l + 1] > lg[l] else np.zeros(0, np.uint32)
        assert not np.intersect1d(pn, np.concatenate([tg, gsrc])).size, l
        assert lp[l + 1] > lp[l] or lg[l + 1] > lg[l], "empty level"


@pytest.mark.parametrize("flags", [0, tn.DIRECTED, tn.TIES_SEQUENTIAL,
                                   tn.DIRECTED | tn.TIES_SEQUENTIAL, tn.FORWARD,
                                   tn.FORWARD | tn.DIRECTED,
                                   tn.FORWARD | tn.DIRECTED | tn.TIES_SEQUENTIAL])
def test_schedule_replay_matches_oracle(flags):
    directed = bool(flags & tn.DIRECTED)
    seq = bool(flags & tn.TIES_SEQUENTIAL)
    fwd = bool(flags & tn.FORWARD)
    for case in range(80):
        n = 2 + (case * 7) % 150
        m = (case * 13) % 400
        Tm = 1 + case % 25
        s, d, t = T.random_tiny(n, m, Tm, seed=7000 + case, allow_self=(case % 4 == 0))
        sch = tn.host_schedule(n, s, d, t, flags)
        check_disjoint(n, sch)
        check_ops_independent(sch)
        got = simulate(n, sch)
        ref = oracle.forward_matrix if fwd else oracle.reverse_matrix
        want = ref(n, s, d, t, directed=directed, sequential=seq)
        assert (got == want).all(), case
        assert (simulate_ops(n, sch) == want).all(), case


def test_schedule_replay_uniform_workload():
    s, d, t = T.make_workload("uniform_n1000_m20000")
    sch = tn.host_schedule(1000, s, d, t)
    check_disjoint(1000, sch)
    check_ops_independent(sch)
    assert sch["stats"]["compound_items"] > 0  # the workload has shared-node ties
    want = oracle.reverse_matrix(1000, s, d, t)
    assert (simulate(1000, sch) == want).all()
    assert (simulate_ops(1000, sch) == want).all()


def test_schedule_replay_activity_driven_sparse():
    s, d, t = T.activity_driven(3000, 6000, 500, seed=77)
    sch = tn.host_schedule(3000, s, d, t)
    check_disjoint(3000, sch)
    check_ops_independent(sch)
    want = oracle.reverse_matrix(3000, s, d, t)
    assert (simulate(3000, sch) == want).all()
    assert (simulate_ops(3000, sch) == want).all()


def test_items_cover_every_event_once_on_distinct_times():
    n = 500
    g = T.rng(3)
    m = 2000
    s = g.integers(0, n, m).astype(np.uint32)
    d = ((s + 1 + g.integers(0, n - 1, m)) % n).astype(np.uint32)
    t = np.arange(m, dtype=np.int64)
    st = tn.host_schedule(n, s, d, t)["stats"]
    assert st["pairs"] == m and st["gathers"] == 0


def test_one_time_step_is_one_level():
    s = np.array([0, 1, 2, 3, 5], dtype=np.uint32)
    d = np.array([1, 2, 3, 0, 6], dtype=np.uint32)
    sch = tn.host_schedule(8, s, d, np.zeros(5, dtype=np.int64))
    st = sch["stats"]
    assert st["levels"] == 1 and st["pairs"] == 1 and st["compound_items"] == 1
    assert st["gathers"] == 4


def test_self_loops_and_empty():
    sch = tn.host_schedule(4, [1, 2], [1, 2], [0, 1])
    assert sch["stats"]["levels"] == 0
    sch = tn.host_schedule(4, [], [], [])
    assert sch["stats"]["levels"] == 0 and sch["stats"]["pairs"] == 0


def test_planner_rejects_bad_input():
    with pytest.raises(tn.TNError) as e:
        tn.host_schedule(4, [0, 4], [1, 2], [0, 1])
    assert e.value.code == -2
    with pytest.raises(tn.TNError) as e:
        tn.host_schedule(4, [0, 1], [1, 2], [1, 0])
    assert e.value.code == -3
    with pytest.raises(tn.TNError) as e:
        tn.host_schedule(0, [], [], [])
    assert e.value.code == -1
    with pytest.raises(tn.TNError) as e:
        tn.host_schedule(4, [0], [1], [0], flags=8)
    assert e.value.code == -1


def test_forward_schedule_is_the_transpose():
    # Algorithm 1 in time order gives the transpose of the reverse-time
    # matrix, here through the planner's own schedules
    n = 120
    s, d, t = T.random_tiny(n, 900, 60, seed=77)
    f = simulate_ops(n, tn.host_schedule(n, s, d, t, tn.FORWARD))
    r = simulate_ops(n, tn.host_schedule(n, s, d, t))
    assert (oracle.to_dense(f, n) == oracle.to_dense(r, n).T).all()


def test_wide_levels_are_split_and_big_compound_items_fold():
    # one time step with 3000 events on 600 nodes: a single compound item of
    # many targets, and a first level far wider than the cap
    g = T.rng(12)
    n, m = 600, 3000
    s_ = g.integers(0, n, m).astype(np.uint32)
    d_ = g.integers(0, n, m).astype(np.uint32)
    t_ = np.zeros(m, dtype=np.int64)
    s2, d2, t2 = T.uniform_pairs(n, 5000, 10, seed=13)
    s_ = np.concatenate([s_, s2])
    d_ = np.concatenate([d_, d2])
    t_ = np.concatenate([t_, t2 + 1])
    sch = tn.host_schedule(n, s_, d_, t_)
    check_ops_independent(sch)
    assert sch["stats"]["scratch_rows"] >= 500
    assert (simulate_ops(n, sch) == oracle.reverse_matrix(n, s_, d_, t_)).all()


@pytest.mark.parametrize("flags", [0, tn.DIRECTED])
def test_compound_over_every_node_needs_fewer_scratch_rows_than_nodes(flags):
    # one time step whose events join all K = 4096 nodes: a compound item of
    # (nearly) every node as a target.  Its last target folds in place, so the
    # schedule needs at most K - 1 scratch rows: K + scratch + 1 LDS words fit
    # the one-wavefront kernel's 8192.
    g = T.rng(14)
    K = 4096
    perm = g.permutation(K).astype(np.uint32)
    s_ = np.concatenate([perm, g.integers(0, K, 6000).astype(np.uint32)])
    d_ = np.concatenate([np.roll(perm, -1), g.integers(0, K, 6000).astype(np.uint32)])
    t_ = np.zeros(s_.shape[0], dtype=np.int64)
    s2, d2, t2 = T.uniform_pairs(K, 3000, 40, seed=15)
    s_ = np.concatenate([s_, s2])
    d_ = np.concatenate([d_, d2])
    t_ = np.concatenate([t_, t2 + 1])
    sch = tn.host_schedule(K, s_, d_, t_, flags)
    check_ops_independent(sch)
    assert 1024 < sch["stats"]["scratch_rows"] <= K - 1
    want = oracle.reverse_matrix(K, s_, d_, t_, directed=bool(flags & tn.DIRECTED))
    assert (simulate_ops(K, sch) == want).all()


@pytest.mark.parametrize("flags", [0, tn.DIRECTED, tn.TIES_SEQUENTIAL, tn.FORWARD])
def test_forwarded_schedule_replay_matches_oracle(flags):
    # the plain kernel's form: results of the level before come from LDS, and
    # rows the next level overwrites are never stored; replayed with the
    # matrix holding only stored values, it must still give the oracle's
    # matrix (a wrongly skipped store or a stale read would show)
    cases = [T.random_tiny(150, 900, 30, seed=61), T.activity_driven(400, 6000, 300, seed=62),
             T.star_steps(300, 400, 12, seed=63), T.uniform_pairs(2000, 40000, 400, seed=66)]
    for k, (s_, d_, t_) in enumerate(cases):
        n = (150, 400, 300, 2000)[k]
        sch = tn.host_schedule(n, s_, d_, t_, flags)
        ref = oracle.forward_matrix if flags & tn.FORWARD else oracle.reverse_matrix
        want = ref(n, s_, d_, t_, directed=bool(flags & tn.DIRECTED),
                   sequential=bool(flags & tn.TIES_SEQUENTIAL))
        assert (simulate_fwd(n, sch) == want).all(), k
        fo = sch["fwd_ops"].astype(np.int64)
        assert (fo[:, :2] & FWD).any() and ((fo[:, 2:] != NOROW) & (fo[:, 2:] & FWD != 0)).any()


def fwd_layout_ok(sch):
    """Layout rules of the forwarded form: within a level the ops with both
    operands from memory come first, an op with one operand from memory has
    it second, and a forwarded operand names an op of the level before."""
    lv, fo = sch["fwd_lvl"], sch["fwd_ops"].astype(np.int64)
    cx, cy = (fo[:, 0] & FWD) == 0, (fo[:, 1] & FWD) == 0
    assert not (cx & ~cy).any()
    prev = 0
    for l in range(len(lv) - 1):
        both = (cx & cy)[lv[l]:lv[l + 1]]
        k = int(both.sum())
        assert both[:k].all(), l
        for c in (0, 1):
            hot = fo[lv[l]:lv[l + 1], c]
            hot = hot[(hot & FWD) != 0] & 0x3FF
            assert (hot < prev).all(), l
        prev = lv[l + 1] - lv[l]


@pytest.mark.parametrize("flags", [0, tn.DIRECTED, tn.FORWARD])
@pytest.mark.parametrize("cap", [0, 300, 97])
def test_forwarded_schedule_layout_and_level_caps(cap, flags):
    # the kernels' form (cap 0 = 768) and smaller caps, which split most
    # levels into parts decided one after the other: the replay must still
    # give the oracle's matrix, and splitting must only lose forwarding
    cases = [T.activity_driven(400, 6000, 300, seed=67), T.uniform_pairs(2000, 40000, 400, seed=68),
             T.star_steps(300, 400, 12, seed=69)]
    for k, (s_, d_, t_) in enumerate(cases):
        n = (400, 2000, 300)[k]
        sch = tn.host_schedule(n, s_, d_, t_, flags, fwd_level_cap=cap)
        fwd_layout_ok(sch)
        assert np.diff(sch["fwd_lvl"]).max() <= (cap or 768)
        ref = oracle.forward_matrix if flags & tn.FORWARD else oracle.reverse_matrix
        want = ref(n, s_, d_, t_, directed=bool(flags & tn.DIRECTED),
                   sequential=bool(flags & tn.TIES_SEQUENTIAL))
        assert (simulate_fwd(n, sch) == want).all(), (k, cap)
        if cap:
            full = tn.host_schedule(n, s_, d_, t_, flags)
            hot = lambda sc: int(((sc["fwd_ops"][:, :2].astype(np.int64) & FWD) != 0).sum())
            assert hot(sch) <= hot(full)


def test_forwarded_schedule_splits_wide_levels():
    # one time step of 3000 events: levels of up to 1024 ops become parts of
    # at most 768, and the replay still matches
    g = T.rng(64)
    n, m = 2000, 3000
    s_ = g.integers(0, n, m).astype(np.uint32)
    d_ = ((s_.astype(np.int64) + 1 + g.integers(0, n - 1, m)) % n).astype(np.uint32)
    s2, d2, t2 = T.uniform_pairs(n, 20000, 5, seed=65)
    s_, d_ = np.concatenate([s_, s2]), np.concatenate([d_, d2])
    t_ = np.concatenate([np.zeros(m, dtype=np.int64), t2 + 1])
    sch = tn.host_schedule(n, s_, d_, t_)
    widths = np.diff(sch["fwd_lvl"])
    assert widths.max() <= 768 and np.diff(sch["lvl_op"]).max() > 768
    assert len(widths) > sch["stats"]["op_levels"]
    assert (simulate_fwd(n, sch) == oracle.reverse_matrix(n, s_, d_, t_)).all()


@pytest.mark.parametrize("sw", [1, 2, 8])
def test_saturation_skips_keep_the_matrix(sw):
    # skipping the loads of saturated operands and the stores of full results
    # into full rows must not change any bit; with skipping off the counts are
    # the plain ones (2 row slices read per op, one written per destination)
    import satmodel
    for case, (n, m, Tm) in enumerate([(70, 900, 300), (300, 4000, 1500), (200, 3000, 5)]):
        s, d, t = T.random_tiny(n, m, Tm, seed=8100 + case)
        sch = tn.host_schedule(n, s, d, t)
        want = oracle.reverse_matrix(n, s, d, t)
        got, ld, st = satmodel.replay(n, sch, sw)
        assert (got == want).all(), case
        got0, ld0, st0 = satmodel.replay(n, sch, sw, saturation=False)
        assert (got0 == want).all(), case
        ops = sch["ops"]
        nw = oracle.words(n)
        assert ld0 == 2 * ops.shape[0] * nw
        assert st0 == int((ops[:, 2:] != satmodel.NOROW).sum()) * nw
        assert ld < ld0 and st < st0, case  # these networks saturate


@pytest.mark.parametrize("sw", [1, 4])
def test_zero_skips_keep_the_matrix(sw):
    # sparse networks: most row slices stay all zero for many levels; not
    # loading zero operands and not storing zero results into zero rows must
    # not change any bit, and must move fewer words than the full-row rule
    # alone
    import satmodel
    for case, (n, m, Tm) in enumerate([(700, 600, 300), (1000, 3000, 2000), (260, 400, 50)]):
        s, d, t = T.random_tiny(n, m, Tm, seed=8400 + case)
        sch = tn.host_schedule(n, s, d, t)
        want = oracle.reverse_matrix(n, s, d, t)
        got, ld, st = satmodel.replay(n, sch, sw)
        assert (got == want).all(), case
        got1, ld1, st1 = satmodel.replay(n, sch, sw, zero=False)
        assert (got1 == want).all(), case
        assert ld < ld1 and st <= st1, case


def test_saturation_model_stops_full_slices():
    # a slice whose rows are all full stops: no traffic after that level,
    # same matrix; n = 64 k + 1 gives a last slice of one column whose only
    # row starts full
    import satmodel
    n = 129
    s, d, t = T.random_tiny(n, 6000, 3000, seed=8200)
    sch = tn.host_schedule(n, s, d, t)
    want = oracle.reverse_matrix(n, s, d, t)
    assert oracle.sizes(want, n)[0].min() == n  # every row ends full
    got, ld, st = satmodel.replay(n, sch, 1)
    assert (got == want).all()
    _, ld0, st0 = satmodel.replay(n, sch, 1, saturation=False)
    assert ld < ld0 // 4


@pytest.mark.parametrize("blocks", [False, True])
def test_scratch_rows_live_across_the_forwarding_cut(blocks):
    # the premise of the GPU tests of the saturating path with a forwarding
    # phase: some compound items' scratch rows are written before the level
    # at which the ops reach 9 n and read after it, so the launches on
    # either side must find them at the same place
    n = 16385
    if blocks:
        s, d, t = T.two_block_pairs(n, 600_000, 2000, seed=8410)
    else:
        s, d, t = T.uniform_pairs(n, 400_000, 2000, seed=8400)
    sch = tn.host_schedule(n, s, d, t)
    lv, L = sch["lvl_op"].astype(np.int64), sch["stats"]["op_levels"]
    ops = sch["ops"].astype(np.int64)
    mid = int(np.searchsorted(lv[:L], 9 * n, side="left"))
    lvl = np.repeat(np.arange(L), np.diff(lv[:L + 1]))
    SCR, NOROW = 0x80000000, 0xFFFFFFFF
    last = {}
    crossing = 0
    for i in range(ops.shape[0]):
        for c in (0, 1):
            x = int(ops[i, c])
            if x != NOROW and x & SCR and last.get(x, mid) < mid <= lvl[i]:
                crossing += 1
        for c in (2, 3):
            x = int(ops[i, c])
            if x != NOROW and x & SCR:
                last[x] = lvl[i]
    assert crossing > 100
