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
                                   tn.DIRECTED | tn.TIES_SEQUENTIAL])
def test_schedule_replay_matches_oracle(flags):
    directed = bool(flags & tn.DIRECTED)
    seq = bool(flags & tn.TIES_SEQUENTIAL)
    for case in range(80):
        n = 2 + (case * 7) % 150
        m = (case * 13) % 400
        Tm = 1 + case % 25
        s, d, t = T.random_tiny(n, m, Tm, seed=7000 + case, allow_self=(case % 4 == 0))
        sch = tn.host_schedule(n, s, d, t, flags)
        check_disjoint(n, sch)
        got = simulate(n, sch)
        want = oracle.reverse_matrix(n, s, d, t, directed=directed, sequential=seq)
        assert (got == want).all(), case


def test_schedule_replay_uniform_workload():
    s, d, t = T.make_workload("uniform_n1000_m20000")
    sch = tn.host_schedule(1000, s, d, t)
    check_disjoint(1000, sch)
    assert sch["stats"]["compound_items"] > 0  # the workload has shared-node ties
    assert (simulate(1000, sch) == oracle.reverse_matrix(1000, s, d, t)).all()


def test_schedule_replay_activity_driven_sparse():
    s, d, t = T.activity_driven(3000, 6000, 500, seed=77)
    sch = tn.host_schedule(3000, s, d, t)
    check_disjoint(3000, sch)
    got = simulate(3000, sch)
    assert (got == oracle.reverse_matrix(3000, s, d, t)).all()


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
