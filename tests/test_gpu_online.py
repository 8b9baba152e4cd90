"""GPU parity of forward streaming (Algorithm 1 in time order, rows are
in-components) and of online insertion into a live matrix, in both time
directions, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import tn_inputs as T
from gpu_util import host

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def tick_batches(t, k, seed):
    """Cut a time-ordered list into k batches on time-step boundaries."""
    g = T.rng(seed)
    ticks = np.unique(t)
    cuts = np.sort(g.choice(ticks[1:], size=min(k - 1, len(ticks) - 1), replace=False))
    edges = [0] + [int(np.searchsorted(t, c, side="left")) for c in cuts] + [len(t)]
    return [(edges[i], edges[i + 1]) for i in range(len(edges) - 1)]


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_forward_plan_and_streamed_build_match_the_forward_oracle(flags):
    F = tn.FORWARD | flags
    for case, (n, m, Tm) in enumerate([(300, 4000, 1500), (129, 6000, 3000), (2000, 9000, 700)]):
        s, d, t = T.random_tiny(n, m, Tm, seed=9900 + case)
        want = oracle.forward_matrix(n, s, d, t, directed=bool(flags & 1),
                                     sequential=bool(flags & 2))
        p = tn.Plan(n, s, d, t, F)
        assert (host(p.execute()) == want).all(), case
        p.close()
        for chunk in (0, 9, 700):
            C, st = tn.build_component_matrix_streamed(n, s, d, t, F, chunk_events=chunk)
            assert (host(C) == want).all(), (case, chunk)
    # the transpose of the reverse-time matrix
    n = 500
    s, d, t = T.activity_driven(n, 3000, 1000, seed=5)
    Cf = oracle.to_dense(host(tn.build_component_matrix(n, s, d, t, flags=tn.FORWARD)), n)
    Cr = oracle.to_dense(host(tn.build_component_matrix(n, s, d, t)), n)
    assert (Cf == Cr.T).all()


@pytest.mark.parametrize("flags", [tn.FORWARD, tn.FORWARD | tn.DIRECTED, 0, tn.DIRECTED])
def test_online_batches_equal_the_whole_stream(flags):
    n = 3000
    s, d, t = T.activity_driven(n, 40_000, 6_000, seed=31)
    fwd = bool(flags & tn.FORWARD)
    ref = oracle.forward_matrix if fwd else oracle.reverse_matrix
    want = ref(n, s, d, t, directed=bool(flags & tn.DIRECTED))
    o = tn.Online(n, flags)
    batches = tick_batches(t, 7, seed=3)
    if not fwd:
        batches = batches[::-1]  # reverse time: the latest events first
    for k, (a, b) in enumerate(batches):
        st = o.insert(s[a:b], d[a:b], t[a:b], chunk_events=1500 if k % 2 else 0)
        assert st["events_run"] <= b - a
    assert (host(o.C) == want).all()
    # sizes of the live matrix
    out, inn = tn.component_sizes(o.C, n)
    wo, wi = oracle.sizes(want, n)
    assert (out.cpu().numpy() == wo).all() and (inn.cpu().numpy() == wi).all()
    o.close()


def test_online_order_rules_and_saturation():
    n = 400
    o = tn.Online(n, tn.FORWARD)
    o.insert([0, 1], [1, 2], [5, 6])
    for src, dst, tt in (([2], [3], [6]), ([2], [3], [4])):  # not later than t = 6
        with pytest.raises(tn.TNError) as e:
            o.insert(src, dst, tt)
        assert e.value.code == -3
    with pytest.raises(tn.TNError) as e:
        o.insert([0], [400], [9])
    assert e.value.code == -2
    o.insert([2], [3], [7])
    want = oracle.forward_matrix(n, np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32),
                                 np.array([5, 6, 7], np.int64))
    assert (host(o.C) == want).all()
    o.close()
    # sequential ties may continue the last time step
    o = tn.Online(n, tn.FORWARD | tn.TIES_SEQUENTIAL)
    o.insert([0], [1], [5])
    o.insert([1], [2], [5])
    want = oracle.forward_matrix(n, np.array([0, 1], np.uint32), np.array([1, 2], np.uint32),
                                 np.array([5, 5], np.int64), sequential=True)
    assert (host(o.C) == want).all()
    o.close()
    # a saturated matrix skips later batches
    s, d, t = T.activity_driven(n, 60_000, 6_000, seed=8)
    o = tn.Online(n, tn.FORWARD)
    o.insert(s, d, t, chunk_events=2000)
    assert (oracle.to_dense(host(o.C), n)).all()
    tn.get_context().sync()
    st = o.insert([0], [1], [10**9])
    assert st["chunks_run"] == 0 and st["saturated"] == 1
    o.close()
