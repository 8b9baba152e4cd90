"""GPU parity of the streamed one-shot build: the event list cut into chunks
of whole time steps, planned on host threads and applied in reverse time,
with each column slice's saturation state carried from launch to launch and
the build stopping once every slice is all ones."""
import numpy as np
import pytest
import torch

import oracle
import tn_inputs as T
from gpu_util import host

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def flag_kw(flags):
    return dict(directed=bool(flags & tn.DIRECTED), sequential=bool(flags & tn.TIES_SEQUENTIAL))


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_streamed_matches_oracle_for_any_chunk_size(flags):
    cases = [(300, 4000, 1500), (129, 6000, 3000), (1000, 20000, 6000), (5000, 12000, 3000),
             (70, 50, 5), (2, 10, 3)]
    for case, (n, m, Tm) in enumerate(cases):
        s, d, t = T.random_tiny(n, m, Tm, seed=8500 + case, allow_self=case % 2 == 0)
        want = oracle.reverse_matrix(n, s, d, t, **flag_kw(flags))
        for chunk in (0, 1, 7, 500):
            C, st = tn.build_component_matrix_streamed(n, s, d, t, flags, chunk_events=chunk)
            assert (host(C) == want).all(), (case, chunk)
            assert 0 <= st["chunks_run"] <= st["chunks"] and st["events_run"] <= m


def test_saturating_stream_stops_early_and_skipping_off_runs_all():
    n, m = 3000, 300_000
    s, d, t = T.activity_driven(n, m, 30_000, seed=21)
    want = oracle.reverse_matrix(n, s, d, t)
    assert oracle.sizes(want, n)[0].min() == n  # every row ends full
    ctx = tn.get_context()
    C, st = tn.build_component_matrix_streamed(n, s, d, t, chunk_events=4096)
    assert (host(C) == want).all()
    assert st["saturated"] == 1 and st["events_run"] < m and st["chunks_run"] < st["chunks"]
    try:
        ctx.saturation(False)
        C0, st0 = tn.build_component_matrix_streamed(n, s, d, t, chunk_events=4096)
    finally:
        ctx.saturation(True)
    assert (host(C0) == want).all()
    assert st0["saturated"] == 0 and st0["chunks_run"] == st0["chunks"]


def test_one_shot_build_is_the_streamed_build():
    s, d, t = T.uniform_pairs(2000, 30000, 800, seed=4)
    want = oracle.reverse_matrix(2000, s, d, t)
    C = tn.build_component_matrix(2000, s, d, t)
    assert (host(C) == want).all()
    ld = oracle.words(2000) + 2
    C2 = torch.full((2000, ld), -1, dtype=torch.int64, device="cuda")
    C2, _ = tn.build_component_matrix_streamed(2000, s, d, t, C=C2, chunk_events=1000)
    got = host(C2)
    assert (got[:, :oracle.words(2000)] == want).all() and not got[:, oracle.words(2000):].any()


def test_streamed_errors_enqueue_nothing():
    C = torch.zeros((100, 2), dtype=torch.int64, device="cuda")
    for (s, d, t), code in [(([0, 100], [1, 2], [0, 1]), -2), (([0, 1], [1, 2], [3, 1]), -3)]:
        with pytest.raises(tn.TNError) as e:
            tn.build_component_matrix_streamed(100, s, d, t, C=C)
        assert e.value.code == code
    with pytest.raises(tn.TNError) as e:
        tn.build_component_matrix_streamed(100, [0], [1], [0], C=C, chunk_events=-1)
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert (C.cpu() == 0).all()


@pytest.mark.parametrize("flags", [0, tn.FORWARD, tn.TIES_SEQUENTIAL | tn.FORWARD])
def test_default_chunks_grow_from_the_first_applied_end(flags):
    # chunk_events = 0: a first chunk of 2^16 events (a quarter of 2^18)
    # doubling up to 2^18, cut from the end in reverse time and from the
    # start forward: 64k + the rest of 180k events = 2 chunks
    n, m = 1500, 180_000
    s, d, t = T.uniform_pairs(n, m, 60_000, seed=31)
    ref = oracle.forward_matrix if flags & tn.FORWARD else oracle.reverse_matrix
    want = ref(n, s, d, t, sequential=bool(flags & tn.TIES_SEQUENTIAL))
    ctx = tn.get_context()
    try:
        ctx.saturation(False)  # every chunk runs
        C, st = tn.build_component_matrix_streamed(n, s, d, t, flags)
    finally:
        ctx.saturation(True)
    assert (host(C) == want).all()
    assert st["chunks"] == 2 and st["chunks_run"] == 2 and st["events_run"] == m


def _matchings_then_singles(n, steps, singles, seed, wide_first):
    # `steps` time steps of a random perfect matching (n / 2 simultaneous,
    # node-disjoint events: levels of about 1000 ops, the workgroup kernel)
    # and `singles` time steps of one event each along a path (one op per
    # level, the wavefront kernel), in either order along time
    g = T.rng(seed)
    wide = []
    for _ in range(steps):
        p = g.permutation(n).astype(np.uint32)
        wide.append((p[0::2], p[1::2]))
    start = int(g.integers(0, n))
    one = [(np.array([(start + k) % n], dtype=np.uint32),
            np.array([(start + k + 1) % n], dtype=np.uint32)) for k in range(singles)]
    parts = wide + one if wide_first else one + wide
    s = np.concatenate([a for a, _ in parts])
    d = np.concatenate([b for _, b in parts])
    t = np.concatenate([np.full(a.shape[0], k, dtype=np.int64) for k, (a, _) in enumerate(parts)])
    return s, d, t


@pytest.mark.parametrize("wide_first", [True, False])
def test_stream_switches_kernels_between_chunks(wide_first):
    # chunks of short levels run on one wavefront per word column, chunks of
    # wide levels on the workgroup kernel; each hands its per-column slice
    # state to the other
    n = 6000
    s, d, t = _matchings_then_singles(n, 6, 4000, seed=61 + wide_first, wide_first=wide_first)
    for a, b in ((0, 3000), (t.shape[0] - 3000, t.shape[0])):
        st = tn.host_schedule(n, s[a:b], d[a:b], t[a:b])["stats"]
        wide = t[a] < 6 if wide_first else t[a] >= 4000
        assert (st["ops"] > 640 * st["op_levels"]) == wide, (a, st["ops"], st["op_levels"])
    want = oracle.reverse_matrix(n, s, d, t)
    ctx = tn.get_context()
    try:
        for sat in (True, False):
            ctx.saturation(sat)
            C, st = tn.build_component_matrix_streamed(n, s, d, t, chunk_events=3000)
            assert (host(C) == want).all(), (wide_first, sat)
            assert st["slice_words"] == 1 and st["chunks"] >= 4
            if not sat:
                assert st["chunks_run"] == st["chunks"]
    finally:
        ctx.saturation(True)
