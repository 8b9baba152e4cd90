"""GPU parity of the persistent multi-network kernel (LDS and global tiles,
work queues, autotuned shape, HIP graph replays) against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import tn_inputs as T
from gpu_util import host

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def suite(seed=0):
    nets = []
    sizes = [2, 3, 63, 64, 65, 129, 500, 1000, 2047, 5000, 20000, 30000]
    for i, n in enumerate(sizes):
        m = min(3 * n, 60000)
        if i % 3 == 0:
            s, d, t = T.uniform_pairs(n, m, max(1, m // 4), seed=seed + i)
        elif i % 3 == 1:
            s, d, t = T.activity_driven(n, m, max(1, m // 5), seed=seed + i)
        else:
            s, d, t = T.random_tiny(n, m, max(1, m // 3), seed=seed + i, allow_self=True)
        nets.append((n, s, d, t))
    nets.append((700, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64)))
    return nets


def check(nets, Cs, **kw):
    for (n, s, d, t), C in zip(nets, Cs):
        got = host(C)
        want = oracle.reverse_matrix(n, s, d, t, **kw)
        assert (got[:, :oracle.words(n)] == want).all(), n
        assert not got[:, oracle.words(n):].any(), n


def test_batch_matches_oracle_and_uses_both_tile_kinds():
    nets = suite()
    b = tn.Batch(nets)
    stats, tiles, lds_tiles = b.stats()
    assert tiles >= len(nets) and 0 < lds_tiles < tiles  # n = 30000 needs global tiles
    Cs = b.execute()
    check(nets, Cs)
    b.close()


@pytest.mark.parametrize("flags", [tn.DIRECTED, tn.TIES_SEQUENTIAL, tn.DIRECTED | tn.TIES_SEQUENTIAL])
def test_batch_flags(flags):
    nets = [net for net in suite(100) if net[0] <= 5000]
    Cs = tn.build_component_matrix_batched(nets, flags=flags)
    check(nets, Cs, directed=bool(flags & 1), sequential=bool(flags & 2))


def test_graph_replays_and_rebinding():
    nets = suite(200)
    b = tn.Batch(nets)
    Cs = b.alloc()
    for rep in range(3):
        for C in Cs:
            C.fill_(-1)  # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        b.execute(Cs)
        check(nets, Cs)
        assert torch.isfinite(junk)
    # new outputs with padded rows
    Ds = [torch.full((n, oracle.words(n) + 2), -1, dtype=torch.int64, device="cuda")
          for (n, _, _, _) in nets]
    b.execute(Ds)
    check(nets, Ds)
    b.execute(Cs)
    check(nets, Cs)
    b.close()


def test_many_uneven_networks_one_launch():
    specs = T.batched_suite(48, seed=4000, n_range=(500, 6000), m_range=(10_000, 60_000))
    nets = [(sp.n,) + sp.generate() for sp in specs]
    Cs = tn.Batch(nets).execute()
    for (n, s, d, t), C in zip(nets[::6], Cs[::6]):
        assert (host(C) == oracle.reverse_matrix(n, s, d, t)).all(), n
    for (n, s, d, t), C in zip(nets, Cs):
        out, inn = tn.component_sizes(C, n)
        o, i = out.cpu().numpy(), inn.cpu().numpy()
        assert o.sum() == i.sum() and (o >= 1).all()


def test_batch_errors():
    with pytest.raises(tn.TNError) as e:
        tn.Batch([(10, [0], [11], [0])])
    assert e.value.code == -2
    with pytest.raises(tn.TNError) as e:
        tn.Batch([(10, [0, 1], [1, 2], [3, 2])])
    assert e.value.code == -3


def test_saturating_networks_with_and_without_skipping():
    # dense networks whose rows all fill up (tiles stop early), an n = 64 k + 1
    # network whose last slice has one column, and a global-memory tile
    nets = []
    for i, (n, m) in enumerate([(129, 20000), (700, 60000), (2049, 150000), (30000, 600000)]):
        s, d, t = T.activity_driven(n, m, max(1, m // 10), seed=300 + i)
        nets.append((n, s, d, t))
    want = [oracle.reverse_matrix(n, s, d, t) for n, s, d, t in nets]
    assert all(oracle.sizes(w, n)[0].min() == n for w, (n, _, _, _) in zip(want[:3], nets))
    ctx = tn.get_context()
    b = tn.Batch(nets)
    try:
        for sat in (True, False, True):
            ctx.saturation(sat)
            Cs = b.execute()
            for (n, _, _, _), C, w in zip(nets, Cs, want):
                assert (host(C)[:, :oracle.words(n)] == w).all(), (sat, n)
        for flags in (tn.DIRECTED, tn.DIRECTED | tn.TIES_SEQUENTIAL):
            Cs = tn.build_component_matrix_batched(nets[:3], flags=flags)
            check(nets[:3], Cs, directed=True, sequential=bool(flags & 2))
    finally:
        ctx.saturation(True)
        b.close()


def test_dense_unsaturated_networks():
    # dense activity-driven networks in which nodes active only late in time
    # keep small out-components: tiles never saturate, although most of
    # their items have full operands and full destinations
    nets = []
    for i, (n, m, Tm) in enumerate([(3000, 36_000, 3_600), (6000, 72_000, 7_200),
                                    (1200, 14_400, 1_440), (4000, 40_000, 4_000)]):
        s, d, t = T.activity_driven(n, m, Tm, seed=910 + i)
        nets.append((n, s, d, t))
    want = [oracle.reverse_matrix(n, s, d, t) for n, s, d, t in nets]
    assert all(oracle.sizes(w, n)[0].min() < n for w, (n, _, _, _) in zip(want, nets))
    ctx = tn.get_context()
    b = tn.Batch(nets)
    try:
        for sat in (True, False):
            ctx.saturation(sat)
            Cs = b.execute()
            for (n, _, _, _), C, w in zip(nets, Cs, want):
                assert (host(C)[:, :oracle.words(n)] == w).all(), (sat, n)
        for flags in (tn.DIRECTED, tn.FORWARD):
            Cs = tn.build_component_matrix_batched(nets[:2], flags=flags)
            for (n, s, d, t), C in zip(nets[:2], Cs):
                ref = oracle.forward_matrix if flags == tn.FORWARD else oracle.reverse_matrix
                assert (host(C)[:, :oracle.words(n)] ==
                        ref(n, s, d, t, directed=bool(flags & tn.DIRECTED))).all()
    finally:
        ctx.saturation(True)
        b.close()


def test_star_steps_wide_and_narrow_gathers():
    # one star per time step: the hub's compound item gathers from up to
    # 1 + max_k rows (records with more than three sources read the rest from
    # the source list), partners gather from two rows, self-loops from one;
    # an LDS tile, a dense saturating one and a global-memory tile
    nets = []
    for i, (n, steps, k) in enumerate([(300, 3000, 9), (2000, 20000, 12), (30000, 4000, 6)]):
        s, d, t = T.star_steps(n, steps, k, seed=950 + i)
        nets.append((n, s, d, t))
    sizes = set()
    for n, s, d, t in nets:
        sizes |= set(np.diff(tn.host_schedule(n, s, d, t)["gat_ptr"]).tolist())
    assert min(sizes) <= 2 and max(sizes) >= 8
    ctx = tn.get_context()
    try:
        for sat in (True, False):
            ctx.saturation(sat)
            for flags in (0, tn.DIRECTED):
                Cs = tn.build_component_matrix_batched(nets, flags=flags)
                check(nets, Cs, directed=bool(flags & tn.DIRECTED))
    finally:
        ctx.saturation(True)
