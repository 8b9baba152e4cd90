"""GPU parity of the exact component-matrix path against the CPU oracle:
bit-exact matrices and sizes, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import tn_inputs as T
from gpu_util import host

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def gpu_matrix(n, s, d, t, flags=0, ld=None, slice_words=0):
    p = tn.Plan(n, s, d, t, flags)
    C = tn.api.alloc_matrix(n, ld=ld)
    p.execute(C, slice_words=slice_words)
    out = host(C)
    p.close()
    return out


def flag_kw(flags):
    return dict(directed=bool(flags & tn.DIRECTED), sequential=bool(flags & tn.TIES_SEQUENTIAL))


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_tiny_tie_heavy_suites(flags):
    for case in range(40):
        n = 2 + (case * 11) % 200
        m = (case * 37) % 600
        s, d, t = T.random_tiny(n, m, 1 + case % 15, seed=9100 + case, allow_self=case % 3 == 0)
        got = gpu_matrix(n, s, d, t, flags)
        want = oracle.reverse_matrix(n, s, d, t, **flag_kw(flags))
        assert (got == want).all(), (flags, case, n, m)


def test_uniform_pairs_n1000_matrix_and_sizes():
    s, d, t = T.make_workload("uniform_n1000_m20000")
    C = tn.build_component_matrix(1000, s, d, t)
    out, inn = tn.component_sizes(C, 1000)
    want = oracle.reverse_matrix(1000, s, d, t)
    assert (host(C) == want).all()
    wo, wi = oracle.sizes(want, 1000)
    assert (out.cpu().numpy() == wo).all() and (inn.cpu().numpy() == wi).all()


@pytest.mark.parametrize("n,m,T_", [(5000, 12000, 3000), (20000, 40000, 20000)])
def test_sparse_activity_driven_all_slice_widths(n, m, T_):
    s, d, t = T.activity_driven(n, m, T_, seed=n)
    want = oracle.reverse_matrix(n, s, d, t)
    wo, wi = oracle.sizes(want, n)
    assert len(np.unique(wo)) > 10  # out-components of many sizes
    p = tn.Plan(n, s, d, t)
    for sw in (1, 2, 4, 8, 16, 32, 64):
        C = p.execute(slice_words=sw)
        assert (host(C) == want).all(), sw
        out, inn = tn.component_sizes(C, n)
        assert (out.cpu().numpy() == wo).all() and (inn.cpu().numpy() == wi).all()
    p.close()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129, 1000, 4097])
def test_ragged_sizes_and_padding(n):
    s, d, t = T.random_tiny(max(n, 2), 3 * n, 7, seed=n)
    if n == 1:
        s, d, t = np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64)
    want = oracle.reverse_matrix(n, s, d, t)
    ld = oracle.words(n) + 3
    got = gpu_matrix(n, s, d, t, ld=ld)
    assert (got[:, :oracle.words(n)] == want).all()
    assert not got[:, oracle.words(n):].any()


def test_no_events_gives_identity():
    C = tn.build_component_matrix(300, [], [], [])
    assert (oracle.to_dense(host(C), 300) == np.eye(300, dtype=bool)).all()
    out, inn = tn.component_sizes(C, 300)
    assert (out.cpu().numpy() == 1).all() and (inn.cpu().numpy() == 1).all()


def test_deterministic_repeat():
    s, d, t = T.activity_driven(8000, 30000, 2000, seed=5)
    p = tn.Plan(8000, s, d, t)
    a = host(p.execute())
    b = host(p.execute(slice_words=1))
    assert (a == b).all()


def test_errors_enqueue_nothing():
    with pytest.raises(tn.TNError) as e:
        tn.Plan(4, [0], [4], [0])
    assert e.value.code == -2
    with pytest.raises(tn.TNError) as e:
        tn.Plan(4, [0, 1], [1, 2], [5, 1])
    assert e.value.code == -3
    p = tn.Plan(100, [0], [1], [0])
    C = torch.zeros((100, 1), dtype=torch.int64, device="cuda")  # ld 1 < 2 words
    rc = tn.lib.tn_plan_execute(tn.get_context().bind_stream(), p.h, tn.api._dp(C), 1, 0)
    assert rc == -1
    big = torch.zeros((100, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(tn.TNError):
        p.execute(big, slice_words=3)  # not a power of two
    torch.cuda.synchronize()
    assert (C.cpu() == 0).all() and (big.cpu() == 0).all()  # nothing was enqueued
    p.execute(big)
    assert oracle.to_dense(host(big), 100)[0, 1]


def test_profile_records_each_kernel():
    ctx = tn.get_context()
    s, d, t = T.uniform_pairs(2000, 5000, 100, seed=3)
    p = tn.Plan(2000, s, d, t)
    ctx.profile(True)
    C = p.execute()
    tn.component_sizes(C, 2000)
    recs = ctx.profile_take()
    ctx.profile(False)
    names = [r[0] for r in recs]
    assert names == ["identity", "rowor", "out_sizes", "in_sizes"]
    assert all(ms >= 0 for _, ms in recs)


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_saturation_counts_match_host_model(flags):
    # the kernel's own traffic counters against the host model of its skip
    # rule, with skipping on and off, on networks that saturate and ragged n
    import satmodel
    ctx = tn.get_context()
    cases = [(300, 4000, 1500), (200, 3000, 5), (1000, 20000, 6000), (130, 50, 40),
             (129, 6000, 3000), (513, 9000, 4000)]
    try:
        for case, (n, m, Tm) in enumerate(cases):
            s, d, t = T.random_tiny(n, m, Tm, seed=8300 + case)
            sch = tn.host_schedule(n, s, d, t, flags)
            want = oracle.reverse_matrix(n, s, d, t, **flag_kw(flags))
            p = tn.Plan(n, s, d, t, flags)
            for sat in (True, False):
                ctx.saturation(sat)
                for sw in (1, 4, 8, 16, 64):
                    C = p.execute(slice_words=sw)
                    assert (host(C) == want).all(), (case, sat, sw)
                    if not sat and sw <= 16:
                        # the plain recurrence on the forwarded schedule
                        ld, st = satmodel.fwd_traffic(n, sch)
                    else:
                        _, ld, st = satmodel.replay(n, sch, sw, saturation=sat)
                    assert ctx.last_traffic() == (ld, st), (case, sat, sw)
            p.close()
    finally:
        ctx.saturation(True)


@pytest.fixture(scope="module")
def c2():
    s, d, t = T.make_workload("activity_n100000_m10M")
    p = tn.Plan(100_000, s, d, t)
    C = p.execute()
    out, inn = tn.component_sizes(C, 100_000)
    torch.cuda.synchronize()
    yield dict(s=s, d=d, t=t, C=C, out=out.cpu().numpy(), inn=inn.cpu().numpy(), plan=p)
    p.close()


def test_full_size_sampled_columns(c2):
    n = 100_000
    nw = oracle.words(n)
    for w0, k in ((0, 2), (700, 1), (nw - 2, 2)):
        want = oracle.reverse_matrix(n, c2["s"], c2["d"], c2["t"], w0=w0, nw=k)
        got = c2["C"][:, w0:w0 + k].cpu().numpy().view(np.uint64)
        assert (got == want).all(), w0
        cols = oracle.col_counts(want)
        lo, hi = 64 * w0, min(n, 64 * (w0 + k))
        assert (c2["inn"][lo:hi] == cols[:hi - lo]).all()


def test_full_size_sampled_rows(c2):
    # rows of C are columns of the forward matrix S (the transpose identity)
    n = 100_000
    for w0 in (3, 1000):
        S = oracle.forward_matrix(n, c2["s"], c2["d"], c2["t"], w0=w0, nw=1)
        Sd = oracle.to_dense(S, 64)  # n x 64: column b = source 64*w0 + b
        rows = c2["C"][64 * w0:64 * w0 + 64].cpu().numpy().view(np.uint64)
        Rd = oracle.to_dense(rows, n)  # 64 x n
        assert (Rd == Sd.T).all(), w0
        assert (c2["out"][64 * w0:64 * w0 + 64] == Sd.sum(axis=0)).all()


def test_full_size_invariants(c2):
    n = 100_000
    assert c2["out"].sum() == c2["inn"].sum()
    assert (c2["out"] >= 1).all() and (c2["out"] <= n).all()
    diag = torch.arange(n, device="cuda")
    words_ = c2["C"][diag, diag // 64]
    assert bool((((words_ >> (diag % 64)) & 1) == 1).all())
    assert not bool((c2["C"][:, -1] >> (n % 64)).any())


def test_full_size_saturation_off_gives_same_matrix(c2):
    ctx = tn.get_context()
    C = c2["plan"].execute()
    ld_on, st_on = ctx.last_traffic()
    ctx.saturation(False)
    try:
        C0 = c2["plan"].execute()
        ld_off, st_off = ctx.last_traffic()
    finally:
        ctx.saturation(True)
    assert torch.equal(C, c2["C"]) and torch.equal(C0, c2["C"])
    # the plain recurrence runs on the forwarded schedule: about half the
    # operands come from the level before through LDS
    import satmodel
    sch = tn.host_schedule(100_000, c2["s"], c2["d"], c2["t"])
    assert (ld_off, st_off) == satmodel.fwd_traffic(100_000, sch)
    nw = oracle.words(100_000)
    assert ld_off < 2 * c2["plan"].stats["ops"] * nw
    assert ld_on < ld_off and st_on < st_off


def test_full_size_sixteen_word_slices(c2):
    # whole 128-byte lines per row access: the one-frame forwarding kernel
    # (saturation off) and, with saturation, its forwarding phase and the
    # slice state of 16-word slices
    import satmodel
    ctx = tn.get_context()
    C1 = c2["plan"].execute(slice_words=16).clone()
    ctx.saturation(False)
    try:
        C0 = c2["plan"].execute(slice_words=16)
        traffic = ctx.last_traffic()
    finally:
        ctx.saturation(True)
    assert torch.equal(C0, c2["C"]) and torch.equal(C1, c2["C"])
    sch = tn.host_schedule(100_000, c2["s"], c2["d"], c2["t"])
    assert traffic == satmodel.fwd_traffic(100_000, sch)


def test_full_size_streamed_build_stops_early(c2):
    C, st = tn.build_component_matrix_streamed(100_000, c2["s"], c2["d"], c2["t"])
    assert torch.equal(C, c2["C"])
    assert st["saturated"] == 1 and st["events_run"] < 10_000_000


def test_node_relabeling_gives_the_relabeled_matrix():
    # a race check: a random relabeling of the nodes changes every row
    # address and the order of the items inside each level, so any result
    # that depended on item order or on unsynchronized row traffic would
    # differ; the plan, the streamed build and the batched kernel must all
    # give C'[pi(u)][pi(w)] = C[u][w]
    n = 1500
    s, d, t = T.activity_driven(n, 40_000, 2_000, seed=77)
    pi = T.rng(78).permutation(n).astype(np.uint32)
    want = oracle.to_dense(oracle.reverse_matrix(n, s, d, t), n)
    ps, pd = pi[s], pi[d]
    p = tn.Plan(n, ps, pd, t)
    outs = [p.execute(), tn.build_component_matrix_streamed(n, ps, pd, t, chunk_events=3000)[0]]
    outs += tn.build_component_matrix_batched([(n, ps, pd, t), (n, s, d, t)])[:1]
    for k, C in enumerate(outs):
        D = oracle.to_dense(host(C)[:, :oracle.words(n)], n)
        assert (D[np.ix_(pi, pi)] == want).all(), k
    p.close()


@pytest.mark.parametrize("flags", [0, tn.DIRECTED, tn.TIES_SEQUENTIAL, tn.FORWARD])
def test_small_networks_on_one_wavefront_per_column(flags):
    # small n with the slice width left to the library: one wavefront per
    # word column runs every level with the column in LDS.  Long schedules
    # (many op and level windows), compound-heavy star steps, a column count
    # that is not a multiple of anything; against the oracle and against the
    # workgroup kernel (an explicit slice width selects it)
    cases = [T.er_poisson(100, 200_000, 20_000_000, seed=81), T.star_steps(700, 5000, 9, seed=82),
             T.activity_driven(3000, 60_000, 30_000, seed=83)]
    for k, (s, d, t) in enumerate(cases):
        n = (100, 700, 3000)[k]
        st = tn.host_schedule(n, s, d, t, flags)["stats"]
        assert st["ops"] <= 640 * st["op_levels"], k  # short levels: the wavefront kernel
        ref = oracle.forward_matrix if flags & tn.FORWARD else oracle.reverse_matrix
        want = ref(n, s, d, t, directed=bool(flags & tn.DIRECTED),
                   sequential=bool(flags & tn.TIES_SEQUENTIAL))
        assert (gpu_matrix(n, s, d, t, flags) == want).all(), k
        assert (gpu_matrix(n, s, d, t, flags, slice_words=1) == want).all(), k
        C, st = tn.build_component_matrix_streamed(n, s, d, t, flags, chunk_events=7000)
        assert (host(C)[:, :oracle.words(n)] == want).all(), k
        assert st["chunks_run"] <= st["chunks"]


def test_wavefront_kernel_stops_full_columns():
    # networks whose rows all fill up long before their earliest events: the
    # wavefront kernel stops a full column partway through the schedule (a
    # ragged last column among them); with saturation on and off, resident
    # and streamed, against the oracle
    ctx = tn.get_context()
    cases = [(129, 30_000, 3_000, 91), (700, 60_000, 6_000, 92), (2500, 120_000, 12_000, 93)]
    try:
        for n, m, Tm, seed in cases:
            s, d, t = T.activity_driven(n, m, Tm, seed=seed)
            want = oracle.reverse_matrix(n, s, d, t)
            assert (oracle.sizes(want, n)[0] == n).all(), n  # every row fills up
            st = tn.host_schedule(n, s, d, t)["stats"]
            assert st["ops"] <= 640 * st["op_levels"] and st["ops"] > 4096, n
            for sat in (True, False):
                ctx.saturation(sat)
                assert (gpu_matrix(n, s, d, t) == want).all(), (n, sat)
                C, _ = tn.build_component_matrix_streamed(n, s, d, t, chunk_events=m // 5)
                assert (host(C)[:, :oracle.words(n)] == want).all(), (n, sat)
    finally:
        ctx.saturation(True)


@pytest.mark.parametrize("sw", [1, 2, 4, 8, 16])
def test_saturating_path_with_a_forwarding_phase(sw):
    # n = 256 * 64 + 1: every slice width ends on a one-column slice.  Past
    # the zero phase, a network of this size runs the forwarding kernel until
    # its ops reach 9 n, then the saturating kernel from slice state rebuilt
    # out of the matrix, on one-word slices in a grid of its own (257
    # workgroups, against 17..257 before) and the slices with the most rows
    # still not full first; compound scratch rows live across that cut
    # (test_planner).  The matrix must be the plain recurrence's and the
    # oracle's
    n = 16385
    s, d, t = T.uniform_pairs(n, 400_000, 2000, seed=8400)
    sch = tn.host_schedule(n, s, d, t)
    lv, L = sch["lvl_op"], sch["stats"]["op_levels"]
    zl = int(np.searchsorted(lv[:L], n, side="left"))
    mid = int(np.searchsorted(lv[:L], 9 * n, side="left"))
    assert 0 < zl < mid < L
    ctx = tn.get_context()
    p = tn.Plan(n, s, d, t)
    try:
        C1 = p.execute(slice_words=sw).clone()
        ld1, _ = ctx.last_traffic()
        ctx.saturation(False)
        C0 = p.execute(slice_words=sw)
        ld0, _ = ctx.last_traffic()
    finally:
        ctx.saturation(True)
        p.close()
    assert torch.equal(C1, C0)
    assert ld1 < ld0
    got = host(C1)
    nw = oracle.words(n)
    for w0 in (0, 130, nw - 1):
        want = oracle.reverse_matrix(n, s, d, t, w0=w0, nw=1)
        assert (got[:, w0:w0 + 1] == want).all(), (sw, w0)


@pytest.mark.parametrize("sw", [2, 8])
def test_saturating_path_on_two_blocks(sw):
    # the same three launches on a network whose matrix never fills: events
    # only among the even and among the odd nodes.  Where the matrix ends all
    # ones, a row-OR that read a wrong row (say a scratch row looked up at
    # another place after the forwarding phase) only saturates sooner; here
    # any bit across the blocks is an error
    n = 16385
    s, d, t = T.two_block_pairs(n, 600_000, 2000, seed=8410)
    sch = tn.host_schedule(n, s, d, t)
    lv, L = sch["lvl_op"], sch["stats"]["op_levels"]
    zl = int(np.searchsorted(lv[:L], n, side="left"))
    mid = int(np.searchsorted(lv[:L], 9 * n, side="left"))
    assert 0 < zl < mid < L
    ctx = tn.get_context()
    p = tn.Plan(n, s, d, t)
    try:
        C1 = p.execute(slice_words=sw).clone()
        ctx.saturation(False)
        C0 = p.execute(slice_words=sw)
    finally:
        ctx.saturation(True)
        p.close()
    assert torch.equal(C1, C0)
    got = host(C1)
    nw = oracle.words(n)
    even = np.uint64(0x5555555555555555)  # the even columns of a word
    assert not (got[0::2, :nw] & ~even).any() and not (got[1::2, :nw] & even).any()
    for w0 in (0, 131, nw - 1):
        want = oracle.reverse_matrix(n, s, d, t, w0=w0, nw=1)
        assert (got[:, w0:w0 + 1] == want).all(), (sw, w0)


def _partial_network(n, m, word, seed):
    # directed events; the nodes of one word column never receive, so no
    # other node reaches them: that column never fills, every other one does
    s, d, t = T.uniform_pairs(n, m, 2000, seed=seed)
    s, d = s.astype(np.int64), d.astype(np.int64)
    bad = (d >= 64 * word) & (d < 64 * (word + 1))
    d[bad] = (d[bad] + 64 * 7) % n
    keep = s != d
    return n, s[keep].astype(np.uint32), d[keep].astype(np.uint32), t[keep], tn.DIRECTED


@pytest.mark.parametrize("case", ["partial", "two_blocks", "small_partial"])
def test_sizes_from_the_slice_state(case):
    # tn_plan_execute_sizes counts the columns of slices that the execution
    # left all ones from its slice state, without reading them.  Through the
    # three-phase path (last launch on one-word slices): a network where all
    # but one word column fill (256 of 257 slices counted from the state) and
    # one where no slice fills (two blocks); through the two launches of a
    # smaller network, 4-word slices with all but one filled
    if case == "partial":
        n, s, d, t, flags = _partial_network(16385, 500_000, 100, 8420)
        widths = (0, 2, 8)
    elif case == "small_partial":
        n, s, d, t, flags = _partial_network(8001, 400_000, 50, 8430)
        widths = (0, 4)
    else:
        n = 16385
        s, d, t = T.two_block_pairs(n, 600_000, 2000, seed=8410)
        flags = 0
        widths = (0, 2, 8)
    want = oracle.reverse_matrix(n, s, d, t, **flag_kw(flags))
    nw = oracle.words(n)
    full = np.full(nw, np.uint64(0xFFFFFFFFFFFFFFFF))
    full[-1] = np.uint64((1 << (n % 64)) - 1)
    filled = int((want[:, :nw] == full[None, :]).all(axis=0).sum())
    assert filled == (0 if case == "two_blocks" else nw - 1)
    wo, wi = oracle.sizes(want, n)
    p = tn.Plan(n, s, d, t, flags)
    try:
        for sw in widths:
            C, out, inn = p.execute_sizes(slice_words=sw)
            assert (host(C)[:, :nw] == want).all(), (case, sw)
            assert (out.cpu().numpy() == wo).all(), (case, sw)
            assert (inn.cpu().numpy() == wi).all(), (case, sw)
    finally:
        p.close()


def test_full_size_sizes_from_the_slice_state(c2):
    # at n = 10^5 every slice ends all ones: the sizes come from the state
    # alone, and equal the ones counted from the matrix
    C, out, inn = c2["plan"].execute_sizes()
    assert torch.equal(C, c2["C"])
    o2, i2 = tn.component_sizes(C, 100_000)
    assert torch.equal(out, o2) and torch.equal(inn, i2)
    assert (out == 100_000).all() and (inn == 100_000).all()
