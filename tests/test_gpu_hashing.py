"""GPU parity of network hashing (Sec. 4.1), the hashed proxies built in one
batched launch (Sec. 4.3) and the fusion estimator (Sec. 4.2) against the CPU
oracle; bit-exact buckets, proxies and estimates."""
import numpy as np
import pytest
import torch

import oracle
import tn_inputs as T
from gpu_util import host

pytestmark = pytest.mark.gpu

tn = pytest.importorskip("paper_2307_04890_amd")


def run_hashed(n, s, d, t, H, K, seed, flags=0):
    A = T.hash_coefficients(H, seed=seed)
    bucket, count, proxies = tn.hash_compress(n, s, d, t, A, K, flags=flags)
    ldK = oracle.words(K)
    P = torch.empty((H, K, ldK), dtype=torch.int64, device="cuda")
    proxies.execute([P[j] for j in range(H)])
    est, lifted = tn.recombine(P, bucket, count, n)
    torch.cuda.synchronize()
    return A, bucket.cpu().numpy().view(np.uint32), count.cpu().numpy(), host(P), \
        est.cpu().numpy(), lifted.cpu().numpy(), proxies


@pytest.mark.parametrize("n,m,H,K,mixed", [(300, 900, 3, 40, False), (2000, 8000, 4, 64, False),
                                           (5000, 30000, 5, 1500, False),
                                           (3000, 12000, 2, 4096, False), (2000, 300, 2, 64, True),
                                           (3000, 250, 2, 40, True),
                                           # odd K: tables staged in 4-byte units; H = 5
                                           # leaves a group of one hash
                                           (1200, 4000, 3, 45, False), (2500, 6000, 5, 999, False),
                                           # two copies of one hash's tables in LDS (the next
                                           # chunk streams in while one is read); one copy
                                           (2500, 10000, 3, 7000, False),
                                           (2000, 8000, 2, 16000, False),
                                           # tables too large for LDS: read from global memory
                                           (1500, 3000, 2, 32768, False)])
def test_hash_proxies_and_recombine_match_oracle(n, m, H, K, mixed):
    Tm = m if mixed else m // 3
    s, d, t = T.uniform_pairs(n, m, Tm, seed=n + K)
    A, bucket, count, P, est, lifted, _ = run_hashed(n, s, d, t, H, K, seed=K)
    wb = oracle.hash_nodes(n, A, K)
    assert (bucket == wb).all()
    assert (count == oracle.bucket_counts(wb, K)).all()
    WP = oracle.proxies(K, s, d, t, wb)
    assert (P == WP).all()
    us = np.arange(n) if n <= 2000 else T.rng(1).choice(n, 300, replace=False)
    we, wl = oracle.recombine(n, WP, wb, us)
    if mixed:
        # a mix of nodes whose proxy rows are full in every hash (estimate n)
        # and nodes that need the AND over all chunks
        assert (we == n).any() and (we < n).any()
    assert (est[us] == we).all()
    assert (lifted[:, us] == wl).all()


def test_estimator_properties_against_exact_gpu_path():
    n, m, H, K = 6000, 15000, 8, 300
    s, d, t = T.activity_driven(n, m, 2000, seed=12)
    A, bucket, count, P, est, lifted, _ = run_hashed(n, s, d, t, H, K, seed=13)
    C = tn.build_component_matrix(n, s, d, t)
    exact, _ = tn.component_sizes(C, n, inn=False)
    exact = exact.cpu().numpy()
    assert (exact <= est).all()                 # superset property (Sec. 4.2)
    assert (est <= lifted.min(axis=0)).all() and (lifted <= n).all()
    assert (est >= 1).all()


def test_identity_and_single_bucket_maps():
    n = 700
    s, d, t = T.uniform_pairs(n, 1200, 500, seed=3)
    C = tn.build_component_matrix(n, s, d, t)
    exact, _ = tn.component_sizes(C, n, inn=False)
    ident = torch.arange(n, dtype=torch.int32, device="cuda")[None, :].contiguous()
    cnt = torch.ones((1, n), dtype=torch.int32, device="cuda")
    est, lifted = tn.recombine(C[None].contiguous(), ident, cnt, n)
    assert (est == exact).all() and (lifted[0] == exact).all()
    P1 = torch.ones((2, 1, 1), dtype=torch.int64, device="cuda")
    zero = torch.zeros((2, n), dtype=torch.int32, device="cuda")
    cnt1 = torch.full((2, 1), n, dtype=torch.int32, device="cuda")
    est1, lifted1 = tn.recombine(P1, zero, cnt1, n)
    assert (est1 == n).all() and (lifted1 == n).all()


def test_hashed_directed_and_sequential():
    n, m, H, K = 1500, 5000, 3, 100
    s, d, t = T.random_tiny(n, m, 800, seed=9)
    for flags in (1, 2):
        A, bucket, count, P, est, lifted, _ = run_hashed(n, s, d, t, H, K, seed=flags, flags=flags)
        WP = oracle.proxies(K, s, d, t, oracle.hash_nodes(n, A, K), directed=bool(flags & 1),
                            sequential=bool(flags & 2))
        assert (P == WP).all()


def test_activity_driven_scaled_hashed_workload():
    # the shape of the n = 10^6, m = 10^8, H = 16, K = 4096 workload at 1/20 of the events
    n, m, H, K = 200_000, 5_000_000, 16, 4096
    s, d, t = T.activity_driven(n, m, 500_000, seed=3)
    A, bucket, count, P, est, lifted, proxies = run_hashed(n, s, d, t, H, K, seed=1003)
    wb = oracle.hash_nodes(n, A, K)
    assert (bucket == wb).all()
    for j in (0, 7):
        assert (P[j] == oracle.reverse_matrix(K, wb[j][s], wb[j][d], t)).all(), j
    us = T.rng(5).choice(n, 64, replace=False)
    we, wl = oracle.recombine(n, P, wb, us)
    assert (est[us] == we).all() and (lifted[:, us] == wl).all()
    stats, tiles, lds_tiles = proxies.stats()
    assert lds_tiles == tiles  # K = 4096 proxies are LDS-resident


def test_hash_errors():
    with pytest.raises(tn.TNError) as e:
        tn.hash_compress(10, [0], [1], [0], T.hash_coefficients(2, 1), 70000)
    assert e.value.code == -6
    bad = T.hash_coefficients(1, 1)
    bad[0, 0, 0] = (1 << 61) - 1
    with pytest.raises(tn.TNError) as e:
        tn.hash_compress(10, [0], [1], [0], bad, 8)
    assert e.value.code == -1


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_streamed_proxies_equal_the_batched_proxies(flags):
    # the streamed build (chunks, resume from the proxies in HBM, stop once
    # every tile is full) against the one-launch batch and the oracle
    cases = [(2000, 8000, 4, 64, 2000, 500), (3000, 60000, 3, 100, 6000, 4096),
             (1500, 5000, 2, 4096, 800, 700), (500, 0, 2, 50, 1, 0)]
    for case, (n, m, H, K, Tm, chunk) in enumerate(cases):
        s, d, t = T.random_tiny(n, max(m, 1), max(Tm, 1), seed=400 + case)
        s, d, t = s[:m], d[:m], t[:m]
        A = T.hash_coefficients(H, seed=40 + case)
        bucket, count, P, st = tn.hash_build_proxies(n, s, d, t, A, K, flags=flags,
                                                     chunk_events=chunk)
        wb = oracle.hash_nodes(n, A, K)
        assert (bucket.cpu().numpy().view(np.uint32) == wb).all()
        WP = oracle.proxies(K, s, d, t, wb, directed=bool(flags & 1), sequential=bool(flags & 2))
        assert (host(P) == WP).all(), case
        assert st["chunks_run"] <= st["chunks"]
        if case == 1 and flags == 0:
            assert st["saturated"] == 1 and st["chunks_run"] < st["chunks"]


@pytest.mark.parametrize("flags", [0, 3])
def test_streamed_proxies_on_both_sides_of_the_wavefront_limit(flags):
    # proxies of at most 4096 super-nodes run one wavefront per word column,
    # larger ones as batched tiles: both, over several chunks, with and
    # without saturation tracking, and with a padded row stride
    n, m, H = 9000, 40000, 3
    s, d, t = T.activity_driven(n, m, 4000, seed=77)
    ctx = tn.get_context()
    try:
        for K in (4095, 4096, 4097):
            A = T.hash_coefficients(H, seed=K)
            wb = oracle.hash_nodes(n, A, K)
            WP = oracle.proxies(K, s, d, t, wb, directed=bool(flags & 1), sequential=bool(flags & 2))
            for sat in (True, False):
                ctx.saturation(sat)
                ld = oracle.words(K) + (1 if sat else 0)
                P = torch.full((H, K, ld), -1, dtype=torch.int64, device="cuda")
                _, _, P, st = tn.hash_build_proxies(n, s, d, t, A, K, flags=flags,
                                                    chunk_events=7000, P=P)
                got = host(P)
                # host() also checks that the padding word is written as 0
                assert (got == WP).all(), (K, sat)
                assert st["chunks"] > 1 and st["slice_words"] >= 1
    finally:
        ctx.saturation(True)


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_streamed_small_proxies_edge_shapes(flags):
    # the wavefront path at its smallest shapes: one super-node, one hash,
    # a ragged second word column (K = 65), a single time step, many ties
    cases = [(300, 2000, 1, 1, 50), (400, 3000, 1, 65, 3), (250, 1500, 4, 65, 1),
             (600, 4000, 2, 127, 40)]
    for n, m, H, K, Tm in cases:
        s, d, t = T.random_tiny(n, m, Tm, seed=n + K + flags)
        A = T.hash_coefficients(H, seed=K + 10 * flags)
        _, _, P, st = tn.hash_build_proxies(n, s, d, t, A, K, flags=flags, chunk_events=m // 3)
        WP = oracle.proxies(K, s, d, t, oracle.hash_nodes(n, A, K), directed=bool(flags & 1),
                            sequential=bool(flags & 2))
        assert (host(P) == WP).all(), (n, H, K, flags)
        assert st["slice_words"] == 1, (n, H, K)


def test_streamed_proxies_of_few_super_nodes():
    # ER networks with Poisson events at the paper's n_s = 0.3 n and H = 5,
    # tiny proxies (fewer super-nodes than a word, or exactly one word) over
    # several chunks, with saturation on and off; the rare
    # simultaneous events make a few compound steps in every chunk
    ctx = tn.get_context()
    try:
        for n, K, m in [(60, 18, 20_000), (150, 45, 60_000), (210, 63, 90_000), (220, 64, 90_000)]:
            s, d, t = T.er_poisson(n, m, 100 * m, seed=n)
            A = T.hash_coefficients(5, seed=K)
            WP = oracle.proxies(K, s, d, t, oracle.hash_nodes(n, A, K))
            for sat in (True, False):
                ctx.saturation(sat)
                _, _, P, st = tn.hash_build_proxies(n, s, d, t, A, K, chunk_events=m // 4)
                assert (host(P) == WP).all(), (n, K, sat)
                assert st["chunks_run"] >= 1
    finally:
        ctx.saturation(True)


def test_streamed_proxies_at_the_scaled_hashed_workload():
    n, m, H, K = 200_000, 5_000_000, 16, 4096
    s, d, t = T.activity_driven(n, m, 500_000, seed=3)
    A = T.hash_coefficients(H, seed=1003)
    bucket, count, P, st = tn.hash_build_proxies(n, s, d, t, A, K)
    wb = oracle.hash_nodes(n, A, K)
    for j in (0, 9):
        assert (host(P[j]) == oracle.reverse_matrix(K, wb[j][s], wb[j][d], t)).all(), j
    assert st["saturated"] == 1 and st["events_run"] < m


def test_paper_setting_er_poisson_exact_and_hashed():
    # G(n, 2/n) with a Poisson process per link, n_s = 0.3 n, H = 5
    n, m, H = 300, 20_000, 5
    K = 90
    s, d, t = T.er_poisson(n, m, 100 * m, seed=11)
    C = tn.build_component_matrix(n, s, d, t)
    want = oracle.reverse_matrix(n, s, d, t)
    assert (host(C) == want).all()
    A = T.hash_coefficients(H, seed=12)
    bucket, count, P, _ = tn.hash_build_proxies(n, s, d, t, A, K)
    wb = oracle.hash_nodes(n, A, K)
    WP = oracle.proxies(K, s, d, t, wb)
    assert (host(P) == WP).all()
    est, lifted = tn.recombine(P, bucket, count, n)
    we, wl = oracle.recombine(n, WP, wb)
    assert (est.cpu().numpy() == we).all() and (lifted.cpu().numpy() == wl).all()


@pytest.mark.parametrize("flags", [0, 1])
def test_streamed_small_proxies_with_a_time_step_over_every_bucket(flags):
    # one time step whose mapped events join nearly all of K = 4096
    # super-nodes: a compound item of more than 1024 targets inside a chunk
    # of the wavefront path (its last target folds in place, so the chunk's
    # scratch rows still fit beside the K rows in LDS)
    n, H, K = 20000, 2, 4096
    g = T.rng(31)
    s1, d1, t1 = T.uniform_pairs(n, 4000, 400, seed=32)
    s2 = g.integers(0, n, 30000).astype(np.uint32)
    d2 = ((s2.astype(np.int64) + 1 + g.integers(0, n - 1, 30000)) % n).astype(np.uint32)
    t2 = np.full(30000, 400, dtype=np.int64)
    s3, d3, t3 = T.uniform_pairs(n, 4000, 400, seed=33)
    s = np.concatenate([s1, s2, s3])
    d = np.concatenate([d1, d2, d3])
    t = np.concatenate([t1, t2, t3 + 401])
    A = T.hash_coefficients(H, seed=34)
    wb = oracle.hash_nodes(n, A, K)
    sch = tn.host_schedule(K, wb[0][s], wb[0][d], t, flags)
    assert 1024 < sch["stats"]["scratch_rows"] <= K - 1
    WP = oracle.proxies(K, s, d, t, wb, directed=bool(flags & 1))
    _, _, P, st = tn.hash_build_proxies(n, s, d, t, A, K, flags=flags, chunk_events=1500)
    assert (host(P) == WP).all()
    assert st["chunks"] > 2
