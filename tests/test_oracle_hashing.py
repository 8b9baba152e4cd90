"""Pins of the oracle's hash family (Sec. 4.1), hashed proxies and
recombination (Sec. 4.2): exact big-integer arithmetic, closed forms of the
polynomial, universality statistics, brute force with Python sets from the
definitions, and the estimator's stated properties."""
import math

import numpy as np
import pytest

import oracle
import tn_inputs as T
from oracle import si

P61 = (1 << 61) - 1


def test_multaddmod_exact_against_big_integers():
    g = T.rng(1)
    vals = [0, 1, 2, P61 - 1, P61 - 2, (1 << 32) - 1, 1 << 32, (1 << 33) - 2]
    vals += [int(x) for x in g.integers(0, P61, 200, dtype=np.uint64)]
    for i in range(len(vals)):
        x = vals[i] % (1 << 34)  # characters are at most 33 bits
        acc = vals[(i * 7 + 3) % len(vals)]
        a = vals[(i * 13 + 5) % len(vals)]
        assert oracle.multaddmod(x, acc, a) == (x * acc + a) % P61


def test_polynomial_closed_forms():
    A = T.hash_coefficients(4, seed=3)  # (H, 3, 4)
    for j in range(4):
        for i in range(3):
            Ai = A[j, i]
            # acc starts at A(i,0) and folds A(i,1..3): the constant term is A(i,3)
            assert oracle.poly(Ai, 0) == int(Ai[3]) % P61
            assert oracle.poly(Ai, 1) == sum(int(a) for a in Ai) % P61
            x = 12345 + 17 * j
            p = [oracle.poly(Ai, x + k) for k in range(5)]
            # third finite difference of a cubic is 3! times its leading coefficient
            d3 = (p[3] - 3 * p[2] + 3 * p[1] - p[0]) % P61
            assert d3 == (6 * int(Ai[0])) % P61
            d4 = sum((-1) ** k * math.comb(4, k) * p[k] for k in range(5)) % P61
            assert d4 == 0


def test_hash_uses_low_high_and_sum_characters():
    A = T.hash_coefficients(1, seed=4)[0]
    for u in [0, 1, 77, (1 << 32) - 1, (1 << 32) + 5, (3 << 32) + 9]:
        x0, x1 = u & 0xFFFFFFFF, u >> 32
        expect = oracle.poly(A[0], x0) ^ oracle.poly(A[1], x1) ^ oracle.poly(A[2], x0 + x1)
        assert oracle.hash_raw(A, u) == expect


def test_bucket_uniformity_chi_square():
    n, K = 200_000, 64
    b = oracle.hash_nodes(n, T.hash_coefficients(3, seed=5), K)
    for j in range(3):
        cnt = np.bincount(b[j], minlength=K)
        e = n / K
        chi2 = float(((cnt - e) ** 2 / e).sum())
        # 63 degrees of freedom: the 1e-6 upper quantile is about 135
        assert chi2 < 135, chi2


def test_pairwise_and_fourwise_independence_statistics():
    K, draws = 4, 6000
    A = T.hash_coefficients(draws, seed=6)
    keys = [3, 1000, 77777, 123456789]
    hv = np.array([[oracle.hash_raw(A[d], k) % K for k in keys] for d in range(draws)])
    coll = np.mean(hv[:, 0] == hv[:, 1])
    assert abs(coll - 1 / K) < 4 * math.sqrt((1 / K) * (1 - 1 / K) / draws)
    pattern = np.mean((hv[:, 0] == 0) & (hv[:, 1] == 1) & (hv[:, 2] == 2) & (hv[:, 3] == 3))
    p = 1 / K ** 4
    assert abs(pattern - p) < 5 * math.sqrt(p * (1 - p) / draws)


def test_hashing_is_deterministic():
    A = T.hash_coefficients(2, seed=7)
    assert (oracle.hash_nodes(1000, A, 100) == oracle.hash_nodes(1000, A, 100)).all()
    assert (T.hash_coefficients(2, seed=7) == A).all()


def _brute_estimate(n, K, s, d, t, bucket):
    """Eq. DefEstOCMerge from sets: OCs of the hashed networks by SI brute force."""
    H = bucket.shape[0]
    inv = [[set(np.nonzero(bucket[j] == r)[0]) for r in range(K)] for j in range(H)]
    ocs = [si.out_components(K, bucket[j][s], bucket[j][d], t) for j in range(H)]
    est = []
    for u in range(n):
        acc = None
        for j in range(H):
            lifted = set()
            for x in ocs[j][bucket[j][u]]:
                lifted |= inv[j][x]
            acc = lifted if acc is None else acc & lifted
        est.append(len(acc))
    return np.array(est)


def test_recombine_matches_set_brute_force():
    for case in range(12):
        n, K, H = 14 + case, 5 + case % 4, 1 + case % 3
        s, d, t = T.random_tiny(n, 30, 10, seed=500 + case)
        bucket = oracle.hash_nodes(n, T.hash_coefficients(H, seed=600 + case), K)
        P = oracle.proxies(K, s, d, t, bucket)
        est, lifted = oracle.recombine(n, P, bucket)
        assert (est == _brute_estimate(n, K, s, d, t, bucket)).all()


def test_estimator_properties():
    n, K, H = 300, 40, 6
    s, d, t = T.uniform_pairs(n, 500, 400, seed=21)
    exact = oracle.row_counts(oracle.reverse_matrix(n, s, d, t))
    A = T.hash_coefficients(H, seed=22)
    bucket = oracle.hash_nodes(n, A, K)
    P = oracle.proxies(K, s, d, t, bucket)
    est, lifted = oracle.recombine(n, P, bucket)
    assert (exact <= est).all()                       # superset property (Sec. 4.2)
    assert (est <= lifted.min(axis=0)).all()
    assert (lifted <= n).all() and (est >= 1).all()
    prev = None
    for h in range(1, H + 1):                          # nested hashes never grow the estimate
        e, _ = oracle.recombine(n, P[:h], bucket[:h])
        if prev is not None:
            assert (e <= prev).all()
        prev = e
    # lifted size = sum of |h^{-1}(r)| over the super-nodes r in the proxy row
    cnt = oracle.bucket_counts(bucket, K)
    for j in range(H):
        Dj = oracle.to_dense(P[j], K)
        assert (lifted[j] == (Dj[bucket[j]] * cnt[j][None, :]).sum(axis=1)).all()


def test_proxy_is_homomorphic_image():
    n, K = 250, 30
    s, d, t = T.activity_driven(n, 1500, 200, seed=31)
    C = oracle.to_dense(oracle.reverse_matrix(n, s, d, t), n)
    bucket = oracle.hash_nodes(n, T.hash_coefficients(3, seed=32), K)
    P = oracle.proxies(K, s, d, t, bucket)
    for j in range(3):
        Pj = oracle.to_dense(P[j], K)
        u, w = np.nonzero(C)
        assert Pj[bucket[j][u], bucket[j][w]].all()


def test_identity_hash_is_exact_and_single_bucket_is_everything():
    n = 90
    s, d, t = T.uniform_pairs(n, 150, 60, seed=41)
    exact = oracle.row_counts(oracle.reverse_matrix(n, s, d, t))
    ident = np.arange(n, dtype=np.uint32)[None, :]
    est, _ = oracle.recombine(n, oracle.proxies(n, s, d, t, ident), ident)
    assert (est == exact).all()
    one = np.zeros((2, n), dtype=np.uint32)
    est1, _ = oracle.recombine(n, oracle.proxies(1, s, d, t, one), one)
    assert (est1 == n).all()


def _hash_by_big_integers(A, u):
    # Sec. 4.1 written out as plain polynomials: T_i(x) = A_i0 x^3 + A_i1 x^2 +
    # A_i2 x + A_i3 mod (2^61 - 1), characters x0 = low 32 bits, x1 = high 32
    # bits, x2 = x0 + x1, and the three table values XORed.
    def T_(row, x):
        return sum(int(row[l]) * x ** (3 - l) for l in range(4)) % P61
    x0, x1 = u & 0xFFFFFFFF, u >> 32
    return T_(A[0], x0) ^ T_(A[1], x1) ^ T_(A[2], x0 + x1)


def test_hash_nodes_each_table_and_modulus_against_big_integers():
    # every hash j must use its own table (stride of 3 x order entries) and the
    # reduction mod K; shared or shifted tables would pass the statistics above
    H, n = 5, 2500
    A = T.hash_coefficients(H, seed=91)
    assert len({A[j].tobytes() for j in range(H)}) == H
    raw = [[_hash_by_big_integers(A[j], u) for u in range(n)] for j in range(H)]
    for K in (1, 7, 1000, 4096, 65536):
        b = oracle.hash_nodes(n, A, K)
        want = np.array([[r % K for r in raw[j]] for j in range(H)], dtype=np.uint32)
        assert (b == want).all(), K
    # the tables really give different maps (a shared table would repeat rows)
    b = oracle.hash_nodes(n, A, 4096)
    for j in range(1, H):
        assert (b[j] != b[0]).mean() > 0.9


def test_hash_raw_against_big_integers_above_32_bits():
    A = T.hash_coefficients(3, seed=92)
    for j in range(3):
        for u in (0, 5, (1 << 32) - 1, 1 << 32, (1 << 32) + 77, (5 << 32) + 3, (1 << 40) + 11):
            assert oracle.hash_raw(A[j], u) == _hash_by_big_integers(A[j], u)
