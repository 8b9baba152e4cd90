"""Pins of the CPU oracle's component matrix against facts fixed by the paper and
by mathematics (brute force, closed forms, a library BFS, invariants)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
import tn_inputs as T
from oracle import si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_rev(n, s, d, t, **kw):
    return oracle.to_dense(oracle.reverse_matrix(n, s, d, t, **kw), n)


def read_golden(name):
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.isalpha():
                cur = line
                sections[cur] = []
                continue
            sections[cur].append([int(x) for x in line.split()])
    return sections


def test_golden_five_node_ties():
    g = read_golden("five_node_ties.txt")
    ev = np.array(g["events"], dtype=np.int64)
    s, d, t = ev[:, 0].astype(np.uint32), ev[:, 1].astype(np.uint32), ev[:, 2]
    for mode, seq in (("strict", False), ("sequential", True)):
        D = dense_rev(5, s, d, t, sequential=seq)
        for row in g[mode]:
            u, members = row[0], set(row[1:])
            assert set(np.nonzero(D[u])[0]) == members, (mode, u)


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("sequential", [False, True])
def test_matches_si_brute_force(directed, sequential):
    for case in range(150):
        n = 2 + case % 9
        m = case % 37
        Tmax = 1 + case % 6  # few time steps: many ties
        s, d, t = T.random_tiny(n, m, Tmax, seed=1000 + case, allow_self=(case % 5 == 0))
        D = dense_rev(n, s, d, t, directed=directed, sequential=sequential)
        oc = si.out_components(n, s, d, t, directed=directed, sequential=sequential)
        for u in range(n):
            assert set(np.nonzero(D[u])[0]) == oc[u], (case, u)


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("sequential", [False, True])
def test_transpose_of_forward_algorithm(directed, sequential):
    for case in range(60):
        n = 3 + case % 70
        s, d, t = T.random_tiny(n, 4 * n, 1 + case % 20, seed=2000 + case)
        C = dense_rev(n, s, d, t, directed=directed, sequential=sequential)
        S = oracle.to_dense(oracle.forward_matrix(n, s, d, t, directed=directed,
                                                  sequential=sequential), n)
        assert (C == S.T).all()


def test_no_events_is_identity():
    for n in (1, 5, 64, 65, 130):
        D = dense_rev(n, [], [], [])
        assert (D == np.eye(n, dtype=bool)).all()


def test_single_event():
    n = 100
    D = dense_rev(n, [3], [77], [5])
    E = np.eye(n, dtype=bool)
    E[3, 77] = E[77, 3] = True
    assert (D == E).all()
    Dd = dense_rev(n, [3], [77], [5], directed=True)
    E = np.eye(n, dtype=bool)
    E[3, 77] = True
    assert (Dd == E).all()


@pytest.mark.parametrize("directed", [False, True])
def test_one_time_step_is_identity_plus_adjacency(directed):
    n = 90
    g = T.rng(5)
    m = 400
    s = g.integers(0, n, m).astype(np.uint32)
    d = g.integers(0, n, m).astype(np.uint32)
    t = np.zeros(m, dtype=np.int64)
    A = np.eye(n, dtype=bool)
    A[s, d] = True
    if not directed:
        A[d, s] = True
    assert (dense_rev(n, s, d, t, directed=directed) == A).all()


@pytest.mark.parametrize("rounds", [1, 2, 3, 5])
def test_static_graph_rounds_are_bfs_balls(rounds):
    n = 120
    (a, b), (s, d, t) = T.static_graph_rounds(n, 150, rounds, seed=rounds)
    G = sp.coo_matrix((np.ones(a.shape[0]), (a, b)), shape=(n, n))
    dist = shortest_path(G, directed=False, unweighted=True)
    assert (dense_rev(n, s, d, t) == (dist <= rounds)).all()


def test_chronological_path_closed_form():
    k = 70
    s, d, t = T.chronological_path(k)
    D = dense_rev(k + 1, s, d, t)
    for i in range(k + 1):
        expect = set(range(k + 1)) if i == 0 else set(range(i - 1, k + 1))
        assert set(np.nonzero(D[i])[0]) == expect


def test_four_cycle_tie_group_does_not_chain():
    # a-b-c-d-a at one time step: each node reaches exactly its two neighbours
    s = np.array([0, 1, 2, 3], dtype=np.uint32)
    d = np.array([1, 2, 3, 0], dtype=np.uint32)
    D = dense_rev(4, s, d, np.zeros(4, dtype=np.int64))
    for u in range(4):
        assert set(np.nonzero(D[u])[0]) == {u, (u + 1) % 4, (u + 3) % 4}


def test_strict_equals_sequential_on_distinct_times():
    for case in range(20):
        n = 10 + case
        g = T.rng(300 + case)
        m = 5 * n
        s = g.integers(0, n, m).astype(np.uint32)
        d = g.integers(0, n, m).astype(np.uint32)
        t = np.arange(m, dtype=np.int64)
        for directed in (False, True):
            a = oracle.reverse_matrix(n, s, d, t, directed=directed)
            b = oracle.reverse_matrix(n, s, d, t, directed=directed, sequential=True)
            assert (a == b).all()


def test_invariants_diagonal_tail_and_eq1():
    for case, (n, m, Tm) in enumerate([(1000, 2000, 10_000), (257, 3000, 50), (64, 100, 3)]):
        s, d, t = T.uniform_pairs(n, m, Tm, seed=40 + case)
        C = oracle.reverse_matrix(n, s, d, t)
        D = oracle.to_dense(C, n)
        assert D.diagonal().all()
        tail = oracle.to_dense(C, 64 * C.shape[1])[:, n:]
        assert not tail.any()
        out, inn = oracle.sizes(C, n)
        assert out.sum() == inn.sum() == D.sum()  # Eq. (1): the sums interchange
        assert (out >= 1).all() and (out <= n).all() and (inn >= 1).all()


def test_adding_events_never_clears_bits():
    n = 200
    s, d, t = T.uniform_pairs(n, 600, 100, seed=9)
    full = dense_rev(n, s, d, t)
    g = T.rng(10)
    for _ in range(5):
        keep = g.random(s.shape[0]) < 0.6
        sub = dense_rev(n, s[keep], d[keep], t[keep])
        assert not (sub & ~full).any()


def test_column_slices_concatenate():
    n = 700
    s, d, t = T.activity_driven(n, 5000, 300, seed=11)
    full = oracle.reverse_matrix(n, s, d, t)
    nw = full.shape[1]
    parts = [oracle.reverse_matrix(n, s, d, t, w0=w0, nw=min(3, nw - w0))
             for w0 in range(0, nw, 3)]
    assert (np.concatenate(parts, axis=1) == full).all()
    fwd_full = oracle.forward_matrix(n, s, d, t)
    fwd_part = oracle.forward_matrix(n, s, d, t, w0=4, nw=2)
    assert (fwd_full[:, 4:6] == fwd_part).all()


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.reverse_matrix(5, [0], [5], [0])
    with pytest.raises(ValueError):
        oracle.reverse_matrix(5, [0, 1], [1, 2], [3, 2])


def _dense_by_unpackbits(M, n_cols):
    # numpy's own bit unpacking, little-endian within each byte: column b is
    # bit b & 63 of word b >> 6
    bits = np.unpackbits(np.ascontiguousarray(M).view(np.uint8), axis=1, bitorder="little")
    return bits[:, :n_cols].astype(np.int64)


def test_col_counts_hand_placed_bits_at_word_edges():
    # Sec. 3.1: the in-component size of w is the number of rows holding bit w.
    # Bits at the first and last position of a word and in the next word catch
    # a wrong bit order or word offset, which leave the column total unchanged.
    nw = 3
    M = np.zeros((4, nw), dtype=np.uint64)
    placed = {0: [0, 63, 64, 130], 1: [63, 64, 191], 2: [64, 65, 130], 3: [1, 130]}
    for row, cols in placed.items():
        for b in cols:
            M[row, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    want = np.zeros(64 * nw, dtype=np.int64)
    for cols in placed.values():
        for b in cols:
            want[b] += 1
    assert (oracle.col_counts(M) == want).all()
    assert (oracle.row_counts(M) == [len(placed[r]) for r in range(4)]).all()


def test_col_and_row_counts_per_column_against_numpy_bits():
    g = T.rng(71)
    for n_rows, nw in ((1, 1), (37, 2), (200, 5)):
        M = g.integers(0, 2 ** 63, size=(n_rows, nw), dtype=np.uint64)
        M ^= g.integers(0, 2, size=(n_rows, nw), dtype=np.uint64) << np.uint64(63)
        D = _dense_by_unpackbits(M, 64 * nw)
        assert (oracle.col_counts(M) == D.sum(axis=0)).all()
        assert (oracle.row_counts(M) == D.sum(axis=1)).all()


def test_in_sizes_per_column_equal_forward_rows_and_si():
    # Sec. 3.4: the reverse-time matrix is the transpose of forward Algorithm 1's,
    # so column w's count (w's in-component) is row w's count of the forward
    # matrix; SI brute force from every source gives the same per-column count.
    for case, (n, m, Tm, directed) in enumerate([(150, 900, 60, False), (131, 700, 40, True),
                                                 (65, 300, 20, False)]):
        s, d, t = T.uniform_pairs(n, m, Tm, seed=80 + case)
        C = oracle.reverse_matrix(n, s, d, t, directed=directed)
        S = oracle.forward_matrix(n, s, d, t, directed=directed)
        inn = oracle.col_counts(C, n)
        assert (inn == oracle.row_counts(S)).all()
        assert (inn == _dense_by_unpackbits(C, n).sum(axis=0)).all()
        oc = si.out_components(n, s, d, t, directed=directed)
        by_si = np.zeros(n, dtype=np.int64)
        for comp in oc:
            for w in comp:
                by_si[w] += 1
        assert (inn == by_si).all()
        assert len(set(inn.tolist())) > 3  # the counts really differ by column
