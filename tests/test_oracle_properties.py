"""Property-based pins of the CPU oracle (hypothesis, derandomized): on
generated tiny tie-heavy networks, the reverse-time matrix equals the
deterministic SI brute force from every node (Sec. 1) and the transpose of
forward Algorithm 1 (Sec. 3.1, 3.4), and it satisfies Eq. 1 and the
diagonal, tail and monotonicity invariants."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from oracle import si


@st.composite
def tiny_networks(draw):
    n = draw(st.integers(1, 12))
    m = draw(st.integers(0, 40))
    T = draw(st.integers(1, 8))  # few time steps: many ties
    ev = draw(st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1),
                                 st.integers(0, T - 1)), min_size=m, max_size=m))
    ev.sort(key=lambda e: e[2])  # stable: ties keep their drawn order
    s = np.array([e[0] for e in ev], dtype=np.uint32)
    d = np.array([e[1] for e in ev], dtype=np.uint32)
    t = np.array([e[2] for e in ev], dtype=np.int64)
    return n, s, d, t, draw(st.booleans()), draw(st.booleans())


@settings(max_examples=300, derandomize=True, deadline=None)
@given(tiny_networks())
def test_reverse_matrix_is_si_brute_force_and_forward_transpose(net):
    n, s, d, t, directed, sequential = net
    R = oracle.reverse_matrix(n, s, d, t, directed=directed, sequential=sequential)
    D = oracle.to_dense(R, n)
    oc = si.out_components(n, s, d, t, directed=directed, sequential=sequential)
    for u in range(n):
        assert set(np.nonzero(D[u])[0]) == oc[u], u
    F = oracle.to_dense(oracle.forward_matrix(n, s, d, t, directed=directed,
                                              sequential=sequential), n)
    assert (F == D.T).all()
    # diagonal, tail bits, Eq. 1 (sum of out-sizes = sum of in-sizes)
    assert D.diagonal().all()
    nw = oracle.words(n)
    if n % 64:
        assert not (R[:, nw - 1] >> np.uint64(n % 64)).any()
    out, inn = oracle.sizes(R, n)
    assert out.sum() == inn.sum() == D.sum()
    # appending later events never clears a bit
    if n > 1:
        t2 = np.append(t, (t.max() + 1) if t.size else 0)
        R2 = oracle.reverse_matrix(n, np.append(s, np.uint32(0)), np.append(d, np.uint32(n - 1)),
                                   t2, directed=directed, sequential=sequential)
        assert ((R2 & R) == R).all()


def test_two_blocks_never_join():
    # events only among the even and among the odd nodes: no node reaches one
    # of the other parity, and with enough events every node reaches its
    # whole block (the brute force agrees on a small case)
    import tn_inputs as T
    for n in (4, 9, 64):
        s, d, t = T.two_block_pairs(n, 40 * n, 8, seed=8500 + n)
        assert (s % 2 == d % 2).all() and (s != d).all()
        D = oracle.to_dense(oracle.reverse_matrix(n, s, d, t), n)
        par = np.arange(n) % 2
        assert not D[par[:, None] != par[None, :]].any(), n
        oc = si.out_components(n, s, d, t)
        for u in range(n):
            assert set(np.nonzero(D[u])[0]) == oc[u], (n, u)
