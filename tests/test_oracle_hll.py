"""Pins of the HyperLogLog oracle (Sec. 2.2 and Sec. 3.4): register
definition on hand-made hashes, the union property against the exact
component matrix, the estimator's closed forms and its published accuracy."""
import math

import numpy as np
import pytest

import oracle
import tn_inputs as T
from oracle import hll


def test_register_definition_by_hand():
    b = 4  # 16 registers, 60 bits of rho width
    assert hll.register_of(0xF000000000000000, b) == (15, 61)        # all-zero tail
    assert hll.register_of(0x1800000000000000, b) == (1, 1)          # tail starts with 1
    assert hll.register_of(0x0000000000000001, b) == (0, 60)         # last bit only
    assert hll.register_of(0x0400000000000000, b) == (0, 2)          # tail 0b01...
    M = hll.registers_of_set([0x1800000000000000, 0x1000000000000001, 0x0400000000000000], b)
    assert M[1] == 60 and M[0] == 2 and M.sum() == 62


@pytest.mark.parametrize("flags", [(False, False, False), (True, False, False),
                                   (False, True, False), (False, False, True),
                                   (True, False, True)])
def test_stream_equals_registers_of_exact_components(flags):
    directed, sequential, forward = flags
    ref = oracle.forward_matrix if forward else oracle.reverse_matrix
    for case in range(12):
        n = 5 + (case * 7) % 60
        m = (case * 29) % 300
        s, d, t = T.random_tiny(n, m, 1 + case % 9, seed=600 + case)
        h = T.hll_node_hashes(n, seed=case)
        b = 4 + case % 3
        M = hll.stream_registers(n, s, d, t, h, b, directed, sequential, forward)
        C = oracle.to_dense(ref(n, s, d, t, directed=directed, sequential=sequential), n)
        for u in range(n):
            assert (M[u] == hll.registers_of_set(h[C[u]], b)).all(), (case, u)


def test_estimator_closed_forms():
    s = 64
    M = np.zeros((1, s), dtype=np.uint8)
    M[0, 5] = 1  # one element: linear counting s ln(s / (s - 1))
    assert hll.estimate(M)[0] == pytest.approx(s * math.log(s / (s - 1)))
    full = np.full((1, s), 10, dtype=np.uint8)  # no zero register: the raw formula
    assert hll.estimate(full)[0] == pytest.approx(0.709 * s * s / (s * 2.0 ** -10))
    assert hll.alpha(16) == 0.673 and hll.alpha(32) == 0.697 and hll.alpha(64) == 0.709
    assert hll.alpha(1024) == pytest.approx(0.7213 / (1 + 1.079 / 1024))


def test_estimator_accuracy_is_the_published_one():
    # standard error about 1.04 / sqrt(s) over random sets of one size
    g = T.rng(9)
    for b in (6, 8):
        s = 1 << b
        for size in (50, 2000, 20000):
            errs = []
            for rep in range(40):
                x = g.integers(0, 2**63, size=size, dtype=np.uint64) * np.uint64(2) + \
                    g.integers(0, 2, size=size, dtype=np.uint64)
                errs.append(hll.estimate(hll.registers_of_set(x, b))[0] / size - 1.0)
            errs = np.array(errs)
            assert abs(errs.mean()) < 3 * 1.04 / math.sqrt(s) / math.sqrt(len(errs)) + 0.02
            assert errs.std() < 1.6 * 1.04 / math.sqrt(s)
