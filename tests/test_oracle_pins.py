"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import pins
import refs


@pytest.mark.parametrize("name", list(pins.ALL_CHECKS))
def test_pin(oracle_lib, name):
    fails = pins.ALL_CHECKS[name](oracle_lib)
    assert not fails, "\n".join(fails)


def test_references_agree_with_each_other():
    """The independent references agree on the tiny cases (sanity of the pins)."""
    for (q, s, M, a, b), bf in zip(pins.tiny_cases()[:120], pins._brute_table()):
        assert refs.general_gap_dp(q, s, M, a, b) == bf
        if a == b:
            assert refs.linear_gap_sw(q, s, M, a) == bf


def test_empty_inputs(oracle_lib):
    M = np.eye(4, dtype=np.int8) * 5
    assert oracle_lib.sw_score(np.array([], np.uint8), np.array([1, 2], np.uint8), M, 1, 3) == 0
    assert oracle_lib.sw_score(np.array([1, 2], np.uint8), np.array([], np.uint8), M, 1, 3) == 0


def test_zero_init_equals_minus_infinity_init(oracle_lib):
    """E and F start at 0 in the paper; the textbook starts them at -inf.  The
    scores agree, checked here against the cubic DP, which has no E/F state."""
    rng = np.random.Generator(np.random.PCG64(21))
    for _ in range(40):
        A = 4
        M = rng.integers(-3, 6, size=(A, A)).astype(np.int8)
        q = rng.integers(0, A, size=10).astype(np.uint8)
        s = rng.integers(0, A, size=12).astype(np.uint8)
        # alpha = 0: a gap opened at the border could extend for free if the
        # border started above -inf in a way that mattered.
        for a, b in [(0, 0), (0, 5), (1, 1), (2, 9)]:
            assert oracle_lib.sw_score(q, s, M, a, b) == refs.general_gap_dp(q, s, M, a, b)


def test_large_values_int32(oracle_lib):
    """Long identical sequences under a high diagonal: exact in int32."""
    A = 20
    M = np.full((A, A), -4, np.int8)
    np.fill_diagonal(M, 127)
    rng = np.random.Generator(np.random.PCG64(3))
    q = rng.integers(0, A, size=3000).astype(np.uint8)
    assert oracle_lib.sw_score(q, q, M, 2, 12) == 127 * 3000


@settings(max_examples=150, deadline=None)
@given(st.integers(2, 6), st.lists(st.integers(0, 5), min_size=1, max_size=5),
       st.lists(st.integers(0, 5), min_size=1, max_size=5), st.integers(0, 6), st.integers(0, 6),
       st.integers(0, 2 ** 31 - 1))
def test_hypothesis_vs_brute_force(oracle_lib, A, qs, ss, a, b, mseed):
    alpha, beta = min(a, b), max(a, b)
    q = np.array([x % A for x in qs], np.uint8)
    s = np.array([x % A for x in ss], np.uint8)
    M = np.random.Generator(np.random.PCG64(mseed)).integers(-5, 6, size=(A, A)).astype(np.int8)
    assert oracle_lib.sw_score(q, s, M, alpha, beta) == refs.brute_force(q, s, M, alpha, beta)


def test_topk_order_and_fill():
    import oracle
    scores = np.array([5, 9, 5, 9, 1, 9, 0], np.int32)
    s, i = oracle.topk(scores, 5)
    assert s.tolist() == [9, 9, 9, 5, 5] and i.tolist() == [1, 3, 5, 0, 2]
    s, i = oracle.topk(scores, 9)
    assert s.tolist()[-2:] == [-1, -1] and i.tolist()[-2:] == [-1, -1]
    assert i.tolist()[:7] == [1, 3, 5, 0, 2, 4, 6]


def test_topk_heavy_ties_properties():
    import oracle
    rng = np.random.Generator(np.random.PCG64(4))
    scores = rng.integers(0, 4, size=1000).astype(np.int32)
    s, i = oracle.topk(scores, 50)
    assert (scores[i] == s).all()
    keys = list(zip((-s).tolist(), i.tolist()))
    assert keys == sorted(keys)
    # nothing left out ranks above the last entry returned
    rest = np.setdiff1d(np.arange(1000), i)
    assert all((-scores[r], r) > keys[-1] for r in rest)
