"""Pins for the oracle's fixed-point weights and within-island resampling.

Systematic resampling (Kitagawa 1996; Carpenter, Clifford and Fearnhead
1999) on integer cumulative weights.  Properties the definition fixes:
  * averaged over every offset U in [0, Q), particle i gets exactly N q_i / Q
    offspring per draw (sum over U of its offspring = N q_i), the lack-of-bias
    requirement Theorem 1 rests on;
  * every particle gets floor(N q_i/Q) or ceil(N q_i/Q) offspring;
  * ancestors are non-decreasing in the slot index.
"""
import numpy as np
import pytest


def test_quantise(orc):
    lw = np.array([-1.0, 0.5, -np.inf, 0.5 - 40 * np.log(2) - 1e-9, 0.25])
    q, mx = orc.quantise(lw)
    assert mx == 0.5
    assert q[1] == 2**40
    assert q[2] == 0
    assert q[3] == 0                       # weight below 2^-40 of the island max
    assert q[0] == int(np.floor(np.exp(-1.5) * 2.0**40))
    assert q[4] == int(np.floor(np.exp(-0.25) * 2.0**40))
    q, mx = orc.quantise(np.full(4, -np.inf))
    assert mx == -np.inf and (q == 0).all()


def test_systematic_hand_cases(orc):
    # q = (3, 0, 5, 2), Q = 10, N = 4: N C = (12, 12, 32, 40); thresholds U + 10 j
    q = np.array([3, 0, 5, 2], dtype=np.uint64)
    assert orc.systematic(q, 0).tolist() == [0, 0, 2, 2]      # t = 0, 10, 20, 30
    assert orc.systematic(q, 5).tolist() == [0, 2, 2, 3]      # t = 5, 15, 25, 35
    assert orc.systematic(q, 2).tolist() == [0, 2, 2, 3]      # t = 2, 12, 22, 32 (ties go right)
    assert orc.systematic(q, 9).tolist() == [0, 2, 2, 3]
    assert orc.systematic(np.array([7], dtype=np.uint64), 3).tolist() == [0]


@pytest.mark.parametrize("seed", range(6))
def test_systematic_exact_expected_offspring(orc, seed):
    g = np.random.default_rng(seed)
    N = int(g.integers(1, 9))
    q = g.integers(0, 40, N).astype(np.uint64)
    if q.sum() == 0:
        q[0] = 1
    Q = int(q.sum())
    total = np.zeros(N, dtype=np.int64)
    for U in range(Q):
        a = orc.systematic(q, U)
        assert (np.diff(a) >= 0).all()
        off = np.bincount(a, minlength=N)
        assert off.sum() == N
        lo = (N * q.astype(np.int64)) // Q
        assert ((off == lo) | (off == lo + 1)).all()
        assert (off[q == 0] == 0).all()
        total += off
    assert (total == N * q.astype(np.int64)).all()


def test_systematic_large_weights(orc):
    # N = 2048 with every q = 2^40 (the maximum): N C_i up to 2^62, no overflow
    N = 2048
    q = np.full(N, 2**40, dtype=np.uint64)
    Q = N * 2**40
    for U in (0, 1, Q // 2, Q - 1):
        a = orc.systematic(q, U)
        assert (a == np.arange(N)).all()
