"""Pins for the oracle's Philox4x32-10 and its word layout (Sec. 3.1)."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("|")
            a = [int(v, 16) for v in lhs.split()]
            b = [int(v, 16) for v in rhs.split()]
            rows.append((a[:4], a[4:], b))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox(ctr, key)) == expect


def test_kat_file_has_three_vectors():
    assert len(_kat_rows()) == 3


def test_word_layout_one_block_per_four_variables():
    seed, swarm, t, n, d = 0x0123456789ABCDEF, 7, 42, 3, 10
    w = oracle.words(seed, swarm, t, n, d)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(n):
        for q in range((d + 3) // 4):
            blk = oracle.philox([q, i, t, swarm], key)
            for e in range(4):
                j = 4 * q + e
                if j < d:
                    assert w[i, j] == blk[e]


def test_words_differ_across_each_counter_field():
    base = oracle.words(5, 0, 1, 4, 8)
    assert not np.array_equal(base, oracle.words(6, 0, 1, 4, 8))   # seed
    assert not np.array_equal(base, oracle.words(5, 1, 1, 4, 8))   # swarm
    assert not np.array_equal(base, oracle.words(5, 0, 2, 4, 8))   # generation
    assert len(np.unique(base)) == base.size                        # particles, variables


def test_word_bytes_are_uniform():
    w = oracle.words(99, 0, 3, 512, 512).ravel()
    for shift in (0, 8, 16, 24):
        counts = np.bincount((w >> shift) & 0xFF, minlength=256)
        p = stats.chisquare(counts).pvalue
        assert p > 1e-4, (shift, p)
