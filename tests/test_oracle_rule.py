"""Pins for the oracle's integer form of Eq. (2.1) and its draws on [varMin, varMax]."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle

TWO32 = 1 << 32


def exact_threshold(c):
    return math.ceil(Fraction(c) * TWO32)


@pytest.mark.parametrize("c", [0.0, 0.1, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99,
                               1.0 / 3.0, 2.0 ** -32, 0.5 + 2.0 ** -33])
def test_thresholds_are_exact_ceilings(c):
    r = oracle.Rule(c, c, c, -1.0, 1.0) if c < 0.99 else oracle.Rule(0.0, 0.0, c, -1.0, 1.0)
    assert r.thresholds[2] == exact_threshold(c)


@pytest.mark.parametrize("order,cs,srcs", [
    (oracle.ORDER_GPS, (0.4, 0.7, 0.9), (oracle.SRC_GBEST, oracle.SRC_PBEST, oracle.SRC_SELF)),
    (oracle.ORDER_EQ21, (0.3, 0.6, 0.8), (oracle.SRC_SELF, oracle.SRC_PBEST, oracle.SRC_GBEST)),
])
def test_interval_boundaries(order, cs, srcs):
    if order == oracle.ORDER_GPS:
        cg, cp, cw = cs
    else:
        cw, cp, cg = cs
    r = oracle.Rule(cg, cp, cw, -100.0, 100.0, order=order)
    th = [exact_threshold(c) for c in cs]
    assert r.thresholds == tuple(th)
    assert r.sources == srcs
    seq = list(srcs) + [oracle.SRC_FRESH]
    assert r.source(0) == seq[0]
    assert r.source(TWO32 - 1) == oracle.SRC_FRESH
    for k in range(3):
        assert r.source(th[k] - 1) == seq[k]
        assert r.source(th[k]) == seq[k + 1]


def test_empty_intervals_are_skipped():
    r = oracle.Rule(0.5, 0.5, 0.5, 0.0, 1.0)
    th = exact_threshold(0.5)
    assert r.source(th - 1) == oracle.SRC_GBEST
    assert r.source(th) == oracle.SRC_FRESH
    r = oracle.Rule(0.0, 0.0, 0.0, 0.0, 1.0)
    assert r.source(0) == oracle.SRC_FRESH


@pytest.mark.parametrize("args", [
    (0.7, 0.4, 0.9, -1.0, 1.0),          # cg > cp
    (0.4, 0.95, 0.9, -1.0, 1.0),         # cp > cw
    (0.4, 0.7, 1.0 - 2.0 ** -8, -1.0, 1.0),  # fresh interval holds only 2^24 words
    (0.4, 0.7, 0.9, 1.0, 1.0),           # empty box
    (0.4, 0.7, 0.9, 1.0, -1.0),          # reversed box
    (0.4, 0.7, float("nan"), -1.0, 1.0),
    (-0.1, 0.7, 0.9, -1.0, 1.0),
    (0.4, 0.7, 0.9, -3e38, 3e38),        # span overflows FP32
])
def test_invalid_parameters_rejected(args):
    with pytest.raises(ValueError):
        oracle.Rule(*args)


def test_largest_valid_cw_accepted():
    cw = 1.0 - 2.0 ** -8 - 2.0 ** -30
    r = oracle.Rule(0.1, 0.2, cw, -1.0, 1.0)
    assert TWO32 - r.thresholds[2] > (1 << 24)


def test_branch_frequencies_match_interval_widths():
    cg, cp, cw = 0.4, 0.7, 0.9
    r = oracle.Rule(cg, cp, cw, -100.0, 100.0)
    th = np.array(r.thresholds, dtype=np.uint64)
    # 1.2e7 words (12000 particles x 1000 variables of one generation).
    used = oracle.set_threads(min(8, os.cpu_count() or 1))
    try:
        w = oracle.words(11, 0, 1, 12000, 1000).ravel()
    finally:
        oracle.set_threads(1)
    del used
    b = (w >= np.uint32(th[0])).astype(np.int8)
    b += w >= np.uint32(th[1])
    b += w >= np.uint32(th[2])
    counts = np.bincount(b, minlength=4)
    probs = np.array([cg, cp - cg, cw - cp, 1.0 - cw])
    n = w.size
    z = (counts - n * probs) / np.sqrt(n * probs * (1 - probs))
    assert np.all(np.abs(z) < 5.0), z


def test_init_value_endpoints_and_single_rounding():
    lo, hi = np.float32(-100.0), np.float32(100.0)
    r = oracle.Rule(0.4, 0.7, 0.9, lo, hi)
    span = float(np.float32(hi - lo))
    assert r.init_value(0) == lo
    top = r.init_value(TWO32 - 1)
    assert top <= hi and top >= hi - 2 * span * 2.0 ** -24
    rng = np.random.default_rng(3)
    for word in rng.integers(0, TWO32, size=2000, dtype=np.uint64):
        u = int(word) >> 8
        # lo + u 2^-24 span is exact in FP64 here; one rounding gives the FP32 draw.
        exact = float(lo) + u * 2.0 ** -24 * span
        assert r.init_value(int(word)) == np.float32(exact)


def test_init_values_uniform_on_box():
    r = oracle.Rule(0.4, 0.7, 0.9, -3.0, 5.0)
    w = oracle.words(21, 0, 0, 400, 500).ravel()[:100000]
    v = np.array([r.init_value(int(k)) for k in w])
    assert v.min() >= -3.0 and v.max() <= 5.0
    assert stats.kstest(v, "uniform", args=(-3.0, 8.0)).pvalue > 1e-4


@pytest.mark.parametrize("cs", [(0.4, 0.7, 0.9), (0.0, 0.0, 0.0), (0.1, 0.2, 0.99)])
def test_fresh_value_endpoints_and_monotone(cs):
    lo, hi = -10.0, 10.0
    r = oracle.Rule(*cs, lo, hi)
    t2 = r.thresholds[2]
    span = r.span
    assert r.fresh_value(t2) == np.float32(lo)
    top = r.fresh_value(TWO32 - 1)
    assert top <= hi and top >= hi - 2 * span * 2.0 ** -24
    rng = np.random.default_rng(5)
    ks = np.sort(rng.integers(t2, TWO32, size=3000, dtype=np.uint64))
    vals = np.array([r.fresh_value(int(k)) for k in ks])
    assert np.all(np.diff(vals) >= 0)


def test_fresh_values_uniform_on_box():
    r = oracle.Rule(0.4, 0.7, 0.9, -100.0, 100.0)
    t2 = r.thresholds[2]
    w = oracle.words(31, 0, 5, 1000, 1000).ravel()
    w = w[w >= t2][:100000]
    v = np.array([r.fresh_value(int(k)) for k in w])
    assert v.min() >= -100.0 and v.max() <= 100.0
    assert stats.kstest(v, "uniform", args=(-100.0, 200.0)).pvalue > 1e-4


def test_pure_random_search_fresh_map_equals_init_map():
    # With every threshold at 0 the fresh interval is all of [0, 2^32) and the
    # rescale to 24 bits must reduce to the top 24 bits of the word.
    r = oracle.Rule(0.0, 0.0, 0.0, -1.0, 3.0)
    assert r.r == 1 << 24
    rng = np.random.default_rng(8)
    for k in rng.integers(0, TWO32, size=500, dtype=np.uint64):
        assert r.fresh_value(int(k)) == r.init_value(int(k))
