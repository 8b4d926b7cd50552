"""Pins for the oracle's generation (Eq. 2.1, Algorithms 2-4): brute force over
every branch vector of tiny swarms, invariants on random runs, the pure random
search special case, and convergence on the shifted sphere."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2110_01470_amd.inputs import WORKLOADS, make_objective

TWO32 = 1 << 32
KIND = {"sphere": oracle.SPHERE, "ripple": oracle.RIPPLE, "dense": oracle.DENSE}
G, P, S, F = "g", "p", "self", "fresh"
# Interval order by definition: thresholds listed first to last.
ORDERS = {
    oracle.ORDER_GPS: (lambda cg, cp, cw: (cg, cp, cw), (G, P, S, F)),
    oracle.ORDER_EQ21: (lambda cg, cp, cw: (cw, cp, cg), (S, P, G, F)),
}


def exact_thresholds(order, cg, cp, cw):
    pick, _ = ORDERS[order]
    return [math.ceil(Fraction(c) * TWO32) for c in pick(cg, cp, cw)]


def source_of(word, th, labels):
    for k in range(3):
        if word < th[k]:
            return labels[k]
    return labels[3]


def independent_fitness(kind, x, s, w=None, a=None):
    d = x.astype(np.float64) - s.astype(np.float64)
    if kind == "sphere":
        return math.fsum(float(u) * float(u) for u in d)
    if kind == "ripple":
        return (math.fsum(float(wi) * float(u) * float(u) for wi, u in zip(w, d))
                + 0.5 * math.fsum(math.sin(3.0 * float(u)) ** 2 for u in d))
    y = a.astype(np.float64) @ d
    return math.fsum(float(v) * float(v) for v in y)


def f32_close(a, b):
    """Equal, or one FP32 ulp apart (double rounding of a sum)."""
    a, b = np.float32(a), np.float32(b)
    return a == b or abs(int(a.view(np.int32)) - int(b.view(np.int32))) <= 1


def make_swarm(kind, n, d, seed, cg=0.4, cp=0.7, cw=0.9, order=oracle.ORDER_GPS,
               lo=-10.0, hi=10.0):
    s, w, a = make_objective(kind, d, seed, lo / 2, hi / 2)
    sw = oracle.Swarm(n, d, KIND[kind], lo, hi, cg, cp, cw, seed, s, w, a, order=order)
    return sw, s, w, a


def check_generation(sw, kind, s, w, a, pre, words, th, labels, lo, hi, rule):
    x0, p0, fp0, _, g0, _, _ = pre
    n, d = x0.shape
    for i in range(n):
        for j in range(d):
            src = source_of(int(words[i, j]), th, labels)
            expect = {G: g0[j], P: p0[i, j], S: x0[i, j]}.get(src)
            if src == F:
                expect = rule.fresh_value(int(words[i, j]))
            assert sw.x[i, j] == expect, (i, j, src)
    assert np.all(sw.x >= lo) and np.all(sw.x <= hi)
    for i in range(n):
        fx = independent_fitness(kind, sw.x[i], s, w, a)
        assert sw.fx64[i] == pytest.approx(fx, rel=1e-12, abs=1e-300)
        better = np.float32(sw.fx64[i]) < fp0[i]
        assert bool(sw.improved[i]) == bool(better)
        if better:
            assert np.array_equal(sw.p[i], sw.x[i])
            assert sw.fp[i] == np.float32(sw.fx64[i])
        else:
            assert np.array_equal(sw.p[i], p0[i])
            assert sw.fp[i] == fp0[i]
        assert sw.fp[i] <= fp0[i]
        assert f32_close(sw.fp[i], independent_fitness(kind, sw.p[i], s, w, a))
    best = min(range(n), key=lambda i: (float(sw.fp[i]), i))
    assert sw.gidx == best
    assert np.array_equal(sw.g, sw.p[best])


@pytest.mark.parametrize("kind,n,d", [("sphere", 2, 2), ("ripple", 3, 1), ("dense", 1, 3),
                                      ("sphere", 3, 2)])
@pytest.mark.parametrize("order", [oracle.ORDER_GPS, oracle.ORDER_EQ21])
def test_brute_force_every_branch_vector(kind, n, d, order):
    lo, hi = -10.0, 10.0
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.8, 0.6, 0.3)
    sw, s, w, a = make_swarm(kind, n, d, 17, cg, cp, cw, order, lo, hi)
    th = exact_thresholds(order, cg, cp, cw)
    labels = ORDERS[order][1]
    rule = oracle.Rule(cg, cp, cw, lo, hi, order=order)
    bounds = [0] + th + [TWO32]
    rng = np.random.default_rng(123)
    # A pre-state where x, p and g all differ, with p's fitness as state.
    x0 = rng.uniform(lo, hi, (n, d)).astype(np.float32)
    p0 = rng.uniform(lo, hi, (n, d)).astype(np.float32)
    fp0 = np.array([np.float32(independent_fitness(kind, p0[i], s, w, a)) for i in range(n)],
                   dtype=np.float32)
    for branch in itertools.product(range(4), repeat=n * d):
        words = np.array([rng.integers(bounds[b], bounds[b + 1]) for b in branch],
                         dtype=np.uint64).astype(np.uint32).reshape(n, d)
        sw.set_state(x0, p0, fp0, 5)
        assert sw.gidx == min(range(n), key=lambda i: (float(fp0[i]), i))
        pre = sw.state()
        sw.step(words)
        assert sw.t == 6
        check_generation(sw, kind, s, w, a, pre, words, th, labels, lo, hi, rule)


@pytest.mark.parametrize("kind,n,d", [("sphere", 17, 13), ("ripple", 9, 33), ("dense", 11, 8)])
@pytest.mark.parametrize("order", [oracle.ORDER_GPS, oracle.ORDER_EQ21])
def test_invariants_along_a_run(kind, n, d, order):
    lo, hi = -10.0, 10.0
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.9, 0.7, 0.4)
    sw, s, w, a = make_swarm(kind, n, d, 29, cg, cp, cw, order, lo, hi)
    th = exact_thresholds(order, cg, cp, cw)
    labels = ORDERS[order][1]
    sw.init()
    assert np.array_equal(sw.x, sw.p)
    rule = oracle.Rule(cg, cp, cw, lo, hi, order=order)
    w0 = oracle.words(29, 0, 0, n, d)
    for i in range(n):
        for j in range(d):
            assert sw.x[i, j] == rule.init_value(int(w0[i, j]))
    prev_fp = sw.fp.copy()
    for _ in range(25):
        pre = sw.state()
        words = oracle.words(29, 0, sw.t + 1, n, d)
        sw.step()
        check_generation(sw, kind, s, w, a, pre, words, th, labels, lo, hi, rule)
        assert np.all(sw.fp <= prev_fp)
        prev_fp = sw.fp.copy()


def test_pure_random_search_best_of_all_draws():
    # cg = cp = cw = 0: every generation redraws every variable, so gBest is the
    # best of the N (T + 1) uniform points seen.  For D = 1 on [-1, 1] with the
    # optimum s inside, P(|g - s| <= r) = 1 - (1 - r)^M for r below the distance
    # from s to the box, M = N (T + 1).
    n, t, s = 8, 24, np.float32(0.3)
    m = n * (t + 1)
    gaps = []
    for seed in range(300):
        sw = oracle.Swarm(n, 1, oracle.SPHERE, -1.0, 1.0, 0.0, 0.0, 0.0, 1000 + seed,
                          np.array([s], np.float32))
        sw.init().run(t)
        gaps.append(abs(float(sw.g[0]) - float(s)))
    gaps = np.array(gaps)
    assert gaps.max() < 0.7
    p = stats.kstest(gaps, lambda r: 1.0 - (1.0 - np.minimum(r, 1.0)) ** m).pvalue
    assert p > 1e-3, p
    # Keeping only the last generation (a broken pBest) would give M = N.
    p_wrong = stats.kstest(gaps, lambda r: 1.0 - (1.0 - np.minimum(r, 1.0)) ** n).pvalue
    assert p_wrong < 1e-6


def test_converges_toward_the_shift_on_the_sphere():
    wl = WORKLOADS["sphere_n100_d30"]
    s, w, a = wl.objective()
    sw = oracle.Swarm(wl.n, wl.d, oracle.SPHERE, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed,
                      s, w, a)
    sw.init()
    f0 = float(sw.fp[sw.gidx])
    dist0 = float(np.linalg.norm(sw.g - s))
    trace = [f0]
    for _ in range(wl.generations):
        sw.step()
        trace.append(float(sw.fp[sw.gidx]))
    trace = np.array(trace)
    assert np.all(np.diff(trace) <= 0)
    assert trace[-1] < 1e-3 * f0
    assert float(np.linalg.norm(sw.g - s)) < 0.05 * dist0


def test_run_equals_steps_and_resume_is_exact():
    kind, n, d = "ripple", 13, 21
    sw1, s, w, a = make_swarm(kind, n, d, 41)
    sw1.init().run(30)
    sw2, *_ = make_swarm(kind, n, d, 41)
    sw2.init()
    for _ in range(12):
        sw2.step()
    snap = sw2.state()
    sw3, *_ = make_swarm(kind, n, d, 41)
    sw3.set_state(snap[0], snap[1], snap[2], snap[6])
    sw3.run(18)
    for other in (sw3,):
        assert np.array_equal(sw1.x, other.x)
        assert np.array_equal(sw1.p, other.p)
        assert np.array_equal(sw1.fp, other.fp)
        assert np.array_equal(sw1.g, other.g)
        assert sw1.gidx == other.gidx and sw1.t == other.t == 30


def test_lowest_index_wins_exact_ties():
    n, d = 6, 3
    s = np.zeros(d, np.float32)
    sw = oracle.Swarm(n, d, oracle.SPHERE, -1.0, 1.0, 0.4, 0.7, 0.9, 3, s)
    p = np.tile(np.array([0.5, -0.25, 0.125], np.float32), (n, 1))
    p[0] += 0.5
    p[1] += 0.25
    fp = np.array([np.float32(independent_fitness("sphere", r, s)) for r in p], np.float32)
    sw.set_state(p, p, fp, 0)
    assert sw.gidx == 2
    assert oracle.argmin(np.array([3, np.nan, 1, 1, np.inf], np.float32)) == 2
    assert oracle.argmin(np.array([np.nan, np.nan], np.float32)) == 0
    assert oracle.argmin(np.array([np.nan, np.inf], np.float32)) == 1
    # -0 and +0 are the same fitness: the lower index wins either way round.
    assert oracle.argmin(np.array([1, -0.0, 0.0], np.float32)) == 1
    assert oracle.argmin(np.array([1, 0.0, -0.0], np.float32)) == 1


def test_nan_orders_above_every_number_in_pbest_updates():
    """Algorithm 3 with NaN ordered above every number (as in the argmin): a
    pBest whose fitness is NaN is replaced by any number, and a NaN fitness
    never replaces a pBest."""
    n, d = 5, 4
    s = np.zeros(d, np.float32)
    sw = oracle.Swarm(n, d, oracle.SPHERE, -1.0, 1.0, 0.0, 0.0, 0.0, 7, s)
    sw.init()
    x, p, fp = sw.x.copy(), sw.p.copy(), sw.fp.copy()
    fp[[1, 3]] = np.nan
    fp[[0, 2, 4]] = 0.0  # nothing can improve on 0
    sw.set_state(x, p, fp, 0)
    assert sw.gidx == 0
    sw.step()
    assert list(sw.improved) == [0, 1, 0, 1, 0]
    assert np.all(np.isfinite(sw.fp)) and np.all(sw.fp[[0, 2, 4]] == 0.0)
    # A NaN objective (shift NaN in one coordinate): every fitness is NaN,
    # so after initialisation nothing is ever replaced and gBest stays 0.
    s_nan = s.copy()
    s_nan[2] = np.nan
    sw = oracle.Swarm(n, d, oracle.SPHERE, -1.0, 1.0, 0.4, 0.7, 0.9, 7, s_nan)
    sw.init()
    p0 = sw.p.copy()
    sw.run(3)
    assert np.all(np.isnan(sw.fp)) and sw.improved.sum() == 0
    assert np.array_equal(sw.p, p0) and sw.gidx == 0


@pytest.mark.parametrize("kind", ["ripple", "dense", "f3"])
def test_thread_count_does_not_change_results(kind):
    """The loops over particles may run on several threads (the all-cores
    timing of the CPU baseline): a run on 4 threads is bit-identical to a run
    on one."""
    n, d = 203, 37
    states = []
    for threads in (1, 4):
        assert oracle.set_threads(threads) == threads
        try:
            if kind == "f3":
                sw = oracle.Swarm(n, d, oracle.F3, -100.0, 100.0, 0.8, 0.6, 0.3, 9, None,
                                  order=oracle.ORDER_EQ21)
                sw.init().run(6)
            else:
                sw, *_ = make_swarm(kind, n, d, 57)
                sw.init().run(6)
            states.append((sw.x.copy(), sw.p.copy(), sw.fp.copy(), sw.fp64.copy(), sw.g.copy(),
                           sw.gidx, sw.improved.copy()))
        finally:
            oracle.set_threads(1)
    for u, v in zip(*states):
        assert np.array_equal(u, v)
    if kind == "dense":
        # The polish runs its particles on several threads too.
        polished = []
        for threads in (1, 4):
            oracle.set_threads(threads)
            try:
                sw, s, w, a = make_swarm(kind, n, d, 57)
                sw.init().run(3)
                sigma = np.linalg.norm(a.astype(np.float64), 2)
                sw.polish(3, 0.05 / sigma**2)
                polished.append((sw.p.copy(), sw.fp.copy(), sw.fx64.copy(), sw.improved.copy(),
                                 sw.gidx))
            finally:
                oracle.set_threads(1)
        for u, v in zip(*polished):
            assert np.array_equal(u, v)
    w1 = oracle.words(3, 0, 5, 40, 9)
    oracle.set_threads(4)
    try:
        w4 = oracle.words(3, 0, 5, 40, 9)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(w1, w4)
