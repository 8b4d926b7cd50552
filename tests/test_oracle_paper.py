"""Pins of the oracle's Table 3.2 benchmark functions.

Each function is checked at points where it has a closed form, at its known
minimiser, and against a library implementation where one exists
(scipy.optimize.rosen for Rosenbrock).  The points are chosen so that a
dropped term, a shifted index or a wrong constant changes the value."""
import math

import numpy as np
import pytest
from scipy.optimize import rosen

import oracle


def f(kind, x):
    return oracle.fitness(kind, np.asarray(x, np.float32), None)


def unit(P, k):
    x = np.zeros(P, np.float32)
    x[k] = 1.0
    return x


@pytest.mark.parametrize("P", [1, 4, 7, 50])
def test_sphere_and_ellipsoid(P):
    assert f(oracle.F1, np.zeros(P)) == 0.0
    assert f(oracle.F1, np.full(P, 3.0)) == 9.0 * P
    assert f(oracle.F2, np.ones(P)) == P * (P + 1) / 2
    for k in range(P):  # the k-th square (0-based) weighs k + 1
        assert f(oracle.F2, unit(P, k)) == k + 1


@pytest.mark.parametrize("P", [1, 5, 50])
def test_schwefel_1_2_sums_running_sums(P):
    assert f(oracle.F3, np.ones(P)) == P * (P + 1) * (2 * P + 1) / 6
    assert f(oracle.F3, unit(P, 0)) == P          # x_1 is in every running sum
    assert f(oracle.F3, unit(P, P - 1)) == 1      # x_P only in the last
    alt = np.array([(-1.0) ** i for i in range(P)], np.float32)  # sums 1, 0, 1, 0, ...
    assert f(oracle.F3, alt) == math.ceil(P / 2)


def test_rosenbrock_equals_library_and_minimum():
    rng = np.random.default_rng(4)
    for P in (2, 3, 17, 50):
        for _ in range(5):
            x = rng.uniform(-2.048, 2.048, P).astype(np.float32)
            ref = rosen(x.astype(np.float64))
            assert abs(f(oracle.F4, x) - ref) <= 1e-12 * max(1.0, ref)
        assert f(oracle.F4, np.ones(P)) == 0.0
        assert f(oracle.F4, np.zeros(P)) == P - 1
    assert f(oracle.F4, [0.7]) == 0.0  # one variable: no pairs


def test_rastrigin():
    P = 50
    assert abs(f(oracle.F5, np.zeros(P))) < 1e-12
    k = np.random.default_rng(5).integers(-5, 6, P).astype(np.float32)
    assert abs(f(oracle.F5, k) - float(np.sum(k.astype(np.float64) ** 2))) < 1e-9
    # x = 1/2: cos(pi) = -1, each term 1/4 + 10 on top of 10 P.
    assert abs(f(oracle.F5, np.full(P, 0.5)) - P * 20.25) < 1e-9


def test_ackley():
    for P in (1, 10, 50):
        assert abs(f(oracle.F6, np.zeros(P))) < 1e-13
        for k in (1.0, 3.0):  # integers: every cosine is 1
            x = np.full(P, k, np.float32)
            ref = 20.0 * (1.0 - math.exp(-0.2 * k))
            assert abs(f(oracle.F6, x) - ref) < 1e-12
    # Half-integers: every cosine is -1, so the second exponential is 1/e.
    x = np.full(8, 0.5, np.float32)
    ref = -20.0 * math.exp(-0.2 * 0.5) - math.exp(-1.0) + 20.0 + math.e
    assert abs(f(oracle.F6, x) - ref) < 1e-12


def test_griewank():
    P = 30
    assert f(oracle.F7, np.zeros(P)) == 0.0
    # x_i = 2 pi sqrt(i) k_i makes every cosine 1 (up to the FP32 rounding of x).
    k = np.random.default_rng(6).integers(-3, 4, P)
    x = (2.0 * np.pi * np.sqrt(np.arange(1, P + 1)) * k).astype(np.float32)
    ref = float(np.sum(x.astype(np.float64) ** 2)) / 4000.0
    assert abs(f(oracle.F7, x) - ref) < 1e-9
    # One variable at pi * sqrt(i): its cosine is -1, the product flips sign.
    for i in (1, 7, 30):
        y = np.zeros(P, np.float32)
        y[i - 1] = np.float32(np.pi * np.sqrt(i))
        ref = float(np.float64(y[i - 1]) ** 2) / 4000.0 + 2.0
        assert abs(f(oracle.F7, y) - ref) < 1e-9


def test_powell():
    assert f(oracle.F8, [3.0, -1.0, 0.0, 1.0]) == 215.0
    assert f(oracle.F8, np.zeros(12)) == 0.0
    # Only whole groups of four count: the two trailing variables do nothing.
    assert f(oracle.F8, [3.0, -1.0, 0.0, 1.0, 7.0, 7.0]) == 215.0
    assert f(oracle.F8, [7.0, 7.0, 7.0]) == 0.0
    # Groups are independent and in place: shifting a group moves its term.
    assert f(oracle.F8, [0, 0, 0, 0, 3.0, -1.0, 0.0, 1.0]) == 215.0
    assert f(oracle.F8, [1.0, 0, 0, 0]) == 1.0 + 10.0  # (x1)^2 + 10 (x1)^4


def test_schwefel_2_26():
    P = 50
    assert f(oracle.F9, np.zeros(P)) == pytest.approx(418.9829 * P, rel=1e-15)
    xs = np.full(P, 420.968746, np.float32)
    assert 0.0 <= f(oracle.F9, xs) < 1e-3 * P
    # The sign of the sum: x sin(sqrt|x|) at x = (pi/2)^2 is x itself.
    x = np.zeros(P, np.float32)
    x[0] = np.float32((np.pi / 2) ** 2)
    assert abs(f(oracle.F9, x) - (418.9829 * P - float(x[0]) * math.sin(math.sqrt(float(x[0]))))) < 1e-9
    assert f(oracle.F9, x) < 418.9829 * P


@pytest.mark.parametrize("kind", range(oracle.F1, oracle.F9 + 1))
def test_scale_bounds_the_value(kind):
    rng = np.random.default_rng(kind)
    for P in (1, 4, 13, 50):
        x = rng.uniform(-5, 5, P).astype(np.float32)
        v = oracle.fitness(kind, x, None)
        sc = oracle.fitness_scale(kind, x)
        assert sc >= abs(v) - 1e-9 * sc
        if kind in (oracle.F1, oracle.F2):
            assert sc == v


def test_fitness_scale_is_only_defined_for_table_3_2():
    """The shifted objectives have no scale: the call returns NaN for them,
    so nothing can lean on an undefined bound."""
    x = np.ones(8, np.float32)
    s = np.zeros(8, np.float32)
    for kind, w, a in ((oracle.SPHERE, None, None), (oracle.RIPPLE, np.ones(8, np.float32), None),
                       (oracle.DENSE, None, np.eye(8, dtype=np.float32))):
        assert np.isnan(oracle.fitness_scale(kind, x, s, w, a))


@pytest.mark.parametrize("kind", range(oracle.F1, oracle.F9 + 1))
def test_swarm_runs_on_each_function(kind):
    """A swarm on each function (no shift arrays): the pBest fitness never
    increases, it is the function's value at the pBest, and gBest is the
    lowest-index argmin."""
    sw = oracle.Swarm(30, 13, kind, -2.0, 2.0, 0.8, 0.6, 0.3, 1001, None, order=oracle.ORDER_EQ21)
    sw.init()
    prev = sw.fp.copy()
    for _ in range(15):
        sw.step()
        assert np.all(sw.fp <= prev)
        prev = sw.fp.copy()
    for i in range(30):
        assert sw.fp64[i] == oracle.fitness(kind, sw.p[i], None)
    assert sw.gidx == oracle.argmin(sw.fp)
