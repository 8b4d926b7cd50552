"""Pins for the oracle's objectives against identities, special cases and
independent summation (math.fsum, numpy)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import make_objective

KIND = {"sphere": oracle.SPHERE, "ripple": oracle.RIPPLE, "dense": oracle.DENSE}


def _rand_x(d, seed, lo=-100.0, hi=100.0):
    return np.random.default_rng(seed).uniform(lo, hi, d).astype(np.float32)


@pytest.mark.parametrize("kind", ["sphere", "ripple", "dense"])
@pytest.mark.parametrize("d", [1, 3, 30, 257])
def test_zero_at_the_shift(kind, d):
    s, w, a = make_objective(kind, d, 7, -5.0, 5.0)
    assert oracle.fitness(KIND[kind], s, s, w, a) == 0.0


@pytest.mark.parametrize("d", [1, 2, 5, 30, 1000])
def test_sphere_matches_fsum(d):
    s, _, _ = make_objective("sphere", d, 1, -50, 50)
    x = _rand_x(d, d)
    ref = math.fsum((float(a) - float(b)) ** 2 for a, b in zip(x, s))
    assert oracle.fitness(oracle.SPHERE, x, s) == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("d", [1, 7, 1000])
def test_ripple_sine_part_by_double_angle(d):
    s, w, _ = make_objective("ripple", d, 2, -50, 50)
    x = _rand_x(d, 100 + d)
    dd = x.astype(np.float64) - s.astype(np.float64)
    # 0.5 sin^2(3u) = 0.25 (1 - cos(6u))
    ref = math.fsum(0.25 * (1.0 - math.cos(6.0 * u)) for u in dd)
    got = oracle.fitness(oracle.RIPPLE, x, s, np.zeros(d, np.float32))
    assert got == pytest.approx(ref, rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("d", [1, 7, 1000])
def test_ripple_is_linear_in_the_weights(d):
    s, w, _ = make_objective("ripple", d, 3, -50, 50)
    x = _rand_x(d, 200 + d)
    dd = x.astype(np.float64) - s.astype(np.float64)
    quad = math.fsum(float(wi) * u * u for wi, u in zip(w, dd))
    f_w = oracle.fitness(oracle.RIPPLE, x, s, w)
    f_0 = oracle.fitness(oracle.RIPPLE, x, s, np.zeros(d, np.float32))
    assert f_w - f_0 == pytest.approx(quad, rel=1e-12)


def test_ripple_small_offsets_approach_quadratic():
    # sin^2(3u) -> 9u^2 as u -> 0, so f -> sum (w + 4.5) u^2.
    d = 16
    s = np.zeros(d, np.float32)
    w = np.linspace(1, 1000, d).astype(np.float32)
    x = np.full(d, 1e-4, np.float32)
    u = float(x[0])
    ref = math.fsum((float(wi) + 4.5) * u * u for wi in w)
    assert oracle.fitness(oracle.RIPPLE, x, s, w) == pytest.approx(ref, rel=1e-6)


@pytest.mark.parametrize("d", [1, 4, 30, 256])
def test_dense_identity_is_sphere_bitwise(d):
    s, _, _ = make_objective("sphere", d, 4, -5, 5)
    x = _rand_x(d, 300 + d, -10, 10)
    eye = np.eye(d, dtype=np.float32)
    assert oracle.fitness(oracle.DENSE, x, s, a=eye) == oracle.fitness(oracle.SPHERE, x, s)


def test_dense_diagonal():
    d = 50
    rng = np.random.default_rng(9)
    diag = rng.uniform(-3, 3, d).astype(np.float32)
    s = rng.uniform(-5, 5, d).astype(np.float32)
    x = _rand_x(d, 9, -10, 10)
    dd = x.astype(np.float64) - s.astype(np.float64)
    ref = math.fsum((float(a) * u) ** 2 for a, u in zip(diag, dd))
    assert oracle.fitness(oracle.DENSE, x, s, a=np.diag(diag)) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("d", [3, 64, 256])
def test_dense_matches_library_products(d):
    s, _, a = make_objective("dense", d, 5, -5, 5)
    x = _rand_x(d, 400 + d, -10, 10)
    A = a.astype(np.float64)
    dd = x.astype(np.float64) - s.astype(np.float64)
    y = A @ dd
    got = oracle.fitness(oracle.DENSE, x, s, a=a)
    assert got == pytest.approx(float(y @ y), rel=1e-12)
    assert got == pytest.approx(float(dd @ (A.T @ A) @ dd), rel=1e-10)
    # The row index of A is the output index: A^T gives a different value.
    yt = A.T @ dd
    assert abs(got - float(yt @ yt)) > 1e-6 * got


def test_objectives_are_nonnegative_and_scale():
    d = 40
    s, w, a = make_objective("ripple", d, 6, -5, 5)
    x = _rand_x(d, 6, -10, 10)
    assert oracle.fitness(oracle.RIPPLE, x, s, w) > 0
    # Sphere is homogeneous of degree 2 in (x - s) when s = 0.
    z = np.zeros(d, np.float32)
    f1 = oracle.fitness(oracle.SPHERE, x, z)
    f2 = oracle.fitness(oracle.SPHERE, (2 * x).astype(np.float32), z)
    assert f2 == pytest.approx(4 * f1, rel=1e-14)
