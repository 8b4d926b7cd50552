"""Pins of the oracle's dense gradient and of the gradient polish.

The gradient of f(x) = ||A (x - s)||^2 is 2 A^T A (x - s); the polish is
projected gradient descent on every pBest with accept-if-better (an
extension outside the paper).  The pins: a library matrix product, FP64
central differences (exact for a quadratic up to rounding), the identity
matrix (where a step has a closed form), descent and projection properties,
and the acceptance rule."""
import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import make_objective

D_CFG = 256  # the dense workload's dimension


def instance(d, seed=3, s_range=(-5.0, 5.0)):
    s, _, a = make_objective("dense", d, seed, *s_range)
    return s, a


def test_gradient_equals_library_product():
    rng = np.random.default_rng(1)
    for d in (1, 5, 33, 64):
        s, a = instance(d, seed=d)
        A = a.astype(np.float64)
        for _ in range(3):
            x = rng.uniform(-10, 10, d)
            g = oracle.dense_grad(x, s, a)
            ref = 2.0 * A.T @ (A @ (x - s.astype(np.float64)))
            assert np.max(np.abs(g - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
            # Not the gradient through A instead of its transpose.
            if d > 1:
                wrong = 2.0 * A @ (A.T @ (x - s.astype(np.float64)))
                assert np.max(np.abs(g - wrong)) > 1e-6 * np.max(np.abs(ref))


def test_gradient_matches_central_differences():
    """FP64 central differences with h = 1e-6: a few points of the full
    256-dimensional instance and 64 points of a 16-dimensional one."""
    h = 1e-6
    for d, npts, seed in ((D_CFG, 3, 5), (16, 64, 6)):
        s, a = instance(d)
        rng = np.random.default_rng(seed)
        for _ in range(npts):
            x = rng.uniform(-10, 10, d)
            g = oracle.dense_grad(x, s, a)
            e = np.eye(d)
            fd = np.array([(oracle.dense_f64(x + h * e[j], s, a) - oracle.dense_f64(x - h * e[j], s, a))
                           / (2 * h) for j in range(d)])
            assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g))


def test_f64_objective_agrees_with_fp32_entry_point():
    s, a = instance(40)
    x = np.random.default_rng(2).uniform(-10, 10, 40).astype(np.float32)
    assert oracle.dense_f64(x.astype(np.float64), s, a) == oracle.fitness(oracle.DENSE, x, s, a=a)
    assert oracle.dense_f64(s.astype(np.float64), s, a) == 0.0
    assert np.all(oracle.dense_grad(s.astype(np.float64), s, a) == 0.0)


def dense_swarm(n, d, a, s, lo=-10.0, hi=10.0, seed=7):
    sw = oracle.Swarm(n, d, oracle.DENSE, lo, hi, 0.4, 0.7, 0.9, seed, s, None, a)
    sw.init()
    return sw


def test_polish_with_identity_matrix_has_a_closed_form():
    """A = I: grad = 2 (p - s), so each step is p <- fl32(clip(p - 2 lr (p - s))),
    the box being the swarm's; one, two and three steps."""
    d, n = 12, 9
    s = np.random.default_rng(3).uniform(-5, 5, d).astype(np.float32)
    a = np.eye(d, dtype=np.float32)
    rejected = 0
    for steps in (1, 2, 3):
        # 0.9 overshoots (|1 - 2 lr| = 0.8, the box clips some values); 1.2
        # diverges (|1 - 2 lr| = 1.4), so those points must be rejected.
        for lr in (0.1, 0.35, 0.9, 1.2):
            sw = dense_swarm(n, d, a, s)
            sw.run(3)
            p0 = sw.p.copy()
            fp0 = sw.fp.copy()
            sw.polish(steps, lr)
            q = p0.copy()
            for _ in range(steps):
                v = q.astype(np.float64) - lr * 2.0 * (q.astype(np.float64) - s.astype(np.float64))
                q = np.clip(v, -10.0, 10.0).astype(np.float32)
            f = np.array([np.sum((q[i].astype(np.float64) - s) ** 2) for i in range(n)])
            better = f.astype(np.float32) < fp0
            assert np.array_equal(sw.p[better], q[better])
            assert np.array_equal(sw.p[~better], p0[~better])
            assert np.array_equal(sw.improved.astype(bool), better)
            rejected += int((~better).sum())
    assert rejected > 0


def test_polish_half_step_lands_on_the_optimum():
    """A = I and lr = 1/2: one step maps every pBest to s exactly."""
    d = 8
    s = np.random.default_rng(4).uniform(-5, 5, d).astype(np.float32)
    sw = dense_swarm(20, d, np.eye(d, dtype=np.float32), s)
    sw.run(2)
    assert sw.polish(1, 0.5) == 20
    assert np.all(sw.p == s) and np.all(sw.fp == 0.0)
    assert sw.fp64[sw.gidx] == 0.0


def test_polish_descends_and_keeps_the_invariants():
    """lr = 0.05 / sigma_max(A)^2 is well inside the descent range of the
    quadratic (step < 1 / L with L = 2 sigma_max^2): nearly every pBest
    improves; fP never increases; X is untouched; gBest is the argmin."""
    d, n = 64, 50
    s, a = instance(d)
    sigma = np.linalg.norm(a.astype(np.float64), 2)
    lr = 0.05 / sigma**2
    sw = dense_swarm(n, d, a, s, lo=-10.0, hi=10.0)
    sw.run(10)
    x0, p0, fp0 = sw.x.copy(), sw.p.copy(), sw.fp.copy()
    replaced = sw.polish(5, lr)
    assert replaced >= n - 1
    assert np.all(sw.fp <= fp0)
    assert np.array_equal(sw.x, x0)
    assert np.all((sw.p >= -10.0) & (sw.p <= 10.0))
    assert sw.gidx == oracle.argmin(sw.fp)
    assert np.array_equal(sw.g, sw.p[sw.gidx])
    # Each improved pBest moved; the others did not.
    moved = np.any(sw.p != p0, axis=1)
    assert np.array_equal(moved, sw.improved.astype(bool))
    # The stored FP64 fitness is that of the stored point.
    for i in np.where(moved)[0][:5]:
        assert sw.fp64[i] == oracle.fitness(oracle.DENSE, sw.p[i], s, a=a)


def test_polish_projects_onto_the_box():
    """A huge step sends values past the bounds: the polished points lie on
    the box faces where the plain step would have left it."""
    d, n = 10, 30
    s, a = instance(d)
    sw = dense_swarm(n, d, a, s, lo=-1.0, hi=1.0)
    sw.run(2)
    p0 = sw.p.copy()
    sw.polish(1, 50.0)
    q = p0.astype(np.float64) - 50.0 * np.array([oracle.dense_grad(r.astype(np.float64), s, a) for r in p0])
    outside = (q < -1.0) | (q > 1.0)
    assert outside.any()
    imp = sw.improved.astype(bool)
    assert np.all((sw.p >= -1.0) & (sw.p <= 1.0))
    assert np.all(np.abs(sw.p[imp][outside[imp]]) == 1.0)


def test_polish_needs_a_dense_swarm():
    sw = oracle.Swarm(4, 3, oracle.SPHERE, -1.0, 1.0, 0.4, 0.7, 0.9, 1, np.zeros(3, np.float32))
    sw.init()
    with pytest.raises(ValueError):
        sw.polish(1, 0.1)
