"""The allocation-free entry point sso_run_static against the workspace entry
points (sso_init, sso_run, sso_get_best) on the same configurations.

Both run the same kernels, so gBest position, fitness and index must be equal
bit for bit.  The calls share the GPU's static state array: every case runs
several calls in a row, later ones with smaller swarms, so a call that relied
on what an earlier one left there would differ."""
import numpy as np
import pytest

from paper_2110_01470_amd import binding
from paper_2110_01470_amd.inputs import make_objective

pytestmark = pytest.mark.gpu


def config(kind, n, d, seed, **kw):
    if kind in ("sphere", "ripple"):
        s, w, _ = make_objective(kind, d, seed, -50.0, 50.0)
        base = dict(lo=-100.0, hi=100.0, cg=0.4, cp=0.7, cw=0.9, s=s, w=w)
    else:  # a Table 3.2 function in Eq. (2.1)'s order, no shift
        base = dict(lo=-30.0, hi=30.0, cg=0.8, cp=0.6, cw=0.3, s=None, w=None,
                    order=binding.ORDER_EQ21)
    base.update(kw)
    return dict(n=n, d=d, kind=kind, seed=seed, **base)


def with_workspace(c, generations):
    c = dict(c)
    args = [c.pop(k) for k in ("n", "d", "kind", "lo", "hi", "cg", "cp", "cw", "seed", "s")]
    sw = binding.Swarm(*args, **c)
    sw.run(generations)
    g, f, idx, t = sw.best()
    sw.close()
    assert t == generations
    return g, f, idx


def static(c, generations):
    c = dict(c)
    args = [c.pop(k) for k in ("n", "d", "kind", "lo", "hi", "cg", "cp", "cw", "seed", "s")]
    return binding.run_static(*args, generations=generations, **c)


def same(a, b):
    ga, fa, ia = a
    gb, fb, ib = b
    assert ia == ib
    assert np.float32(fa).tobytes() == np.float32(fb).tobytes()
    assert ga.dtype == gb.dtype == np.float32 and np.array_equal(ga.view(np.uint32), gb.view(np.uint32))


CASES = [
    # (config, generations), largest first, so later calls reuse a dirty array
    (config("ripple", 3000, 1000, 7), 30),       # STREAM, 24-bit rows, 32 lanes
    (config("ripple", 513, 37, 8), 25),          # ragged d, partial last workgroup
    (config("sphere", 100, 30, 1), 60),          # RESIDENT engine (auto)
    (config("sphere", 100, 30, 1, engine="stream", storage="f32"), 60),
    (config("f4", 350, 50, 1001), 40),           # Table 3.10's Rosenbrock shape
    (config("ripple", 5, 3, 9), 0),              # initialisation only
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_static_run_equals_workspace_run(k):
    c, gens = CASES[k]
    same(static(c, gens), with_workspace(c, gens))


def test_two_calls_in_a_row_second_smaller():
    big, gb = CASES[0]
    small, gs = CASES[1]
    first = static(big, gb)
    second = static(small, gs)
    same(first, with_workspace(big, gb))
    same(second, with_workspace(small, gs))
    # And back: the large swarm again over the small one's leftovers.
    same(static(big, gb), first)


def test_oversized_swarm_is_refused_and_leaves_the_array_usable():
    c = config("ripple", 65536, 1000, 2)
    with pytest.raises(binding.SSOError) as err:
        static(c, 3)
    assert err.value.code == binding.E_NOMEM
    c, gens = CASES[2]
    same(static(c, gens), with_workspace(c, gens))
