"""The dense objective's split contractions -- three exact bf16 parts
(contraction="bf16x3") and two scaled fp16 parts (contraction="f16x2") --
against the CPU oracle, through the C ABI: the same bar as the FP32
contraction -- bit-exact positions, pBests and gBest indices, FP32 fitness
within 1e-5 relative of the oracle's FP64 value, decisions apart only inside
the near-tie band."""
import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import WORKLOADS
from parity import Pair, compare_after_run, oracle_run_with_trace

pytestmark = pytest.mark.gpu


def split_pair(n, d, **over):
    wl = WORKLOADS["dense_n16384_d256"]
    kw = dict(lo=wl.lo, hi=wl.hi, cg=wl.cg, cp=wl.cp, cw=wl.cw, seed=wl.seed,
              s_range=(wl.s_lo, wl.s_hi), contraction="bf16x3")
    kw.update(over)
    return Pair("dense", n, d, **kw)


SPLITS = ["bf16x3", "f16x2"]


@pytest.mark.parametrize("contraction", SPLITS)
@pytest.mark.parametrize("n,d", [(130, 256), (70, 100), (3, 1), (64, 32)])
def test_split_initialisation(n, d, contraction):
    pair = split_pair(n, d, lo=-10.0, hi=10.0, s_range=(-5.0, 5.0), seed=11,
                      contraction=contraction)
    pair.compare()
    fg, gi, im = pair.gpu.trace(0, 1)
    assert gi[0] == pair.orc.gidx and im[0] == n


@pytest.mark.parametrize("n,d,order", [(130, 256, oracle.ORDER_GPS), (64, 256, oracle.ORDER_EQ21),
                                       (70, 100, oracle.ORDER_GPS), (100, 30, oracle.ORDER_GPS),
                                       (65, 255, oracle.ORDER_GPS), (17, 1, oracle.ORDER_GPS),
                                       (200, 64, oracle.ORDER_GPS), (129, 160, oracle.ORDER_EQ21)])
@pytest.mark.parametrize("contraction", SPLITS)
def test_split_generations(n, d, order, contraction):
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.8, 0.6, 0.3)
    pair = split_pair(n, d, order=order, cg=cg, cp=cp, cw=cw, contraction=contraction)
    pair.step(20)


@pytest.mark.parametrize("contraction", ["auto", "bf16x3"])
def test_split_full_size(contraction):
    """The dense workload at full size (N=16384, D=256) with a split
    contraction, as the benchmark launches it (AUTO: the fp16 split)."""
    pair = split_pair(16384, 256, contraction=contraction)
    assert pair.gpu.mapping()[3] == ("f16x2" if contraction == "auto" else "bf16x3")
    pair.compare()
    pair.step(2)


def test_f16x2_rows_of_very_different_scale():
    """Rows of A spanning 2^-60 .. 2^40 in magnitude and a box far from the
    shift on some variables: every row gets its own power-of-two scale, so
    each fitness still meets the oracle's bar."""
    from paper_2110_01470_amd.inputs import make_objective

    d = 64
    rng = np.random.Generator(np.random.PCG64(77))
    scales = 2.0 ** rng.integers(-60, 41, size=d)
    a = (rng.standard_normal((d, d)) * scales[:, None]).astype(np.float32)
    s, _, _ = make_objective("dense", d, 31, -900.0, 900.0)
    pair = Pair("dense", 96, d, lo=-1000.0, hi=1000.0, cg=0.4, cp=0.7, cw=0.9, seed=31,
                objective=(s, None, a), contraction="f16x2")
    assert pair.gpu.mapping()[3] == "f16x2"
    pair.compare()
    pair.step(10)


def test_f16x2_state_outside_the_box_is_refused():
    """The fp16 split's scaling holds for positions inside [lo, hi]:
    sso_set_state refuses others and leaves the swarm as it was."""
    from paper_2110_01470_amd.binding import E_INVAL, SSOError

    pair = split_pair(40, 32, contraction="f16x2")
    pair.step(2)
    x, p, fp, t = pair.gpu.state()
    bad = x.copy()
    bad[3, 5] = np.float32(pair.hi + 1.0)
    with pytest.raises(SSOError) as e:
        pair.gpu.set_state(bad, p, fp, t)
    assert e.value.code == E_INVAL
    pair.gpu.set_state(x, p, fp, t)
    pair.step(2)


def test_split_and_f32_contractions_take_the_same_path():
    """Both contractions from one instance, 30 generations in one call each,
    each against the oracle's run: equal states and traces, or the first
    generation whose gBest index or improvement count differs is one where
    the oracle saw a near-tie.  When neither diverged the two runs are equal
    and their fitness values agree within the tolerance."""
    a = split_pair(96, 256, contraction="f32")
    b = split_pair(96, 256)
    trace_a = oracle_run_with_trace(a.orc, 30)
    trace_b = oracle_run_with_trace(b.orc, 30)
    a.gpu.run(30)
    b.gpu.run(30)
    xa, pa, fa, ta = a.gpu.state()
    xb, pb, fb, tb = b.gpu.state()
    assert ta == tb == 30
    div = compare_after_run(a, 1, trace_a) + compare_after_run(b, 1, trace_b)
    if div == 0:
        assert np.array_equal(xa, xb) and np.array_equal(pa, pb)
        np.testing.assert_allclose(fb, fa, rtol=2e-5)
