"""Table 3.2's benchmark functions on the GPU against the CPU oracle.

The paper's experiment shape (P = 50 variables, N = 100 particles, each
function's feasible box, (Cw, Cp, Cg) = (0.3, 0.6, 0.8) in Eq. (2.1)'s
interval order), generation by generation; positions and pBests bit-exact,
fitness within 1e-5 of the magnitude of the sums it combines (see
tests/parity.py).  Lane counts below the chunk count exercise the running
sums (F3) and neighbour pairs (F4) that cross lanes and passes."""
import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import PAPER_BOUNDS, PAPER_KINDS, PAPER_WORKLOADS
from parity import Pair, compare_after_run, oracle_run_with_trace

pytestmark = pytest.mark.gpu


def paper_pair(kind, n=100, d=50, order=oracle.ORDER_EQ21, seed=1001, engine="stream", **kw):
    lo, hi = PAPER_BOUNDS[kind]
    if order == oracle.ORDER_EQ21:
        cg, cp, cw = 0.8, 0.6, 0.3
    else:
        cg, cp, cw = 0.4, 0.7, 0.9
    return Pair(kind, n, d, lo=lo, hi=hi, cg=cg, cp=cp, cw=cw, seed=seed, order=order,
                engine=engine, **kw)


@pytest.mark.parametrize("kind", PAPER_KINDS)
def test_paper_function_generations(kind):
    pair = paper_pair(kind)
    pair.compare()
    pair.step(20)
    assert pair.band_events <= 2


@pytest.mark.parametrize("kind", PAPER_KINDS)
@pytest.mark.parametrize("order", [oracle.ORDER_EQ21, oracle.ORDER_GPS])
@pytest.mark.parametrize("storage", ["f32", "u24"])
def test_every_function_order_and_storage(kind, order, storage):
    """On the STREAM engine each (function, interval order, row storage) is a
    kernel of its own, with an initialisation twin: a short run of every one
    against the oracle, generation by generation."""
    pair = paper_pair(kind, n=40, d=50, order=order, storage=storage, seed=29)
    assert pair.gpu.mapping()[:2] == ("stream", storage)
    pair.compare()
    pair.step(5)


@pytest.mark.parametrize("kind", ["f3", "f4", "f6", "f7", "f8"])
@pytest.mark.parametrize("d,lanes", [(50, 8), (130, 8), (130, 32), (61, 64), (13, 16)])
def test_cross_lane_functions_over_passes(kind, d, lanes):
    pair = paper_pair(kind, n=37, d=d, lanes=lanes, order=oracle.ORDER_GPS, seed=7)
    pair.compare()
    pair.step(8)


@pytest.mark.parametrize("kind", ["f3", "f4", "f6", "f8", "f9"])
@pytest.mark.parametrize("lanes", [8, 64])
def test_largest_dimension(kind, lanes):
    """d = 1024, the largest the Table 3.2 kernel takes (256 chunks staged)."""
    pair = paper_pair(kind, n=6, d=1024, lanes=lanes, order=oracle.ORDER_GPS, seed=11)
    pair.compare()
    pair.step(4)


@pytest.mark.parametrize("kind,d", [("f8", 3), ("f8", 7), ("f4", 1), ("f3", 1), ("f7", 1),
                                    ("f6", 2), ("f9", 5)])
def test_small_and_ragged_dimensions(kind, d):
    pair = paper_pair(kind, n=9, d=d, storage="f32")
    pair.compare()
    pair.step(6)


@pytest.mark.parametrize("n", [200, 350])
def test_rosenbrock_speedup_shapes(n):
    """Table 3.10's Rosenbrock runs (P = 50, N = 200 and 350)."""
    wl = PAPER_WORKLOADS[f"paper_f4_n{n}_d50"]
    pair = paper_pair("f4", n=wl.n, d=wl.d, seed=wl.seed)
    pair.compare()
    pair.step(10)


def test_full_run_reaches_paper_quality_band():
    """1000 generations of f1 at the paper's settings on the GPU: fG falls
    monotonically to the order of the paper's reported averages (context,
    not parity: Table 3.8 gives 41.0 +- 5.3 for its PSSO), and the final
    gBest is the least pBest fitness."""
    from paper_2110_01470_amd.binding import Swarm

    wl = PAPER_WORKLOADS["paper_f1_n100_d50"]
    sw = Swarm(wl.n, wl.d, "f1", wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, None,
               order=oracle.ORDER_EQ21, engine="stream")
    sw.run(wl.generations)
    fg, _, _ = sw.trace(0, wl.generations + 1)
    assert np.all(np.diff(fg) <= 0)
    g, f, gidx, t = sw.best()
    _, _, fp, _ = sw.state()
    assert t == 1000 and f == fp.min()
    assert 1.0 < f < 200.0
    assert abs(oracle.fitness(oracle.F1, g, None) - f) <= 1e-5 * f


@pytest.mark.parametrize("kind", PAPER_KINDS)
def test_resident_engine_generations(kind):
    """Each function on the RESIDENT engine (one workgroup holds the swarm),
    one launch per step, against the oracle at the paper's shape."""
    pair = paper_pair(kind, engine="resident")
    pair.compare()
    pair.step(12)
    assert pair.band_events <= 2


@pytest.mark.parametrize("kind,n,d,order", [("f4", 200, 50, oracle.ORDER_EQ21),
                                            ("f3", 100, 50, oracle.ORDER_EQ21),
                                            ("f7", 129, 13, oracle.ORDER_GPS),
                                            ("f8", 31, 130, oracle.ORDER_GPS),
                                            ("f6", 5, 1, oracle.ORDER_EQ21),
                                            ("f4", 256, 50, oracle.ORDER_EQ21),
                                            ("f9", 131, 50, oracle.ORDER_GPS),
                                            ("f6", 60, 100, oracle.ORDER_EQ21),
                                            ("f7", 70, 50, oracle.ORDER_GPS)])
def test_resident_equals_stream_bit_for_bit(kind, n, d, order):
    """A whole run in one RESIDENT launch equals the STREAM engine's run at
    the same lanes per particle bit for bit (positions, pBests, fitness,
    trace), up to four particles per thread (N = 256 at D = 50), with 8, 16,
    32 and 64 lanes per particle (D = 13, 50, 100, 130)."""
    from paper_2110_01470_amd.binding import Swarm

    lo, hi = PAPER_BOUNDS[kind]
    cg, cp, cw = (0.8, 0.6, 0.3) if order == oracle.ORDER_EQ21 else (0.4, 0.7, 0.9)
    runs = []
    for engine in ("stream", "resident"):
        sw = Swarm(n, d, kind, lo, hi, cg, cp, cw, 4242, None, order=order, engine=engine)
        sw.run(150)
        runs.append((sw.state(), sw.trace(0, 151), sw.best()))
        sw.close()
    (xa, pa, fa, ta), tra, ba = runs[0]
    (xb, pb, fb, tb), trb, bb = runs[1]
    assert ta == tb == 150
    assert np.array_equal(xa, xb) and np.array_equal(pa, pb)
    assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32))
    for u, v in zip(tra, trb):
        assert np.array_equal(u, v)
    assert ba[2] == bb[2] and np.array_equal(ba[0], bb[0])


def test_resident_single_launch_against_oracle():
    """Table 3.10's N = 200 Rosenbrock swarm, 300 generations in one RESIDENT
    launch, against the oracle's run with the trace rule."""
    wl = PAPER_WORKLOADS["paper_f4_n200_d50"]
    pair = paper_pair("f4", n=wl.n, d=wl.d, seed=wl.seed, engine="resident")
    trace = oracle_run_with_trace(pair.orc, 300)
    pair.gpu.run(300)
    assert compare_after_run(pair, 1, trace) in (0, 1)


@pytest.mark.parametrize("kind,n,d,want", [("f4", 100, 50, ("resident", "f32", 16)),
                                           ("f4", 240, 50, ("resident", "f32", 16)),
                                           ("f4", 241, 50, ("stream", "u24", 16)),
                                           ("f4", 350, 50, ("stream", "u24", 16)),
                                           ("f6", 128, 50, ("resident", "f32", 16)),
                                           ("f6", 129, 50, ("stream", "u24", 16)),
                                           ("f3", 224, 50, ("resident", "f32", 16)),
                                           ("f3", 225, 50, ("stream", "u24", 16)),
                                           ("f5", 177, 50, ("stream", "u24", 16)),
                                           ("f1", 30, 130, ("resident", "f32", 64)),
                                           ("sphere", 100, 30, ("resident", "f32", 8)),
                                           ("ripple", 4096, 1000, ("stream", "u24", 32))])
def test_auto_engine_choice(kind, n, d, want):
    """AUTO takes the one-workgroup engine for Table 3.2's functions up to
    a per-function number of waves of particles per SIMD (N L / 256: 15 for
    f4, 8 for f6, 14 for f3, 11 for f5), STREAM beyond; the context reports
    what it resolved to."""
    from paper_2110_01470_amd.binding import Swarm

    if kind in PAPER_BOUNDS:
        lo, hi = PAPER_BOUNDS[kind]
        s = w = None
    else:
        lo, hi = -100.0, 100.0
        s = np.zeros(d, np.float32)
        w = np.ones(d, np.float32) if kind == "ripple" else None
    sw = Swarm(n, d, kind, lo, hi, 0.8, 0.6, 0.3, 7, s, w, order=oracle.ORDER_EQ21)
    assert sw.mapping()[:3] == want
    sw.run(2)
    assert sw.best()[3] == 2
    sw.close()
