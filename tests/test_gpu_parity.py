"""GPU library against the CPU oracle, through the C ABI.

Bit-exact positions, pBests, gBest indices and random words; FP32 fitness
within 1e-5 relative of the oracle's FP64 value; decisions may differ only
inside the near-tie band (see tests/parity.py)."""
import os

import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import WORKLOADS
from parity import BAND, REL_TOL, Pair, compare_after_run, near, oracle_run_with_trace

pytestmark = pytest.mark.gpu


def wl_pair(name, **over):
    wl = WORKLOADS[name]
    kw = dict(lo=wl.lo, hi=wl.hi, cg=wl.cg, cp=wl.cp, cw=wl.cw, seed=wl.seed,
              s_range=(wl.s_lo, wl.s_hi))
    n = over.pop("n", wl.n)
    d = over.pop("d", wl.d)
    kw.update(over)
    return Pair(wl.kind, n, d, **kw)


@pytest.mark.parametrize("n,d,t,swarm", [(3, 1, 0, 0), (7, 30, 5, 0), (5, 1001, 17, 3),
                                         (64, 256, 1, 9), (2, 6, 4294967295, 1)])
def test_device_words_match_oracle(n, d, t, swarm):
    pair = Pair("sphere", n, d, seed=0x1234_5678_9ABC_DEF0, swarm_id=swarm)
    got = pair.gpu.debug_rng(t)
    assert np.array_equal(got, oracle.words(0x1234_5678_9ABC_DEF0, swarm, t, n, d))


ROCRAND_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rocrand_ref",
                           "librocrand_philox.so")


@pytest.mark.parametrize("n,d,t,swarm,seed", [(300, 1000, 1, 0, 2), (64, 256, 4294967295, 7, 3),
                                              (1000, 101, 77, 511, 0x1234_5678_9ABC_DEF0),
                                              (5, 3, 0, 1, 2**64 - 1)])
def test_device_words_match_rocrand(n, d, t, swarm, seed):
    """A second implementation of Philox4x32-10: rocRAND's device generator
    (run, not read; tests/rocrand_ref), with the counter (chunk, particle,
    generation, swarm) mapped onto its (seed, subsequence, offset)."""
    import ctypes

    lib = ctypes.CDLL(ROCRAND_LIB)
    lib.rocrand_philox_blocks.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.c_void_p]
    lib.rocrand_philox_blocks.restype = ctypes.c_int
    pair = Pair("sphere", n, d, seed=seed, swarm_id=swarm)
    got = pair.gpu.debug_rng(t)
    chunks = (d + 3) // 4
    q, i = np.meshgrid(np.arange(chunks, dtype=np.uint32), np.arange(n, dtype=np.uint32))
    ctr = np.stack([q.ravel(), i.ravel(), np.full(q.size, t, np.uint32),
                    np.full(q.size, swarm, np.uint32)], axis=1).astype(np.uint32)
    out = np.zeros_like(ctr)
    assert lib.rocrand_philox_blocks(seed, ctr.ctypes.data, ctr.shape[0], out.ctypes.data) == 0
    ref = out.reshape(n, chunks * 4)[:, :d]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,d,offset", [(262150, 4, 0), (40, 1000, 0), (9, 8, 1), (33, 12, 2)])
def test_device_words_grid_and_store_paths(n, d, offset):
    """The word kernel's grid-stride loop over particles (n above 4 * 65535),
    several chunk blocks per row, and the scalar stores taken when the
    output is not 16-byte aligned."""
    import torch

    pair = Pair("sphere", n, d, seed=77, swarm_id=5)
    buf = torch.full((n * d + offset,), -1, dtype=torch.int32, device="cuda")
    out = buf[offset:]
    pair.gpu.rng_words_into(9, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(n, d)
    assert np.array_equal(got, oracle.words(77, 5, 9, n, d))
    if offset:
        assert np.all(buf[:offset].cpu().numpy() == -1)


@pytest.mark.parametrize("kind,n,d,engine", [
    ("sphere", 100, 30, "resident"), ("sphere", 100, 30, "stream"),
    ("ripple", 301, 1000, "stream"), ("ripple", 33, 61, "resident"),
    ("dense", 130, 256, "stream"), ("dense", 70, 100, "stream"), ("dense", 3, 1, "stream"),
    ("sphere", 1, 1, "stream"), ("ripple", 1, 3, "resident"),
])
def test_initialisation_matches_oracle(kind, n, d, engine):
    # Dense swarms here take the FP32 contraction (the split one, the
    # default, has its own tests).
    pair = Pair(kind, n, d, lo=-10.0, hi=10.0, s_range=(-5.0, 5.0), seed=11, engine=engine,
                contraction="f32")
    pair.compare()
    # P^0 = X^0 and the trace of the initialisation counts every particle.
    fg, gi, im = pair.gpu.trace(0, 1)
    assert gi[0] == pair.orc.gidx and im[0] == n


def test_sphere_n100_d30_full_run_every_generation():
    """The small sphere workload, all 1000 generations, compared after each."""
    pair = wl_pair("sphere_n100_d30", engine="resident")
    pair.step(WORKLOADS["sphere_n100_d30"].generations)
    assert pair.band_events <= 2


def test_sphere_n100_d30_single_launch_equals_oracle_run():
    """All 1000 generations in one RESIDENT launch against the oracle's run:
    equal states and traces, or the first generation whose gBest index or
    improvement count differs is one where the oracle saw a near-tie."""
    wl = WORKLOADS["sphere_n100_d30"]
    pair = wl_pair("sphere_n100_d30", engine="resident")
    trace = oracle_run_with_trace(pair.orc, wl.generations)
    pair.gpu.run(wl.generations)
    assert compare_after_run(pair, 1, trace) in (0, 1)


@pytest.mark.parametrize("engine,lanes", [("stream", 8), ("stream", 16), ("stream", 64),
                                          ("resident", 0)])
def test_sphere_mappings(engine, lanes):
    pair = wl_pair("sphere_n100_d30", engine=engine, lanes=lanes)
    pair.step(60)


@pytest.mark.parametrize("storage", ["u24", "f32"])
@pytest.mark.parametrize("n,d,order", [(301, 1000, oracle.ORDER_GPS), (67, 1001, oracle.ORDER_GPS),
                                       (45, 37, oracle.ORDER_EQ21), (9, 5, oracle.ORDER_GPS),
                                       (130, 257, oracle.ORDER_EQ21), (1, 1000, oracle.ORDER_GPS)])
def test_ripple_generations(n, d, order, storage):
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.8, 0.6, 0.3)
    pair = wl_pair("ripple_n65536_d1000", n=n, d=d, order=order, cg=cg, cp=cp, cw=cw,
                   engine="stream", storage=storage)
    pair.step(25)


@pytest.mark.parametrize("storage", ["u24", "f32"])
@pytest.mark.parametrize("kind,n,d,order,lanes", [
    ("ripple", 5, 1025, oracle.ORDER_GPS, 0),        # first size without LDS staging
    ("ripple", 3, 5003, oracle.ORDER_EQ21, 0),       # many chunks per lane, ragged
    ("ripple", 7, 2048, oracle.ORDER_GPS, 8),        # 64 chunks per lane
    ("sphere", 2, 1 << 20, oracle.ORDER_GPS, 0),     # the largest d a swarm takes
    ("sphere", 2, (1 << 20) - 3, oracle.ORDER_EQ21, 0),
])
def test_unstaged_and_largest_rows(kind, n, d, order, lanes, storage):
    """Rows of more than 256 chunks: the shift, weights and gBest are read
    from global memory instead of LDS, and each lane walks many chunks; up to
    d = 2^20, the largest the library accepts."""
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.8, 0.6, 0.3)
    name = "ripple_n65536_d1000" if kind == "ripple" else "sphere_n100_d30"
    pair = wl_pair(name, n=n, d=d, order=order, cg=cg, cp=cp, cw=cw, engine="stream",
                   lanes=lanes, storage=storage)
    pair.compare()
    pair.step(3)


@pytest.mark.parametrize("lanes", [8, 16, 32, 64])
def test_sphere_u24_storage_mappings(lanes):
    pair = wl_pair("sphere_n100_d30", engine="stream", lanes=lanes, storage="u24")
    pair.step(40)


def test_u24_storage_rejects_off_grid_state():
    from paper_2110_01470_amd.binding import E_INVAL, SSOError

    pair = wl_pair("ripple_n65536_d1000", n=20, d=9, engine="stream", storage="u24")
    x, p, fp, t = pair.gpu.state()
    bad = x.copy()
    bad[3, 4] = np.nextafter(bad[3, 4], np.float32(np.inf))
    if np.all(bad == x):
        bad[3, 4] = np.float32(0.1234567)
    with pytest.raises(SSOError) as e:
        pair.gpu.set_state(bad, p, fp, t)
    assert e.value.code == E_INVAL
    # The state is unchanged and the run continues in step with the oracle.
    pair.step(3)


@pytest.mark.parametrize("n,d,order", [(130, 256, oracle.ORDER_GPS), (64, 256, oracle.ORDER_EQ21),
                                       (70, 100, oracle.ORDER_GPS), (100, 30, oracle.ORDER_GPS),
                                       (65, 255, oracle.ORDER_GPS), (17, 1, oracle.ORDER_GPS)])
def test_dense_generations(n, d, order):
    cg, cp, cw = (0.4, 0.7, 0.9) if order == oracle.ORDER_GPS else (0.8, 0.6, 0.3)
    pair = wl_pair("dense_n16384_d256", n=n, d=d, order=order, cg=cg, cp=cp, cw=cw,
                   contraction="f32")
    pair.step(20)


def test_pure_random_search_and_single_source_rules():
    # Every threshold at 0 (all fresh) and cg = cp = cw (gBest or fresh only).
    for cg, cp, cw in ((0.0, 0.0, 0.0), (0.5, 0.5, 0.5), (0.0, 0.6, 0.6)):
        pair = Pair("ripple", 40, 50, lo=-3.0, hi=3.0, cg=cg, cp=cp, cw=cw, s_range=(-1, 1), seed=5)
        pair.step(10)


@pytest.mark.parametrize("storage", ["auto", "f32"])
def test_ripple_n65536_d1000_full_size(storage):
    """The large ripple workload at full size, as the benchmark launches it
    (auto storage), and with FP32 rows."""
    pair = wl_pair("ripple_n65536_d1000", storage=storage)
    pair.compare()
    pair.step(2)


def test_dense_n16384_d256_full_size():
    """The dense workload at full size with the FP32 contraction."""
    pair = wl_pair("dense_n16384_d256", contraction="f32")
    pair.compare()
    pair.step(2)


def test_one_generation_from_oracle_states():
    """Lockstep: the GPU is handed the oracle's state of generation t and must
    produce the oracle's generation t + 1."""
    pair = wl_pair("ripple_n65536_d1000", n=200, d=300)
    orc = pair.orc
    for _ in range(4):
        orc.run(7)
        pair.gpu.set_state(orc.x, orc.p, orc.fp, orc.t)
        pair.prev_fp64 = orc.fp64.copy()
        orc.step()
        pair.gpu.step()
        pair.compare()


@pytest.mark.parametrize("storage", ["u24", "f32"])
def test_repeatable_and_resumable(storage):
    kw = dict(n=96, d=200, storage=storage)
    a = wl_pair("ripple_n65536_d1000", **kw).gpu
    b = wl_pair("ripple_n65536_d1000", **kw).gpu
    a.run(30)
    for _ in range(30):
        b.step()
    sa, sb = a.state(), b.state()
    for u, v in zip(sa[:3], sb[:3]):
        assert np.array_equal(u, v)
    # Checkpoint at 12, resume in a fresh context, finish at 30.
    c = wl_pair("ripple_n65536_d1000", **kw).gpu
    c.run(12)
    x, p, fp, t = c.state()
    d_ = wl_pair("ripple_n65536_d1000", **kw).gpu
    d_.set_state(x, p, fp, t)
    d_.run(18)
    sd = d_.state()
    for u, v in zip(sa[:3], sd[:3]):
        assert np.array_equal(u, v)


def test_resident_and_stream_engines_agree():
    r = wl_pair("sphere_n100_d30", engine="resident").gpu
    s = wl_pair("sphere_n100_d30", engine="stream").gpu
    r.run(200)
    s.run(200)
    for u, v in zip(r.state()[:3], s.state()[:3]):
        assert np.array_equal(u, v)
    assert r.best()[2] == s.best()[2]


def test_trace_matches_oracle():
    pair = wl_pair("ripple_n65536_d1000", n=500, d=64)
    fgs, gis, ims = [pair.orc.fp64[pair.orc.gidx]], [pair.orc.gidx], [pair.n]
    for _ in range(40):
        pair.step()
        fgs.append(pair.orc.fp64[pair.orc.gidx])
        gis.append(pair.orc.gidx)
        ims.append(int(pair.orc.improved.sum()))
    if pair.band_events:
        pytest.skip("a near-tie re-synchronised the run; covered by the parity checks")
    fg, gi, im = pair.gpu.trace(0, 41)
    assert np.array_equal(gi, np.array(gis, np.uint32))
    assert np.array_equal(im, np.array(ims, np.uint32))
    assert np.all(np.abs(fg - np.array(fgs)) <= REL_TOL * np.abs(np.array(fgs)))
    assert np.all(np.diff(fg) <= 0)


def test_trace_window_and_errors():
    from paper_2110_01470_amd.binding import E_STATE, SSOError

    pair = wl_pair("sphere_n100_d30", engine="stream", trace_cap=8)
    pair.gpu.run(20)
    pair.gpu.trace(15, 6)
    with pytest.raises(SSOError) as e:
        pair.gpu.trace(10, 3)
    assert e.value.code == E_STATE
    with pytest.raises(SSOError):
        pair.gpu.trace(18, 5)


@pytest.mark.parametrize("engine", ["stream", "resident"])
def test_zero_work_calls_change_nothing(engine):
    """sso_run(0), an empty trace window and a batch run of 0 generations
    leave every state as it was; the run continues in step with the oracle
    afterwards."""
    from paper_2110_01470_amd.binding import Batch

    pair = wl_pair("sphere_n100_d30", n=37, d=30, engine=engine)
    pair.step(3)
    before = pair.gpu.state()
    pair.gpu.run(0)
    after = pair.gpu.state()
    for u, v in zip(before[:3], after[:3]):
        assert np.array_equal(u, v)
    assert before[3] == after[3] == 3
    fg, gi, im = pair.gpu.trace(1, 0)
    assert fg.size == gi.size == im.size == 0
    pair.step(2)

    s = np.zeros(9, np.float32)
    w = np.ones(9, np.float32)
    batch = Batch([dict(n=20, d=9, kind="ripple", lo=-5.0, hi=5.0, cg=0.4, cp=0.7, cw=0.9,
                        seed=3, s=s, w=w)])
    batch.run(2)
    b0 = batch.view(0).state()
    batch.run(0)
    b1 = batch.view(0).state()
    for u, v in zip(b0[:3], b1[:3]):
        assert np.array_equal(u, v)
    assert batch.results()[3] == 2


def test_dropping_a_swarm_with_queued_work_is_safe():
    """A swarm dropped while its own stream still runs its generations: its
    workspace must not be handed to the next allocation before that work
    ends, so a swarm created right after (on the current stream) evolves
    exactly as the oracle does."""
    import torch

    from paper_2110_01470_amd.binding import Swarm

    wl = WORKLOADS["ripple_n65536_d1000"]
    s, w, _ = wl.objective()
    side = torch.cuda.Stream()
    busy = Swarm(4096, wl.d, "ripple", wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w,
                 engine="stream", stream=side)
    busy.run(100)  # several milliseconds of work queued on `side`
    del busy
    pair = wl_pair("ripple_n65536_d1000", n=4096, d=wl.d, engine="stream")
    pair.step(3)
    side.synchronize()
    pair.compare()
