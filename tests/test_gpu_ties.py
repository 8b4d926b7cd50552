"""gBest over particles in different workgroups and gBest sub-slots, on the
device: exact ties go to the lowest index, -0 and +0 are the same fitness,
and NaN sorts above every number (Algorithm 4's argmin, as the oracle's
orc_argmin takes it); a NaN pBest is replaced by any number and a NaN fitness
never replaces a pBest (Algorithm 3 in the same order).

The tied particles hold the shift s itself as pBest and position, with s
chosen on the draw grid so that their fitness is exactly zero on both sides;
no other particle can reach zero in a few generations, and theirs cannot
improve (any fresh draw moves a coordinate off s), so the device's reduction
over workgroups and sub-slots must return the lowest tied index after every
generation."""
import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.binding import Swarm
from paper_2110_01470_amd.inputs import make_objective

pytestmark = pytest.mark.gpu


def grid_shift(kind, d, lo, hi, seed):
    """A shift whose every coordinate is a point of the draw grid (the value
    the initialisation map gives for word u << 8), and the rest of the seeded
    instance."""
    s, w, a = make_objective(kind, d, seed, lo / 2, hi / 2)
    rule = oracle.Rule(0.4, 0.7, 0.9, lo, hi)
    rng = np.random.Generator(np.random.PCG64(seed + 99))
    u = rng.integers(1 << 22, 3 << 22, size=d)
    s = np.array([rule.init_value(int(v) << 8) for v in u], np.float32)
    return s, w, a


# (kind, n, d, box, storage or contraction, lanes, tied particles (the first
# with fitness +0, then alternately -0 and +0), particles given a NaN pBest
# fitness).  Comments give workgroup -> sub-slot for the tied particles.
CASES = [
    # 32 lanes, 8 particles per workgroup, sub-slot = workgroup mod 64:
    # 100 -> 12 -> 12, 1536 -> 192 -> 0, 4111 -> 513 -> 1, 60009 -> 7501 -> 13
    ("ripple", 65536, 1000, (-100.0, 100.0), dict(storage="u24"), [100, 1536, 4111, 60009], [3, 57]),
    # 64 lanes, 4 particles per workgroup:
    # 100 -> 25 -> 25, 1536 -> 384 -> 0, 4111 -> 1027 -> 3, 60009 -> 15002 -> 26
    ("ripple", 65536, 1000, (-100.0, 100.0), dict(storage="f32"), [100, 1536, 4111, 60009], [3, 57]),
    # Dense kernels, 64 particles per workgroup:
    # 100 -> 1, 1536 -> 24, 4111 -> 64 -> 0, 16000 -> 250 -> 58
    ("dense", 16384, 256, (-10.0, 10.0), dict(contraction="bf16x3"), [100, 1536, 4111, 16000], [3, 57]),
    ("dense", 16384, 256, (-10.0, 10.0), dict(contraction="f32"), [100, 1536, 4111, 16000], [3, 57]),
    ("dense", 16384, 256, (-10.0, 10.0), dict(contraction="f16x2"), [100, 1536, 4111, 16000], [3, 57]),
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=["ripple_u24", "ripple_f32", "dense_split",
                                                          "dense_f32", "dense_f16x2"])
def test_ties_nan_and_signed_zero_across_workgroups(case):
    kind, n, d, (lo, hi), extra, tied, nans = CASES[case]
    s, w, a = grid_shift(kind, d, lo, hi, 17 + case)
    seed = 23 + case
    okind = {"ripple": oracle.RIPPLE, "dense": oracle.DENSE}[kind]
    used = oracle.set_threads(16)
    try:
        orc = oracle.Swarm(n, d, okind, lo, hi, 0.4, 0.7, 0.9, seed, s, w, a)
        orc.init()
        gpu = Swarm(n, d, kind, lo, hi, 0.4, 0.7, 0.9, seed, s, w, a, engine="stream", **extra)
        x, p, fp = orc.x.copy(), orc.p.copy(), orc.fp.copy()
        for k, i in enumerate(tied):
            x[i] = s
            p[i] = s
            fp[i] = np.float32(-0.0) if k % 2 else np.float32(0.0)
        fp[nans] = np.float32(np.nan)
        assert oracle.argmin(fp) == tied[0]
        orc.set_state(x, p, fp, 0)
        gpu.set_state(x, p, fp, 0)
        assert orc.gidx == tied[0] and gpu.best()[2] == tied[0]
        for gen in range(1, 4):
            orc.step()
            gpu.step()
            g, fg, gidx, t = gpu.best()
            assert t == gen
            # The device's reduction over all workgroups and sub-slots.
            assert gidx == tied[0] == orc.gidx, (gen, gidx, orc.gidx)
            assert fg == 0.0 and np.array_equal(g, s)
            _, gi, im = gpu.trace(gen, 1)
            assert gi[0] == tied[0]
            if gen == 1:
                _, _, fpg, _ = gpu.state()
                # The NaN pBests were replaced by their particles' finite fitness,
                # the tied ones kept theirs (signs included).
                assert np.all(np.isfinite(fpg[nans])) and np.all(orc.improved[nans] == 1)
                for k, i in enumerate(tied):
                    assert fpg[i] == 0.0 and np.signbit(fpg[i]) == bool(k % 2)
                assert np.array_equal(fpg[nans], orc.fp[nans]) or np.all(
                    np.abs(fpg[nans].astype(np.float64) - orc.fp64[nans])
                    <= 1e-5 * np.abs(orc.fp64[nans]))
        gpu.close()
    finally:
        oracle.set_threads(1)
    assert used >= 1


@pytest.mark.parametrize("gen_pair", [(1, 2)])
def test_philox_words_of_two_full_ripple_generations(gen_pair):
    """Every word of two whole generations of the ripple workload's shape
    (65536 x 1000 each, 1.31e8 words) from the device generator against the
    oracle's, word for word."""
    from paper_2110_01470_amd.inputs import WORKLOADS

    wl = WORKLOADS["ripple_n65536_d1000"]
    s, w, _ = wl.objective()
    gpu = Swarm(wl.n, wl.d, wl.kind, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w)
    used = oracle.set_threads(16)
    try:
        total = 0
        for t in gen_pair:
            got = gpu.debug_rng(t)
            ref = oracle.words(wl.seed, 0, t, wl.n, wl.d)
            assert got.shape == ref.shape == (wl.n, wl.d)
            bad = np.argwhere(got != ref)
            assert bad.size == 0, f"generation {t}: {len(bad)} words differ, first at {bad[0]}"
            total += got.size
        assert total == 2 * 65536 * 1000
    finally:
        oracle.set_threads(1)
        gpu.close()
