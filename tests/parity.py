"""Helpers for comparing the GPU library with the CPU oracle.

The bar:
* positions X, pBests P and gBest g: bit-exact (they are FP32 values that are
  only drawn or copied, never computed);
* Philox words, branch choices and particle indices: bit-exact;
* FP32 fitness against the oracle's FP64 value: relative error <= REL_TOL;
* a pBest or gBest decision may differ from the oracle's only when the two
  FP64 values it compares are within BAND of each other (both sides then hold
  a correct FP32 decision); the test counts such events and re-synchronises
  the GPU to the oracle's state, which is an input to the GPU, never the
  other way round.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2110_01470_amd.inputs import make_objective

REL_TOL = 1e-5
BAND = 2 * REL_TOL
KIND = {"sphere": oracle.SPHERE, "ripple": oracle.RIPPLE, "dense": oracle.DENSE,
        **{f"f{k}": oracle.F1 + k - 1 for k in range(1, 10)}}
# Table 3.2's functions subtract large constants near their optima (Ackley,
# Griewank, Rastrigin, Schwefel 2.26), so their FP32 values are bounded
# against the magnitude of the sums combined, not against |f|: the bar is
# REL_TOL * scale(x) with scale from oracle.fitness_scale (= f for sums of
# non-negative terms), and near-ties are widened by the same amount.
PAPER = {f"f{k}" for k in range(1, 10)}


def near(a, b, band=BAND, slack=0.0):
    return abs(a - b) <= band * max(abs(a), abs(b)) + slack


class Pair:
    """An oracle swarm and a GPU swarm built from the same seeded instance."""

    def __init__(self, kind, n, d, lo=-100.0, hi=100.0, cg=0.4, cp=0.7, cw=0.9, seed=1,
                 s_range=(-50.0, 50.0), order=oracle.ORDER_GPS, engine="auto", lanes=0,
                 swarm_id=0, trace_cap=0, storage="auto", objective=None, gpu=None,
                 contraction="auto"):
        """`objective` = (s, w, a) overrides the seeded instance; `gpu` is an
        already built GPU side (a swarm of a batch) instead of a new Swarm."""
        from paper_2110_01470_amd.binding import Swarm

        self.kind, self.n, self.d = kind, n, d
        self.lo, self.hi = lo, hi
        if objective is None:
            objective = (None, None, None) if kind in PAPER else make_objective(kind, d, seed, *s_range)
        self.s, self.w, self.a = objective
        self.orc = oracle.Swarm(n, d, KIND[kind], lo, hi, cg, cp, cw, seed, self.s, self.w,
                                self.a, swarm=swarm_id, order=order)
        if gpu is None:
            gpu = Swarm(n, d, kind, lo, hi, cg, cp, cw, seed, self.s, self.w, self.a,
                        swarm_id=swarm_id, order=order, engine=engine, lanes=lanes,
                        trace_cap=trace_cap, storage=storage, contraction=contraction)
        self.gpu = gpu
        self.orc.init()
        self.band_events = 0
        self.prev_fp64 = self.orc.fp64.copy()

    def step(self, k=1):
        """k generations on both sides, comparing after each."""
        for _ in range(k):
            self.prev_fp64 = self.orc.fp64.copy()
            self.orc.step()
            self.gpu.step()
            self.compare()

    def scale(self, rows):
        """Per-row magnitude the fitness bar is relative to."""
        if self.kind not in PAPER:
            return None
        k = KIND[self.kind]
        return np.array([oracle.fitness_scale(k, r) for r in rows])

    def compare(self, check_fitness=True):
        orc, gpu = self.orc, self.gpu
        x, p, fp, t = gpu.state()
        assert t == orc.t
        assert np.array_equal(x, orc.x), _first_diff(x, orc.x, "x")
        resync = False
        rows = np.where(~np.all(p == orc.p, axis=1))[0]
        sc_p = self.scale(orc.p)
        sc_x = self.scale(orc.x)
        slack = (lambda i: 0.0) if sc_p is None else (
            lambda i: 2 * REL_TOL * max(sc_p[i], sc_x[i]))
        self.slack = slack
        for i in rows:
            # The GPU and the oracle took different pBest decisions for i.
            assert near(orc.fx64[i], self.prev_fp64[i], slack=slack(i)), (
                f"pBest decision of particle {i} differs outside the band: "
                f"f(x')={orc.fx64[i]!r} fP={self.prev_fp64[i]!r}")
            resync = True
        same = np.ones(self.n, bool)
        same[rows] = False
        if check_fitness:
            ref = orc.fp64[same]
            got = fp[same].astype(np.float64)
            err = np.abs(got - ref)
            lim = REL_TOL * (np.abs(ref) if sc_p is None else sc_p[same])
            bad = np.where(err > lim)[0]
            assert bad.size == 0, (
                f"fitness off by more than {REL_TOL} relative at {bad[:5]}: "
                f"{got[bad[:5]]} vs {ref[bad[:5]]}")
        g, fg, gidx, gen = gpu.best()
        assert gen == orc.t
        assert np.array_equal(g, p[gidx])
        if gidx != orc.gidx:
            assert near(orc.fp64[gidx], orc.fp64[orc.gidx],
                        slack=slack(gidx) + slack(orc.gidx)) or resync, (
                f"gBest index {gidx} vs oracle {orc.gidx} outside the band")
            resync = True
        else:
            assert np.array_equal(g, orc.g)
            if check_fitness:
                assert near(fg, orc.fp64[orc.gidx], REL_TOL, slack=slack(gidx) / 2)
        if resync:
            self.band_events += 1
            gpu.set_state(orc.x, orc.p, orc.fp, orc.t)


def _first_diff(a, b, name):
    idx = np.argwhere(a != b)
    if idx.size == 0:
        return f"{name} equal"
    i = tuple(idx[0])
    return f"{name} differs at {i}: {a[i]!r} vs {b[i]!r} ({len(idx)} elements differ)"


def oracle_run_with_trace(orc, k):
    """k oracle generations; per generation the gBest fitness (FP64), gBest
    index, improved count, and whether any pBest decision was a near-tie."""
    fg, gi, im, tie = [], [], [], []
    for _ in range(k):
        prev = orc.fp64.copy()
        orc.step()
        fg.append(orc.fp64[orc.gidx])
        gi.append(orc.gidx)
        im.append(int(orc.improved.sum()))
        close = np.abs(orc.fx64 - prev) <= BAND * np.maximum(np.abs(orc.fx64), np.abs(prev))
        srt = np.sort(orc.fp64)
        gtie = srt.size > 1 and near(srt[0], srt[1])
        tie.append(bool(close.any()) or bool(gtie))
    return np.array(fg), np.array(gi, np.uint32), np.array(im, np.uint32), np.array(tie)


def compare_after_run(pair, first, trace):
    """After the oracle ran len(trace[0]) generations with oracle_run_with_trace
    and the GPU ran the same generations in one go: either the states agree
    (then the GPU trace must match the oracle's), or the first generation
    whose gBest index or improved count differs must be one in which the
    oracle saw a near-tie decision.  Returns the number of such divergences
    (0 or 1); a diverged swarm is re-synchronised to the oracle."""
    fgs, gis, ims, ties = trace
    x, p, fp, t = pair.gpu.state()
    fg, gi, im = pair.gpu.trace(first, len(gis))
    if np.array_equal(x, pair.orc.x) and np.array_equal(p, pair.orc.p):
        assert np.array_equal(gi, gis), "equal states but different gBest indices"
        assert np.array_equal(im, ims), "equal states but different improvement counts"
        assert np.all(np.abs(fg - fgs) <= REL_TOL * np.abs(fgs))
        pair.prev_fp64 = pair.orc.fp64.copy()
        pair.compare()
        return 0
    diff = np.where((gi != gis) | (im != ims))[0]
    assert diff.size > 0, "states differ although every traced decision agrees"
    k = int(diff[0])
    assert ties[k], f"divergence at generation {first + k} without a near-tie in the oracle"
    pair.gpu.set_state(pair.orc.x, pair.orc.p, pair.orc.fp, pair.orc.t)
    return 1
