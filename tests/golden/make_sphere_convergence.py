"""Convergence record of the small sphere workload (N=100, D=30, box
[-100, 100], shift s ~ U[-50, 50] from seed 1, (cg, cp, cw) = (0.4, 0.7, 0.9),
T=1000) over the Philox seeds 1001..1020, computed with the CPU oracle only.

For every run it records the gBest gap fG - f* (f* = 0 at x = s) after
initialisation and after generation T, and the run's draw floor: in plain SSO
every value a variable ever holds is one of that variable's draws -- the
uniform draws of the initialisation (kernel (I)) and the fresh draws of
Eq. (2.1)'s last interval -- because the other three sources only copy values
of the same variable.  So no position of the run, gBest included, can be
closer to s than the vector x* whose j-th entry is the draw of variable j
closest to s_j, and fG >= f(x*) exactly.  f(x*) is the floor.  For M
uniform draws on a box of width L around an interior s_j, the expected
squared distance of the closest is L^2 / (2 (M + 1)(M + 2)); summed over
the variables with their draw counts this is the expected floor (about
6e-3 here, with about 10,100 draws per variable).

Run from the repository root to rewrite the record:
    python tests/golden/make_sphere_convergence.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2110_01470_amd.inputs import WORKLOADS  # noqa: E402

RECORD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_n100_d30_convergence.txt")
SEEDS = tuple(range(1001, 1021))
WORKLOAD = "sphere_n100_d30"


def closest_draws(rule, seed, n, d, gens, s, lo):
    """Per variable j, the draw of the run closest to s_j (as the oracle
    draws it) and the number of draws of variable j.  Candidates are
    shortlisted with an approximate, monotone map of the words and then
    drawn exactly with the oracle's own maps."""
    words = np.stack([oracle.words(seed, 0, t, n, d) for t in range(gens + 1)])  # [T+1, n, d]
    th = rule.thresholds[2]
    wide = words.astype(np.float64)
    span = rule.span
    approx = np.empty_like(wide)
    approx[0] = lo + np.floor(wide[0] / 256.0) * 2.0 ** -24 * span
    approx[1:] = lo + (wide[1:] - th) / (2.0 ** 32 - th) * span
    drawn = np.ones(words.shape, bool)
    drawn[1:] = words[1:] >= th
    dist = np.where(drawn, np.abs(approx - s.astype(np.float64)), np.inf)
    near = dist.min(axis=(0, 1))
    err = 8.0 * span * 2.0 ** -24 + 1e-4
    best = np.full(d, np.inf)
    x = np.zeros(d, np.float32)
    for t, i, j in np.argwhere(drawn & (dist <= near + 2 * err)):
        k = int(words[t, i, j])
        v = rule.init_value(k) if t == 0 else rule.fresh_value(k)
        dd = abs(float(v) - float(s[j]))
        if dd < best[j]:
            best[j], x[j] = dd, v
    return x, drawn.sum(axis=(0, 1))


def run(seed):
    """One run's record: (seed, gap after init, final gap, floor, expected
    floor, fewest and most draws of a variable) and its FP32 gBest trace."""
    wl = WORKLOADS[WORKLOAD]
    s, _, _ = wl.objective()
    orc = oracle.Swarm(wl.n, wl.d, oracle.SPHERE, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, seed, s)
    orc.init()
    gap0 = float(orc.fp64[orc.gidx])
    trace = [orc.fp[orc.gidx]]
    for _ in range(wl.generations):
        orc.step()
        trace.append(orc.fp[orc.gidx])
    final = float(orc.fp64[orc.gidx])
    rule = oracle.Rule(wl.cg, wl.cp, wl.cw, wl.lo, wl.hi)
    x, counts = closest_draws(rule, seed, wl.n, wl.d, wl.generations, s, float(np.float32(wl.lo)))
    floor = float(oracle.fitness(oracle.SPHERE, x, s))
    width = float(wl.hi - wl.lo)
    expected = float(np.sum(width ** 2 / (2.0 * (counts + 1.0) * (counts + 2.0))))
    return (seed, gap0, final, floor, expected, int(counts.min()), int(counts.max())), \
        np.array(trace, np.float32)


def format_row(row):
    seed, gap0, final, floor, expected, cmin, cmax = row
    return f"{seed} {gap0!r} {final!r} {floor!r} {expected!r} {cmin} {cmax}"


def read_record(path=RECORD):
    rows = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            rows.append((int(f[0]), float(f[1]), float(f[2]), float(f[3]), float(f[4]), int(f[5]),
                         int(f[6])))
    return rows


def main():
    rows = [run(seed)[0] for seed in SEEDS]
    with open(RECORD, "w") as fh:
        fh.write("# Small sphere workload (N=100, D=30, [-100, 100], s from seed 1, (0.4, 0.7, 0.9),\n"
                 "# T=1000), CPU oracle, Philox seeds 1001..1020 (written by\n"
                 "# tests/golden/make_sphere_convergence.py).  Columns: seed, gBest gap after\n"
                 "# initialisation, gBest gap after generation 1000, draw floor f(x*), expected\n"
                 "# floor sum_j L^2 / (2 (M_j + 1)(M_j + 2)), fewest and most draws M_j of a variable.\n")
        for row in rows:
            fh.write(format_row(row) + "\n")
    finals = np.array([r[2] for r in rows])
    floors = np.array([r[3] for r in rows])
    print(f"final gap {finals.mean():.4g} (min {finals.min():.4g}, max {finals.max():.4g}); "
          f"floor {floors.mean():.4g}; expected {np.mean([r[4] for r in rows]):.4g}")


if __name__ == "__main__":
    main()
