"""Seeded synthetic workloads.

This module only draws objective instances and names workloads; it holds none
of the optimiser's arithmetic.  The CPU oracle and the GPU library are both
fed from it, so the two sides see the same FP32 arrays.

The paper's benchmarks are closed-form functions (Table 3.2) on D=50 with
N=100..350 particles and 1000 iterations (Sec. 3.4.2).  The workloads below
keep that form -- a shifted optimum inside a box -- at the sizes the GPU path
is built for.  Instances come from numpy's PCG64 with the workload's seed:
the shift s ~ U[s_lo, s_hi], the ripple weights w = 10**(3 U[0,1]) (log-uniform
on [1, 1e3]) and the dense matrix A_kj ~ N(0,1)/sqrt(D), each rounded once to
FP32.
"""
from __future__ import annotations

import dataclasses

import numpy as np

KINDS = ("sphere", "ripple", "dense")
PAPER_KINDS = ("f1", "f2", "f3", "f4", "f5", "f6", "f7", "f8", "f9")


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: str          # "sphere" | "ripple" | "dense"
    n: int             # particles (Nsol)
    d: int             # variables per particle (Nvar)
    lo: float          # box [varMin, varMax]
    hi: float
    cg: float
    cp: float
    cw: float
    generations: int   # update generations after initialisation
    seed: int          # objective instance seed and Philox key
    s_lo: float        # shift range
    s_hi: float

    def objective(self):
        return make_objective(self.kind, self.d, self.seed, self.s_lo, self.s_hi)

    def scaled(self, **changes) -> "Workload":
        return dataclasses.replace(self, **changes)


WORKLOADS = {
    w.name: w
    for w in (
        Workload("sphere_n100_d30", "sphere", 100, 30, -100.0, 100.0, 0.4, 0.7, 0.9,
                 1000, 1, -50.0, 50.0),
        Workload("ripple_n65536_d1000", "ripple", 65536, 1000, -100.0, 100.0, 0.4, 0.7, 0.9,
                 1000, 2, -50.0, 50.0),
        Workload("dense_n16384_d256", "dense", 16384, 256, -10.0, 10.0, 0.4, 0.7, 0.9,
                 2000, 3, -5.0, 5.0),
    )
}


@dataclasses.dataclass(frozen=True)
class BatchWorkload:
    """Many independent swarms of uneven size, each with its own objective.

    Swarm k draws its size, dimension and thresholds from PCG64 seeded with
    the sequence (seed + k, 0): n ~ U{n_lo..n_hi}, d ~ U{d_lo..d_hi},
    cg ~ U[cg], cp ~ U[cp], cw ~ U[cw] (disjoint ranges, so cg < cp < cw);
    its objective instance comes from make_objective with seed + k, and its
    Philox key is seed + k with swarm word k."""

    name: str
    kind: str
    count: int
    n_range: tuple
    d_range: tuple
    lo: float
    hi: float
    cg_range: tuple
    cp_range: tuple
    cw_range: tuple
    generations: int
    seed: int
    s_lo: float
    s_hi: float

    def swarm(self, k: int) -> dict:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed + k, 0])))
        n = int(rng.integers(self.n_range[0], self.n_range[1] + 1))
        d = int(rng.integers(self.d_range[0], self.d_range[1] + 1))
        cg = float(rng.uniform(*self.cg_range))
        cp = float(rng.uniform(*self.cp_range))
        cw = float(rng.uniform(*self.cw_range))
        s, w, _ = make_objective(self.kind, d, self.seed + k, self.s_lo, self.s_hi)
        return dict(n=n, d=d, kind=self.kind, lo=self.lo, hi=self.hi, cg=cg, cp=cp, cw=cw,
                    seed=self.seed + k, swarm_id=k, s=s, w=w)

    def swarms(self) -> list:
        return [self.swarm(k) for k in range(self.count)]

    def scaled(self, **changes) -> "BatchWorkload":
        return dataclasses.replace(self, **changes)


BATCH_WORKLOADS = {
    b.name: b
    for b in (
        BatchWorkload("batch512_ripple", "ripple", 512, (32, 4096), (10, 500), -100.0, 100.0,
                      (0.3, 0.5), (0.6, 0.75), (0.85, 0.95), 2000, 4_000_000, -50.0, 50.0),
    )
}


# Table 3.2's feasible bounds; F9's printed [-5.12, 5.12] does not fit the
# values the paper reports for it, so F9 takes Schwefel 2.26's usual box.
PAPER_BOUNDS = {"f1": (-5.12, 5.12), "f2": (-5.12, 5.12), "f3": (-65.536, 65.536),
                "f4": (-2.048, 2.048), "f5": (-5.12, 5.12), "f6": (-32.768, 32.768),
                "f7": (-600.0, 600.0), "f8": (-4.0, 5.0), "f9": (-500.0, 500.0)}


@dataclasses.dataclass(frozen=True)
class PaperWorkload:
    """A Table 3.2 function with the paper's experiment settings (Sec. 3.4):
    P = D variables, N particles, T iterations, and (Cw, Cp, Cg) in the
    interval order Eq. (2.1) prints (self, pBest, gBest, fresh)."""

    name: str
    kind: str
    n: int
    d: int
    lo: float
    hi: float
    cw: float
    cp: float
    cg: float
    generations: int
    seed: int


def _paper(kind, n, seed=1001):
    lo, hi = PAPER_BOUNDS[kind]
    return PaperWorkload(f"paper_{kind}_n{n}_d50", kind, n, 50, lo, hi, 0.3, 0.6, 0.8, 1000, seed)


# Each function at N = 100 (Sec. 3.4.2), and the Rosenbrock speed-up runs of
# Table 3.10 (N = 100, 200, 300, 350).  Replicate runs use seeds 1001..1020.
PAPER_WORKLOADS = {w.name: w for w in [_paper(k, 100) for k in PAPER_KINDS] +
                   [_paper("f4", n) for n in (200, 300, 350)]}


def make_objective(kind: str, d: int, seed: int, s_lo: float, s_hi: float):
    """(s, w, a) as FP32 arrays; w is None unless ripple, a is None unless dense."""
    if kind not in KINDS:
        raise ValueError(f"unknown objective kind {kind!r}")
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.uniform(s_lo, s_hi, size=d).astype(np.float32)
    w = a = None
    if kind == "ripple":
        w = (10.0 ** (3.0 * rng.uniform(0.0, 1.0, size=d))).astype(np.float32)
    elif kind == "dense":
        a = (rng.standard_normal((d, d)) / np.sqrt(d)).astype(np.float32)
    return s, w, a
