"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/sso_oracle.c, builds it,
and runs the CPU pin suite against that build (ORACLE_LIB); at least one pin
must fail.  The mistakes are the kind a careful reader could still make when
writing Philox, Eq. (2.1) or Algorithms 2-4 from the paper."""
import os
import subprocess
import sys

import pytest

from oracle.build import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sso_oracle.c")
PINS = ["tests/test_oracle_philox.py", "tests/test_oracle_rule.py",
        "tests/test_oracle_objectives.py", "tests/test_oracle_swarm.py",
        "tests/test_oracle_gradient.py", "tests/test_oracle_paper.py",
        "tests/test_oracle_convergence.py"]

MUTANTS = {
    "philox multipliers swapped": (
        "uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];",
        "uint64_t p0 = (uint64_t)PHILOX_M1 * (uint64_t)c[0];"),
    "philox key not bumped": ("k[0] += PHILOX_W0;", "k[0] += 0u;"),
    "philox nine rounds": ("for (int r = 0; r < 10; ++r) {", "for (int r = 0; r < 9; ++r) {"),
    "word taken from the wrong lane": ("out[(size_t)i * d + j] = blk[j % 4u];",
                                       "out[(size_t)i * d + j] = blk[(j + 1) % 4u];"),
    "counter fields swapped": ("uint32_t ctr[4] = {j / 4u, i, t, swarm};",
                               "uint32_t ctr[4] = {j / 4u, t, i, swarm};"),
    "threshold rounded down": ("return (uint64_t)ceil(c * 4294967296.0);",
                               "return (uint64_t)floor(c * 4294967296.0);"),
    "pBest and self intervals swapped": (
        "out->src[0] = ORC_SRC_GBEST; out->src[1] = ORC_SRC_PBEST; out->src[2] = ORC_SRC_SELF;",
        "out->src[0] = ORC_SRC_GBEST; out->src[1] = ORC_SRC_SELF; out->src[2] = ORC_SRC_PBEST;"),
    "fresh word not offset": ("uint64_t q = (uint64_t)(word - (uint32_t)r->th[2]) * (uint64_t)r->r;",
                              "uint64_t q = (uint64_t)word * (uint64_t)r->r;"),
    "init uses 23 bits": ("return draw(r, word >> 8);", "return draw(r, word >> 9);"),
    "ripple sine factor dropped": ("double sn = sin(3.0 * dj);", "double sn = sin(dj);"),
    "ripple half dropped": ("f = pairwise(t, d) + 0.5 * pairwise(u, d);",
                            "f = pairwise(t, d) + pairwise(u, d);"),
    "dense matrix transposed": ("t[j] = (double)a[(size_t)k * d + j] * (x[j] - (double)s[j]);",
                                "t[j] = (double)a[(size_t)j * d + k] * (x[j] - (double)s[j]);"),
    "gradient without the factor 2": ("out[j] = 2.0 * pairwise(t, d);", "out[j] = pairwise(t, d);"),
    "gradient through A instead of its transpose": (
        "for (uint32_t k = 0; k < d; ++k) t[k] = (double)a[(size_t)k * d + j] * y[k];",
        "for (uint32_t k = 0; k < d; ++k) t[k] = (double)a[(size_t)j * d + k] * y[k];"),
    "polish step uphill": ("double v = p[j] - lr * g[j];", "double v = p[j] + lr * g[j];"),
    "polish leaves the box": ("                if (v < lo) v = lo;\n                if (v > hi) v = hi;\n", ""),
    "polish keeps every point": ("        if (better) {", "        if (1) {"),
    "polish gradient frozen at the first point": (
        "            for (uint32_t j = 0; j < d; ++j) p[j] = (double)q[j];\n            orc_dense_grad(d, p, sw->s, sw->a, g);",
        "            if (k == 0) {\n                for (uint32_t j = 0; j < d; ++j) p[j] = (double)q[j];\n                orc_dense_grad(d, p, sw->s, sw->a, g);\n            }"),
    "ellipsoid weights from zero": ("t[i] = (double)(i + 1) * x[i] * x[i];",
                                    "t[i] = (double)i * x[i] * x[i];"),
    "Schwefel 1.2 without running sums": ("run += scale ? fabs((double)x[i]) : (double)x[i];",
                                          "run = scale ? fabs((double)x[i]) : (double)x[i];"),
    "Rosenbrock pair reversed": ("const double q = scale ? fabs(xn) + xi * xi : xn - xi * xi;",
                                 "const double q = scale ? fabs(xn) + xi * xi : xi - xn * xn;"),
    "Rastrigin without 10 P": ("f = 10.0 * P + pairwise(t, d);", "f = pairwise(t, d);"),
    "Ackley without e": ("f = scale ? 20.0 * e_a + e_b + 20.0 + e1 : -20.0 * e_a - e_b + 20.0 + e1;",
                         "f = scale ? 20.0 * e_a + e_b + 20.0 + e1 : -20.0 * e_a - e_b + 20.0;"),
    "Griewank index from two": ("prod *= cos((double)x[i] / sqrt((double)(i + 1)));",
                                "prod *= cos((double)x[i] / sqrt((double)(i + 2)));"),
    "Powell groups overlap": (
        "const double x1 = x[4 * k], x2 = x[4 * k + 1], x3 = x[4 * k + 2], x4 = x[4 * k + 3];",
        "const double x1 = x[k], x2 = x[k + 1], x3 = x[k + 2], x4 = x[k + 3];"),
    "Schwefel 2.26 sign flipped": (
        "f = scale ? 418.9829 * P + pairwise(t, d) : 418.9829 * P - pairwise(t, d);",
        "f = scale ? 418.9829 * P + pairwise(t, d) : 418.9829 * P + pairwise(t, d);"),
    "pBest replaced on ties": ("if (less_f32(f32, sw->fp[i])) {", "if (!less_f32(sw->fp[i], f32)) {"),
    "gBest ties to the highest index": ("if (less_f32(fp[i], fp[best])) best = i;",
                                        "if (!less_f32(fp[best], fp[i])) best = i;"),
    "gBest taken before the pBest update": [
        ("    /* Evaluate, then Algorithm 3: replace the pBest on a strict improvement. */",
         "    update_gbest(sw);\n    /* Evaluate, then Algorithm 3: replace the pBest on a strict improvement. */"),
        ("    /* Algorithm 4. */\n    update_gbest(sw);\n    sw->t += 1;", "    sw->t += 1;")],
    "NaN pBest never replaced": ("    if (isnan(b)) return 1;", "    if (isnan(b)) return 0;"),
    "pBest kept forever": ("memcpy(sw->p + (size_t)i * d, xi, sizeof(float) * d);\n            sw->fp[i] = f32;",
                           "sw->fp[i] = f32;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    edits = MUTANTS[name]
    if isinstance(edits, tuple):
        edits = [edits]
    text = open(SRC).read()
    for old, new in edits:
        assert text.count(old) == 1, f"mutation site not unique: {old!r}"
        text = text.replace(old, new)
    src = tmp_path / "sso_oracle.c"
    src.write_text(text)
    lib = build(out=str(tmp_path / "liboracle_mutant.so"), sources=[str(src)])
    env = dict(os.environ, ORACLE_LIB=lib)
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"no pin failed for mutant '{name}'\n{res.stdout[-2000:]}"
