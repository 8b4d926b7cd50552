"""The oracle on the small sphere workload over 20 seeds, against what plain
SSO allows (tests/golden/make_sphere_convergence.py explains the floor):

* the gBest fitness never increases, and falls by more than three orders of
  magnitude over the 1000 generations;
* the final gap is never below the run's draw floor -- the best point the
  run's own draws could assemble -- which holds exactly, so a dropped draw,
  a wrong fresh map or a value created other than by Eq. (2.1) would show;
* the floors average the order-statistic expectation for the run's draw
  counts (about 6e-3) within the spread 20 runs allow;
* the record in tests/golden is reproduced bit for bit."""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location(
    "make_sphere_convergence", os.path.join(HERE, "golden", "make_sphere_convergence.py"))
conv = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(conv)


@pytest.fixture(scope="module")
def runs():
    return [conv.run(seed) for seed in conv.SEEDS]


def test_gbest_never_increases_and_falls(runs):
    for (seed, gap0, final, *_), trace in runs:
        assert np.all(np.diff(trace) <= 0), f"seed {seed}: gBest fitness increased"
        assert final < gap0 * 1e-3, f"seed {seed}: {gap0} -> {final}"


def test_final_gap_above_draw_floor(runs):
    for (seed, gap0, final, floor, expected, cmin, cmax), _ in runs:
        assert final >= floor, f"seed {seed}: final gap {final} below the draw floor {floor}"
        # Draw counts: 100 initial draws plus about 10 % of 100 x 1000 words.
        assert 9000 < cmin <= cmax < 11500


def test_floors_match_order_statistics(runs):
    floors = np.array([r[0][3] for r in runs])
    expected = np.array([r[0][4] for r in runs])
    # One floor is a sum of 30 squared minima (relative spread about 0.41);
    # the mean of 20 has a relative spread of about 0.09.
    ratio = floors.mean() / expected.mean()
    assert 0.6 < ratio < 1.4, ratio
    assert 5e-3 < expected.mean() < 7e-3


def test_record_reproduced(runs):
    rec = conv.read_record()
    assert [r[0] for r in rec] == list(conv.SEEDS)
    for got, (row, _) in zip(rec, runs):
        assert conv.format_row(row) == conv.format_row(got)
