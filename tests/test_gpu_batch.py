"""Batched swarms (sso_batch_*) against the CPU oracle, swarm by swarm.

Every swarm of a batch must evolve exactly as the oracle evolves it with the
swarm's own configuration; the bar is the one of tests/parity.py."""
import numpy as np
import pytest

import oracle
from paper_2110_01470_amd.inputs import BATCH_WORKLOADS, make_objective
from parity import REL_TOL, Pair, compare_after_run, oracle_run_with_trace

pytestmark = pytest.mark.gpu

# (n, d): one particle, tiny and ragged rows, tile and sub-slot boundaries,
# the largest d a batch takes.
SHAPES = [(1, 1), (3, 10), (37, 33), (100, 64), (129, 257), (64, 500), (300, 123), (17, 1000),
          (5, 4), (1000, 12)]


def make_swarms(kind="ripple", order=oracle.ORDER_GPS, storage="auto", shapes=SHAPES, lanes=None,
                seed=70):
    out = []
    for k, (n, d) in enumerate(shapes):
        rng = np.random.default_rng(seed + k)
        if order == oracle.ORDER_GPS:
            cg, cp, cw = rng.uniform(0.3, 0.5), rng.uniform(0.6, 0.75), rng.uniform(0.85, 0.95)
        else:
            cw, cp, cg = rng.uniform(0.3, 0.5), rng.uniform(0.6, 0.75), rng.uniform(0.85, 0.95)
        s, w, _ = make_objective(kind, d, seed + k, -50.0, 50.0)
        sw = dict(n=n, d=d, kind=kind, lo=-100.0, hi=100.0, cg=float(cg), cp=float(cp),
                  cw=float(cw), seed=1000 + seed + k, swarm_id=k, s=s, w=w, order=order,
                  storage=storage)
        if lanes is not None:
            sw["lanes"] = lanes[k]
        out.append(sw)
    return out


def pairs_for(batch, swarms):
    ps = []
    for k, sw in enumerate(swarms):
        ps.append(Pair(sw["kind"], sw["n"], sw["d"], lo=sw["lo"], hi=sw["hi"], cg=sw["cg"],
                       cp=sw["cp"], cw=sw["cw"], seed=sw["seed"], order=sw.get("order", 0),
                       swarm_id=sw["swarm_id"], objective=(sw["s"], sw["w"], None),
                       gpu=batch.view(k)))
    return ps


def step_all(batch, pairs, k=1):
    for _ in range(k):
        for pr in pairs:
            pr.prev_fp64 = pr.orc.fp64.copy()
            pr.orc.step()
        batch.step()
        for pr in pairs:
            pr.compare()


def run_all(batch, pairs, k):
    """k generations in one sso_batch_run call (graph blocks of 50 plus a
    remainder), checked at the end."""
    first = pairs[0].orc.t + 1
    traces = [oracle_run_with_trace(pr.orc, k) for pr in pairs]
    batch.run(k)
    return sum(compare_after_run(pr, first, tr) for pr, tr in zip(pairs, traces))


@pytest.mark.parametrize("kind,order,storage", [("ripple", oracle.ORDER_GPS, "auto"),
                                                ("ripple", oracle.ORDER_GPS, "f32"),
                                                ("sphere", oracle.ORDER_EQ21, "auto"),
                                                ("ripple", oracle.ORDER_EQ21, "u24")])
def test_batch_generations_match_oracle(kind, order, storage):
    from paper_2110_01470_amd.binding import Batch

    swarms = make_swarms(kind, order, storage)
    batch = Batch(swarms)
    pairs = pairs_for(batch, swarms)
    for pr in pairs:
        pr.compare()
    step_all(batch, pairs, 5)
    # 57 generations in one call: one replayed graph block and 7 launches.
    assert run_all(batch, pairs, 57) <= 1
    step_all(batch, pairs, 2)
    f, gi, im, t = batch.results()
    assert t == 64
    for k, pr in enumerate(pairs):
        assert gi[k] == pr.orc.gidx
        assert abs(f[k] - pr.orc.fp64[pr.orc.gidx]) <= REL_TOL * abs(pr.orc.fp64[pr.orc.gidx])
        assert im[k] == int(pr.orc.improved.sum())


def test_batch_graph_replays_back_to_back():
    """Several graph replays in a row, with host reads between calls."""
    from paper_2110_01470_amd.binding import Batch

    swarms = make_swarms(shapes=SHAPES[:6], seed=300)
    batch = Batch(swarms)
    pairs = pairs_for(batch, swarms)
    events = 0
    for k in (50, 100, 3, 150):
        events += run_all(batch, pairs, k)
    assert events <= 2
    assert batch.results()[3] == 303


@pytest.mark.parametrize("rule,waves", [(None, 4), (None, 8), (1, 4), (16, 8), ("tuned", None)])
def test_batch_swarm_equals_single_swarm_with_same_lanes(rule, waves):
    """A swarm of a batch is the one-swarm library's run of the same config
    when both use the same lanes per particle, whatever the batch's
    workgroup size: bit-identical states."""
    from paper_2110_01470_amd.binding import Batch, Swarm

    shapes = [(200, 300), (50, 37), (129, 64)]
    lanes = [8, 16, 32] if rule is None else [0, 0, 0]
    swarms = make_swarms(shapes=shapes, lanes=lanes, seed=500)
    batch = Batch(swarms)
    if rule == "tuned":
        batch.tune(1)  # any mapping; then fix the lanes the batch uses
    else:
        batch.set_mapping(8 if rule is None else rule, waves)
        assert batch.mapping()[:2] == (8 if rule is None else rule, waves)
    _, _, used, _ = batch.mapping()
    batch.run(60)
    checked = 0
    for k, sw in enumerate(swarms):
        if used[k] < 8:
            continue  # the one-swarm engine takes 8..64 lanes
        kw = {key: v for key, v in sw.items() if key in ("swarm_id", "order", "storage")}
        single = Swarm(sw["n"], sw["d"], sw["kind"], sw["lo"], sw["hi"], sw["cg"], sw["cp"],
                       sw["cw"], sw["seed"], sw["s"], sw["w"], lanes=int(used[k]),
                       engine="stream", **kw)
        single.run(60)
        a, b = single.state(), batch.view(k).state()
        for u, v in zip(a[:3], b[:3]):
            assert np.array_equal(u, v)
        checked += 1
    assert checked >= 1


def test_batch_tune_picks_a_rule_and_restarts():
    from paper_2110_01470_amd.binding import TUNE_CANDIDATES, TUNE_WAVES, Batch

    swarms = make_swarms(seed=900)
    batch = Batch(swarms)
    assert batch.mapping()[:2] == (8, 4)  # the untuned default
    cpl, waves, ms = batch.tune(3)
    assert cpl in TUNE_CANDIDATES and waves in TUNE_WAVES
    assert set(ms) == {(r, w) for r in TUNE_CANDIDATES for w in TUNE_WAVES}
    assert all(v > 0 for v in ms.values())
    rule, wv, lanes, tiles = batch.mapping()
    assert (rule, wv) == (cpl, waves)
    for k, sw in enumerate(swarms):
        chunks = (sw["d"] + 3) // 4
        L = 1
        while L * cpl < chunks and L < 32:
            L *= 2
        assert lanes[k] == L
    # Workgroups per launch: each swarm's particles in blocks of waves * 64 / L.
    assert tiles == sum(-(-sw["n"] // (waves * 64 // int(lanes[k]))) for k, sw in enumerate(swarms))
    # Back at generation 0 and in step with the oracle.
    pairs = pairs_for(batch, swarms)
    for pr in pairs:
        pr.compare()
    step_all(batch, pairs, 3)


def test_batch_set_state_and_errors():
    from paper_2110_01470_amd.binding import E_INVAL, E_STATE, Batch, SSOError

    swarms = make_swarms(shapes=[(20, 9), (7, 30)], seed=40)
    batch = Batch(swarms)
    pairs = pairs_for(batch, swarms)
    step_all(batch, pairs, 4)
    # A state carrying another generation count than the batch's is refused;
    # the oracle's state at the batch's count is taken.
    orc = pairs[1].orc
    with pytest.raises(SSOError) as e:
        batch.view(1).set_state(orc.x, orc.p, orc.fp, orc.t + 1)
    assert e.value.code == E_STATE
    batch.view(1).set_state(orc.x, orc.p, orc.fp, orc.t)
    step_all(batch, pairs, 3)
    with pytest.raises(SSOError) as e:
        batch.view(5).state()
    assert e.value.code == E_INVAL
    # A mapping is set only at generation 0, and only a known workgroup size.
    with pytest.raises(SSOError) as e:
        batch.set_mapping(8, 4)
    assert e.value.code == E_STATE
    fresh = Batch(swarms)
    for rule, waves in ((8, 5), (0, 4), (65, 8), (4, 16)):
        with pytest.raises(SSOError) as e:
            fresh.set_mapping(rule, waves)
        assert e.value.code == E_INVAL
    assert fresh.mapping()[:2] == (8, 4)


@pytest.mark.parametrize("storage", ["auto", "f32"])
def test_batch_largest_rows(storage):
    """d = 1024, the largest a batched swarm takes, beside ragged and tiny
    rows, under every mapping rule of the tuner."""
    from paper_2110_01470_amd.binding import TUNE_CANDIDATES, Batch

    shapes = [(2, 1024), (3, 1021), (70, 1024), (5, 2)]
    swarms = make_swarms(shapes=shapes, storage=storage, seed=800)
    batch = Batch(swarms)
    batch.tune(1)
    pairs = pairs_for(batch, swarms)
    for pr in pairs:
        pr.compare()
    step_all(batch, pairs, 3)
    assert len(TUNE_CANDIDATES) == 5


def test_batch512_full_size_sampled():
    """The 512-swarm ripple batch at full size, as the benchmark launches it:
    init and two generations; eight swarms compared in full, every swarm's
    gBest checked against its own pBest fitnesses."""
    from paper_2110_01470_amd.binding import Batch

    wl = BATCH_WORKLOADS["batch512_ripple"]
    swarms = wl.swarms()
    batch = Batch(swarms)
    sizes = np.array([sw["n"] * sw["d"] for sw in swarms])
    sample = sorted({0, 1, 511, int(np.argmax(sizes)), int(np.argmin(sizes)),
                     int(np.argmax([sw["d"] for sw in swarms])),
                     int(np.argmin([sw["n"] for sw in swarms])), 257})
    pairs = {k: pairs_for_one(batch, swarms, k) for k in sample}
    for pr in pairs.values():
        pr.compare()
    for _ in range(2):
        for pr in pairs.values():
            pr.prev_fp64 = pr.orc.fp64.copy()
            pr.orc.step()
        batch.step()
        for pr in pairs.values():
            pr.compare()
    f, gi, im, t = batch.results()
    assert t == 2
    for k in range(wl.count):
        _, _, fp, _ = batch.view(k).state(with_rows=False)
        assert gi[k] == int(np.argmin(fp))  # lowest index among equal minima
        assert f[k] == fp.min()


def pairs_for_one(batch, swarms, k):
    sw = swarms[k]
    return Pair(sw["kind"], sw["n"], sw["d"], lo=sw["lo"], hi=sw["hi"], cg=sw["cg"], cp=sw["cp"],
                cw=sw["cw"], seed=sw["seed"], swarm_id=sw["swarm_id"],
                objective=(sw["s"], sw["w"], None), gpu=batch.view(k))


def test_tune_after_generations_is_refused():
    from paper_2110_01470_amd.binding import E_STATE, Batch, SSOError

    swarms = make_swarms(shapes=[(20, 9), (7, 30)], seed=41)
    batch = Batch(swarms)
    batch.run(2)
    with pytest.raises(SSOError) as e:
        batch.tune(1)
    assert e.value.code == E_STATE
    assert batch.results()[3] == 2  # the batch is left as it was
