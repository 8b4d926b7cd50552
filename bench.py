"""Throughput of the SSO generation on one MI355X.

A step is one generation of Algorithm 2 over the whole swarm (Eq. 2.1 select,
fitness, pBest update, gBest argmin) -- one launch of the fused generation
kernel.  The default workload is the large ripple swarm (N=65536 particles,
D=1000 FP32 variables, 1000 generations).  Timing: W warm-up generations on
a throw-away swarm, then a fresh swarm is initialised (untimed, state already
resident in HBM).  When K is below the workload's T generations, that swarm
first runs generations 1..T-K untimed, and the last K generations T-K+1..T of
the run are timed, so the window is the run's steady state (in the first
generations most particles improve, and an improved particle's position row
is its pBest row, so it reads one row instead of two); otherwise generations
1..K are timed.  Timing uses HIP events on the stream the kernels run on.

Prints one JSON line:
  value    = N * D * K / seconds  (particle-variable updates per second,
             fitness included)
  roofline = 12 algorithmic bytes per update (read x, read p, write x')
             / mean generation time, against 8 TB/s HBM3E (dense objective:
             2 N D^2 FLOP per generation against 157.3 TFLOP/s FP32 matrix)
  cpu_baseline = the CPU oracle on a few generations of the same workload on
             this host, on all the host threads it may use (its loops over
             particles; same results), with the one-thread rate beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFLOPS = 157.3
BF16_MATRIX_PEAK_TFLOPS = 2500.0  # dense, no sparsity
BYTES_PER_UPDATE = 12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# Sources each workload's generation kernel is compiled from: a committed
# counter record is valid only while their hash is unchanged.
KERNEL_SOURCES = {
    "sphere": ("sso_device.hpp", "sso_layout.hpp", "resident.hip"),
    "ripple": ("sso_device.hpp", "sso_layout.hpp", "stream_body.hpp", "gen_stream.hip"),
    "dense": ("sso_device.hpp", "sso_layout.hpp", "gen_dense.hip"),
    "batch": ("sso_device.hpp", "sso_layout.hpp", "stream_body.hpp", "gen_batch.hip", "sso_batch.hip"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(kind):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2110_01470_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(wl, window=None, key=None):
    """HBM bytes per launch from the committed counter summary, or None if the
    kernel changed since the counters were taken or they cover another window
    of generations than the line times."""
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh)
    except (OSError, ValueError):
        return None
    key = key or wl.name
    rec = recs.get(key)
    if rec and window is not None and rec.get("timed_generations") != list(window):
        # A record of the same kernel over another window of the run.
        rec = recs.get(f"{key}@{window[0]}-{window[1]}")
    kind = "batch" if hasattr(wl, "count") else wl.kind
    if not rec or rec.get("kernel_hash") != kernel_hash(kind):
        return None
    if window is not None and rec.get("timed_generations") != list(window):
        return None
    return rec.get("bytes_per_launch")


def timed_window(wl, steps):
    """First and last generation of the timed window: the run's last `steps`
    generations when they are fewer than its T, else 1..steps."""
    first = wl.generations - steps + 1 if steps < wl.generations else 1
    return first, first + steps - 1


def time_gpu(wl, steps, warmup, engine, contraction="auto"):
    import torch

    from paper_2110_01470_amd.binding import Swarm

    s, w, a = wl.objective()
    stream = torch.cuda.Stream()
    args = (wl.n, wl.d, wl.kind, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w, a)
    if warmup:
        warm = Swarm(*args, engine=engine, contraction=contraction, stream=stream)
        warm.run(warmup)
        stream.synchronize()
        warm.close()
        del warm
    sw = Swarm(*args, engine=engine, contraction=contraction, stream=stream)
    first, _ = timed_window(wl, steps)
    if first > 1:
        sw.run(first - 1)  # untimed: generations 1..first-1 of the same run
    stream.synchronize()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sw.run(steps)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    g, fg, gidx, gen = sw.best()
    return ms, fg, gen, sw.mapping()


def time_gpu_batch(swarms, steps, tune_gens):
    import torch

    from paper_2110_01470_amd.binding import Batch

    stream = torch.cuda.Stream()
    batch = Batch(swarms, stream=stream)
    cpl, waves, tune_ms = batch.tune(tune_gens)
    log(f"mapping rule {cpl} chunks per lane, {waves} waves per workgroup; tuner ms per "
        f"{tune_gens} generations: {tune_ms}")
    stream.synchronize()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    batch.run(steps)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    f, gi, im, gen = batch.results()
    _, _, lanes, tiles = batch.mapping()
    return ms, f, gen, (cpl, waves), tiles, lanes


def time_gpu_separate(swarms, steps, lanes):
    """Plain SSO for the batch's swarms: one one-swarm context per swarm, each
    run for `steps` generations in turn on one stream (the way the swarms
    would run without batching).  A swarm whose batch lanes the one-swarm
    engine takes (8 or more) is given those lanes, so its run is
    bit-identical to its run in the batch; the others take the engine's own
    choice.  Returns the milliseconds, each swarm's final gBest fitness, and
    which swarms had the batch's lanes."""
    import torch

    from paper_2110_01470_amd.binding import Swarm

    stream = torch.cuda.Stream()
    sws, same = [], []
    for k, sw in enumerate(swarms):
        ln = int(lanes[k]) if lanes[k] >= 8 else 0
        same.append(ln != 0)
        sws.append(Swarm(sw["n"], sw["d"], sw["kind"], sw["lo"], sw["hi"], sw["cg"], sw["cp"],
                         sw["cw"], sw["seed"], sw["s"], sw["w"], swarm_id=sw["swarm_id"],
                         order=sw.get("order", 0), storage=sw.get("storage", "auto"), lanes=ln,
                         engine="stream", stream=stream))
    stream.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for s in sws:
        s.run(steps)
    stop.record(stream)
    stop.synchronize()
    ms = start.elapsed_time(stop)
    f = np.array([s.best()[1] for s in sws], dtype=np.float32)
    for s in sws:
        s.close()
    return ms, f, np.array(same)


def host_threads():
    """Threads for the oracle's all-cores timing: OMP_NUM_THREADS where it is
    set (the host's CPU share), else the CPUs this process may run on."""
    n = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    return max(1, n)


def time_oracle_batch(swarms, gens, threads=1):
    import oracle

    used = oracle.set_threads(threads)
    try:
        updates, sec = _time_oracle_batch(swarms, gens)
    finally:
        oracle.set_threads(1)
    return updates, sec, used


def _time_oracle_batch(swarms, gens):
    import oracle

    sec = 0.0
    updates = 0
    for sw in swarms:
        kind = {"sphere": oracle.SPHERE, "ripple": oracle.RIPPLE}[sw["kind"]]
        orc = oracle.Swarm(sw["n"], sw["d"], kind, sw["lo"], sw["hi"], sw["cg"], sw["cp"], sw["cw"],
                           sw["seed"], sw["s"], sw["w"], None, swarm=sw["swarm_id"])
        orc.init()
        t0 = time.perf_counter()
        orc.run(gens)
        sec += time.perf_counter() - t0
        updates += sw["n"] * sw["d"] * gens
    return updates, sec


def ceilings(reps=20):
    """The two ceilings of the generation kernels, measured on this GPU: a
    plain device-to-device copy (HBM read + write bandwidth) and the rate of
    the library's Philox kernel, which draws every word of one generation of
    the ripple swarm's shape (4 words per Philox4x32-10 block) and writes each
    word to HBM (4 B per word)."""
    import torch

    from paper_2110_01470_amd.binding import Swarm
    from paper_2110_01470_amd.inputs import WORKLOADS

    stream = torch.cuda.Stream()
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
    e1.synchronize()
    copy_s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst

    wl = WORKLOADS["ripple_n65536_d1000"]
    s, w, a = wl.objective()
    sw = Swarm(wl.n, wl.d, wl.kind, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w, a,
               stream=stream)
    out = torch.empty(wl.n * wl.d, dtype=torch.int32, device="cuda")
    sw.rng_words_into(1, out, 3)
    e0.record(stream)
    sw.rng_words_into(1, out, reps)
    e1.record(stream)
    e1.synchronize()
    rng_s = e0.elapsed_time(e1) / 1e3 / reps
    words = wl.n * wl.d
    print(json.dumps({
        "ceilings": {
            "copy": {"bytes": nbytes, "us_per_copy": copy_s * 1e6,
                     "GBps_read_plus_write": 2 * nbytes / copy_s / 1e9,
                     "frac_of_peak": 2 * nbytes / copy_s / 1e9 / HBM_PEAK_GBS},
            "philox": {"words_per_launch": words, "us_per_launch": rng_s * 1e6,
                       "words_per_s": words / rng_s,
                       "write_GBps": 4 * words / rng_s / 1e9,
                       "note": f"one generation's words of {wl.name}, each written to HBM"},
        }}), flush=True)


def time_oracle(wl, gens, threads=1):
    """Seconds for `gens` oracle generations after initialisation, and the
    thread count the oracle used."""
    import oracle

    kind = {"sphere": oracle.SPHERE, "ripple": oracle.RIPPLE, "dense": oracle.DENSE}[wl.kind]
    s, w, a = wl.objective()
    used = oracle.set_threads(threads)
    try:
        orc = oracle.Swarm(wl.n, wl.d, kind, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w, a)
        orc.init()
        t0 = time.perf_counter()
        orc.run(gens)
        sec = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    return sec, used


def copy_calibration(nbytes, reps=5):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes": nbytes, "reps": reps, "seconds_per_copy": sec,
                      "GBps_read_plus_write": 2 * nbytes / sec / 1e9}), flush=True)


def profile_window(path, kernel_regex, last):
    """Summary of the last `last` dispatches of the kernels whose name matches
    `kernel_regex` in a rocprofv3 CSV: a kernel trace (durations, ns) or a
    counter collection (each counter's per-dispatch value).  This is how the
    committed profile summaries relate a whole profiled bench run to the
    generations its line times (the run's last K)."""
    import csv
    import re

    pat = re.compile(kernel_regex)
    with open(path, newline="") as fh:
        rows = [r for r in csv.DictReader(fh) if pat.search(r.get("Kernel_Name", ""))]
    out = {"file": os.path.basename(path), "kernel_regex": kernel_regex, "last": last}
    if rows and "Counter_Name" in rows[0]:
        by = {}
        for r in rows:
            by.setdefault(r["Counter_Name"], []).append(
                (int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0), float(r["Counter_Value"])))
        for name, vals in sorted(by.items()):
            vals.sort()
            v = np.array([x for _, x in vals[-last:]])
            out[name] = {"dispatches": len(vals), "window_mean": float(v.mean()),
                         "window_min": float(v.min()), "window_max": float(v.max()),
                         "all_mean": float(np.mean([x for _, x in vals]))}
    else:
        ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                    for r in rows)
        dur = np.array([d for _, d in ev], dtype=np.float64)
        w = dur[-last:]
        out.update({"dispatches": int(dur.size), "window_mean_ns": float(w.mean()),
                    "window_min_ns": float(w.min()), "window_max_ns": float(w.max()),
                    "all_mean_ns": float(dur.mean())})
    print(json.dumps(out), flush=True)


def main():
    from paper_2110_01470_amd.inputs import BATCH_WORKLOADS, PAPER_WORKLOADS, WORKLOADS

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed generations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ripple_n65536_d1000",
                    choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS) + sorted(PAPER_WORKLOADS))
    ap.add_argument("--paper-quality", action="store_true",
                    help="final gBest of f1..f9 at the paper's settings over seeds 1001..1020")
    ap.add_argument("--polish", action="store_true",
                    help="dense workload: time-to-gap of plain SSO vs SSO with a gradient "
                         "polish of all pBests every 50 generations")
    ap.add_argument("--separate", action="store_true",
                    help="batch workload: also run every swarm alone (plain SSO, one context "
                         "per swarm) for the same generations and compare")
    ap.add_argument("--tune-gens", type=int, default=5,
                    help="generations the batch mapping tuner times per candidate")
    ap.add_argument("--engine", default="auto", choices=["auto", "stream", "resident"])
    ap.add_argument("--contraction", default="auto", choices=["auto", "f32", "bf16x3", "f16x2"],
                    help="dense objective: FP32, split-bf16 or split-fp16 matrix cores")
    ap.add_argument("--cpu-gens", type=int, default=None,
                    help="oracle generations for cpu_baseline (0 = skip)")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure the copy-bandwidth and Philox-rate ceilings")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--profile-window", metavar="CSV",
                    help="only summarise the last --window dispatches of --kernel-regex in a "
                         "rocprofv3 kernel-trace or counter CSV (no GPU)")
    ap.add_argument("--kernel-regex", default=r"sso::k_")
    ap.add_argument("--window", type=int, default=20)
    args = ap.parse_args()

    if args.profile_window:
        profile_window(args.profile_window, args.kernel_regex, args.window)
        return
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.ceilings:
        ceilings()
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the benchmark measures one GPU's swarm; sharding over GPUs is not built)",
              file=sys.stderr)
        sys.exit(2)

    if args.paper_quality:
        paper_quality(PAPER_WORKLOADS, args)
        return
    if args.workload in BATCH_WORKLOADS:
        bench_batch(BATCH_WORKLOADS[args.workload], args)
        return
    if args.workload in PAPER_WORKLOADS:
        bench_paper(PAPER_WORKLOADS[args.workload], args)
        return

    wl = WORKLOADS[args.workload]
    if args.polish:
        bench_polish(wl, args)
        return
    steps = args.steps if args.steps is not None else wl.generations
    window = timed_window(wl, steps)
    log(f"workload {wl.name}: N={wl.n} D={wl.d} steps={steps} warmup={args.warmup}, "
        f"timed generations {window[0]}..{window[1]}")
    ms, fg, gen, (engine, storage, lanes, contraction) = time_gpu(wl, steps, args.warmup,
                                                                   args.engine, args.contraction)
    sec = ms / 1e3
    updates = wl.n * wl.d * steps
    value = updates / sec
    ms_per_step = ms / steps
    log(f"gpu: {ms:.3f} ms for {steps} generations, fG={fg:.6g} at t={gen}")

    split = wl.kind == "dense" and contraction != "f32"
    f32_line = None
    if split:
        # The FP32 contraction the workload names, timed over the same window
        # beside the default split one.
        ms32, _, _, _ = time_gpu(wl, steps, args.warmup, args.engine, "f32")
        t32 = 2.0 * wl.n * wl.d * wl.d / (ms32 / steps / 1e3) / 1e12
        f32_line = {"ms_per_step": ms32 / steps, "value": wl.n * wl.d * steps / (ms32 / 1e3),
                    "achieved_tflops": t32, "frac_of_fp32_matrix_peak": t32 / FP32_MATRIX_PEAK_TFLOPS,
                    "traffic": measured_traffic(wl, window, wl.name + "/f32")}
        log(f"gpu, FP32 contraction: {ms32:.3f} ms for {steps} generations")
    if wl.kind == "dense":
        # Two roofs: the contraction's FLOP against its matrix peak, and the
        # 12 B per update of rows against HBM.  A split contraction runs six
        # bf16 (BF16X3) or three fp16 (F16X2) products per FP32 product on the
        # 16-bit matrix cores (the same dense peak for both types), priced at
        # that work; the FP32-equivalent rate against the FP32 matrix peak is
        # given beside it.  The line's bound is the roof whose ideal time is
        # the longer one; the other roof rides along in "other_roof".
        products = (3 if contraction == "f16x2" else 6) if split else 1
        peak = BF16_MATRIX_PEAK_TFLOPS if split else FP32_MATRIX_PEAK_TFLOPS
        flop = products * 2.0 * wl.n * wl.d * wl.d
        tflops = flop / (ms_per_step / 1e3) / 1e12
        mfma_roof = {"bound": "mfma", "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": tflops / peak}
        byt = BYTES_PER_UPDATE * wl.n * wl.d
        gbs = byt / (ms_per_step / 1e3) / 1e9
        hbm_roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS}
        hbm_binds = byt / (HBM_PEAK_GBS * 1e9) >= flop / (peak * 1e12)
        roofline, other = (hbm_roof, mfma_roof) if hbm_binds else (mfma_roof, hbm_roof)
        roofline = dict(roofline)
        roofline["traffic"] = measured_traffic(wl, window, wl.name + "/" + contraction)
        if split:
            roofline["fp32_equivalent_frac"] = tflops / products / FP32_MATRIX_PEAK_TFLOPS
        roofline["other_roof"] = other
    else:
        byt = BYTES_PER_UPDATE * wl.n * wl.d
        achieved = byt / (ms_per_step / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(wl, window)}
        if engine == "resident":
            roofline["note"] = ("algorithmic rate only: the resident engine keeps the swarm in "
                                "one workgroup's registers and touches HBM only at the start "
                                "and end of the run; a generation is bound by that "
                                "workgroup's dependent chain, not by HBM")

    cpu_gens = args.cpu_gens
    if cpu_gens is None:
        # About 10-30 s of single-threaded oracle work.
        cpu_gens = max(1, min(steps, int(4 * 65536 * 1000 // (wl.n * wl.d)) or 1))
        if wl.kind == "dense":
            cpu_gens = max(1, min(steps, 4 * 16384 * 256 // (wl.n * wl.d)))
    cpu = None
    if cpu_gens > 0:
        csec1, _ = time_oracle(wl, cpu_gens)
        log(f"cpu oracle, one thread: {csec1:.2f} s for {cpu_gens} generations")
        nth = host_threads()
        gens_n = min(steps, max(cpu_gens, cpu_gens * nth // 2))
        csec, used = time_oracle(wl, gens_n, nth)
        log(f"cpu oracle, {used} threads: {csec:.2f} s for {gens_n} generations")
        upd = wl.n * wl.d
        cpu = {"value": upd * gens_n / csec, "unit": "particle-var updates/s",
               "cores": used, "kind": "oracle",
               "sample": f"{gens_n} generations of {wl.name} after initialisation, FP64 oracle "
                         f"on {used} threads ({csec:.2f} s); one thread: {cpu_gens} "
                         f"generations ({csec1:.2f} s)",
               "single_thread": {"value": upd * cpu_gens / csec1, "cores": 1}}

    rec = {
        "metric": "particle-var updates/s incl. fitness",
        "value": value,
        "unit": "particle-var updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": contraction if split else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "objective": wl.kind, "n": wl.n, "d": wl.d,
                   "generations": max(steps, wl.generations),
                   "timed_generations": list(window), "engine": engine,
                   **({"contraction": contraction}
                      if wl.kind == "dense" else {"row_storage": storage,
                                                  "lanes_per_particle": lanes})},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if f32_line is not None:
        rec["f32_contraction"] = f32_line
    print(json.dumps(rec), flush=True)


# The paper's PSSO wall times (GTX 1080) for its Rosenbrock runs, Table 3.10:
# P = 50, 1000 iterations, (Cw, Cp, Cg) = (0.3, 0.6, 0.8).
PAPER_F4_SECONDS = {100: 0.13875, 200: 0.154, 300: 0.1638, 350: 0.1695}
# The paper's PSSO solution quality at D = 50, N = 100, T = 1000 over 20 runs
# (average, standard deviation, minimum), for the functions it lists legibly.
PAPER_QUALITY = {"f1": (41.0156, 5.3095, 28.5125), "f4": (1103.9103, 134.5448, 730.0332),
                 "f5": (220.6183, 16.2710, 189.2935)}


def paper_swarm(pw, seed=None, stream=None, engine="auto"):
    from paper_2110_01470_amd.binding import Swarm

    return Swarm(pw.n, pw.d, pw.kind, pw.lo, pw.hi, pw.cg, pw.cp, pw.cw,
                 pw.seed if seed is None else seed, None, order=1, engine=engine,
                 stream=stream)


def bench_paper(pw, args):
    """A Table 3.2 function at the paper's settings.  The paper times whole
    runs (set-up, T iterations, result back on the host), so the line's value
    is that wall time, measured on the host clock: swarm creation (upload and
    initialisation), the T generations, and the gBest copy back."""
    import torch

    from paper_2110_01470_amd.binding import Swarm  # noqa: F401  (loads the library)

    steps = args.steps if args.steps is not None else pw.generations
    stream = torch.cuda.Stream()
    for _ in range(max(1, args.warmup // 10)):  # warm-up whole runs
        sw = paper_swarm(pw, stream=stream, engine=args.engine)
        sw.run(steps)
        sw.best()
        sw.close()
    walls = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw = paper_swarm(pw, stream=stream, engine=args.engine)
        sw.run(steps)
        g, fg, gidx, gen = sw.best()
        walls.append(time.perf_counter() - t0)
        sw.close()
    wall = float(np.median(walls))
    # The generations alone, with HIP events.
    sw = paper_swarm(pw, stream=stream, engine=args.engine)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sw.run(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    engine, storage, lanes, _ = sw.mapping()
    ms_per_step = ms / steps
    updates = pw.n * pw.d * steps
    log(f"{pw.name}: whole run {wall * 1e3:.2f} ms (median of 5), generations {ms:.2f} ms, "
        f"final fG {fg:.6g}")
    byt = BYTES_PER_UPDATE * pw.n * pw.d
    achieved = byt / (ms_per_step / 1e3) / 1e9
    paper_s = PAPER_F4_SECONDS.get(pw.n) if pw.kind == "f4" and pw.d == 50 else None
    cpu = None
    if args.cpu_gens is None or args.cpu_gens > 0:
        import oracle

        def whole_run(threads):
            used = oracle.set_threads(threads)
            try:
                orc = oracle.Swarm(pw.n, pw.d, oracle.F1 + int(pw.kind[1:]) - 1, pw.lo, pw.hi,
                                   pw.cg, pw.cp, pw.cw, pw.seed, None, order=oracle.ORDER_EQ21)
                t0 = time.perf_counter()
                orc.init()
                orc.run(steps)
                return time.perf_counter() - t0, used
            finally:
                oracle.set_threads(1)

        csec1, _ = whole_run(1)
        csec, used = whole_run(host_threads())
        cpu = {"value": csec, "unit": "s", "cores": used, "kind": "oracle",
               "sample": f"the whole {steps}-generation run of {pw.name}, FP64 oracle on {used} "
                         f"threads; one thread: {csec1:.4f} s",
               "single_thread": {"value": csec1, "cores": 1}}
    rec = {
        "metric": "wall time of a whole run (set-up, T generations, gBest to host)",
        "value": wall,
        "unit": "s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(1, args.warmup // 10),
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": wall / paper_s if paper_s else None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": pw.name, "objective": pw.kind, "n": pw.n, "d": pw.d,
                   "generations": steps, "box": [pw.lo, pw.hi], "order": "eq21", "engine": engine,
                   "row_storage": storage, "lanes_per_particle": lanes,
                   "cw_cp_cg": [pw.cw, pw.cp, pw.cg]},
        "updates_per_s": updates / (ms / 1e3),
        "final_fG": fg,
        "paper_context": ({"seconds": paper_s, "hardware": "GTX 1080", "source": "Table 3.10"}
                          if paper_s else None),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "note": "algorithmic rate only: a swarm this small is bound by each "
                             "generation's dependent chain (one workgroup's ALU work with the "
                             "resident engine, launch and memory latency with the stream one), "
                             "not by HBM"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def paper_quality(workloads, args):
    """Final gBest fitness of each Table 3.2 function at the paper's settings
    (D = 50, N = 100, T = 1000, (Cw, Cp, Cg) = (0.3, 0.6, 0.8)) over the 20
    replicate seeds, beside the paper's own PSSO figures where legible."""
    import torch

    stream = torch.cuda.Stream()
    out = {}
    for k in range(1, 10):
        pw = workloads[f"paper_f{k}_n100_d50"]
        finals = []
        for seed in range(1001, 1021):
            sw = paper_swarm(pw, seed=seed, stream=stream, engine=args.engine)
            sw.run(pw.generations)
            finals.append(sw.best()[1])
            sw.close()
        v = np.array(finals, np.float64)
        out[pw.kind] = {"mean": float(v.mean()), "std": float(v.std(ddof=1)), "min": float(v.min()),
                        "paper": PAPER_QUALITY.get(pw.kind)}
        log(f"{pw.kind}: {v.mean():.4f} +- {v.std(ddof=1):.4f} (min {v.min():.4f})")
    print(json.dumps({"paper_quality": out, "runs": 20, "d": 50, "n": 100, "generations": 1000}),
          flush=True)


POLISH_EVERY, POLISH_STEPS = 50, 5


def time_to_gap(fg, gen_ms, polish_ms, every, gap):
    """Milliseconds until the gBest gap fG - f* (f* = 0) first reaches `gap`:
    generations at gen_ms each plus the polishes done by then; None if never."""
    hit = np.nonzero(fg <= gap)[0]
    if hit.size == 0:
        return None
    t = int(hit[0])
    return t * gen_ms + ((t // every) * polish_ms if every else 0.0)


def bench_polish(wl, args):
    """Plain SSO against SSO with a 5-step projected-gradient polish of all
    pBests every 50 generations (step 0.05 / sigma_max(A)^2) on the dense
    workload: both runs timed with HIP events, the polish kernel timed on its
    own for its MFMA rate, and the time each run needs to reach a gap."""
    import torch

    from paper_2110_01470_amd.binding import Swarm

    steps = args.steps if args.steps is not None else wl.generations
    s, w, a = wl.objective()
    stream = torch.cuda.Stream()
    args_ = (wl.n, wl.d, wl.kind, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw, wl.seed, s, w, a)
    runs = {}
    for name, kw in (("plain", {}), ("polished", dict(polish_every=POLISH_EVERY,
                                                       polish_steps=POLISH_STEPS))):
        sw = Swarm(*args_, stream=stream, trace_cap=steps + 8, contraction=args.contraction, **kw)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sw.run(steps)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        fg, _, _ = sw.trace(0, steps + 1)
        runs[name] = {"ms": ms, "fg": fg.astype(np.float64)}
        log(f"{name}: {ms:.1f} ms for {steps} generations, final fG {fg[-1]:.6g}")
        sw.close()
    # The polish kernel alone: (4 steps + 2) N D^2 FLOP per call.
    sw = Swarm(*args_, stream=stream, contraction=args.contraction)
    contraction = sw.mapping()[3]
    sw.run(10)
    lr = sw.polish(POLISH_STEPS)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # The stream is busy with one more polish when the timed region opens, so
    # it holds no host launch latency.
    sw.polish(POLISH_STEPS, lr)
    e0.record(stream)
    for _ in range(reps):
        sw.polish(POLISH_STEPS, lr)
    e1.record(stream)
    e1.synchronize()
    polish_ms = e0.elapsed_time(e1) / reps
    flop = (4 * POLISH_STEPS + 2) * wl.n * wl.d * wl.d
    tflops = flop / (polish_ms / 1e3) / 1e12
    log(f"polish: {polish_ms * 1e3:.1f} us per call, {tflops:.1f} TFLOP/s")

    plain_gen_ms = runs["plain"]["ms"] / steps
    pol_gen_ms = (runs["polished"]["ms"] - (steps // POLISH_EVERY) * polish_ms) / steps
    gap_target = 1e-6
    final = {k: float(v["fg"][-1]) for k, v in runs.items()}
    if all(final[k] <= gap_target for k in final):
        gap = gap_target
    else:
        gap = max(final.values())  # the best gap both runs reach
    ttg = {"plain": time_to_gap(runs["plain"]["fg"], plain_gen_ms, 0.0, 0, gap),
           "polished": time_to_gap(runs["polished"]["fg"], pol_gen_ms, polish_ms, POLISH_EVERY, gap)}
    reached = {k: time_to_gap(v["fg"], plain_gen_ms if k == "plain" else pol_gen_ms,
                              0.0 if k == "plain" else polish_ms, 0 if k == "plain" else POLISH_EVERY,
                              gap_target) for k, v in runs.items()}
    rec = {
        "metric": "time-to-gap vs plain SSO (dense objective, gradient polish every 50 generations)",
        "value": ttg["polished"] / 1e3 if ttg["polished"] is not None else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": runs["polished"]["ms"] / steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": contraction,
        "data": "synthetic",
        "config": {"workload": wl.name + "+polish", "objective": wl.kind, "n": wl.n, "d": wl.d,
                   "generations": steps, "polish_every": POLISH_EVERY, "polish_steps": POLISH_STEPS,
                   "polish_lr": lr,
                   "contraction": contraction,
                   "polish_contraction": "f32"},
        "gap": {"target": gap_target, "compared_at": gap,
                "time_to_target_ms": reached,
                "time_to_compared_gap_ms": ttg,
                "final_gap": final,
                "speedup_vs_plain": (ttg["plain"] / ttg["polished"]
                                     if ttg["plain"] and ttg["polished"] else None),
                "ms_total": {k: v["ms"] for k, v in runs.items()}},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MATRIX_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP32_MATRIX_PEAK_TFLOPS,
                     "traffic": None, "kernel": "polish (FP32 MFMA), timed alone"},
        "polish_rate": {"value": wl.n / (polish_ms / 1e3), "unit": "pBests polished/s"},
        "cpu_baseline": cpu_polish_baseline(wl, lr) if args.cpu_gens != 0 else None,
    }
    print(json.dumps(rec), flush=True)


def cpu_polish_baseline(wl, lr, sample=1024):
    """The oracle's polish of `sample` pBests of the same instance."""
    import oracle

    s, w, a = wl.objective()

    def timed(threads, count):
        used = oracle.set_threads(threads)
        try:
            orc = oracle.Swarm(count, wl.d, oracle.DENSE, wl.lo, wl.hi, wl.cg, wl.cp, wl.cw,
                               wl.seed, s, None, a)
            orc.init()
            t0 = time.perf_counter()
            orc.polish(POLISH_STEPS, lr)
            return time.perf_counter() - t0, used
        finally:
            oracle.set_threads(1)

    sec1, _ = timed(1, sample)
    nth = host_threads()
    many = sample * max(1, nth // 2)
    sec, used = timed(nth, many)
    return {"value": many / sec, "unit": "pBests polished/s", "cores": used, "kind": "oracle",
            "sample": f"{POLISH_STEPS}-step polish of {many} pBests of {wl.name}, FP64 oracle on "
                      f"{used} threads ({sec:.2f} s); one thread: {sample} pBests ({sec1:.2f} s)",
            "single_thread": {"value": sample / sec1, "cores": 1}}


def bench_batch(bw, args):
    """The batched workload: every swarm advances `steps` generations; a step
    is one generation of all swarms (one launch, replayed from graphs)."""
    from paper_2110_01470_amd.binding import TUNE_CANDIDATES, TUNE_WAVES

    steps = args.steps if args.steps is not None else bw.generations
    swarms = bw.swarms()
    total = sum(sw["n"] * sw["d"] for sw in swarms)
    log(f"workload {bw.name}: {bw.count} swarms, {total} variables, steps={steps}")
    ms, fb, gen, (cpl, waves), tiles, lanes = time_gpu_batch(swarms, steps, args.tune_gens)
    sec = ms / 1e3
    ms_per_step = ms / steps
    log(f"gpu: {ms:.3f} ms for {steps} generations, best fG over swarms={float(fb.min()):.6g} "
        f"at t={gen}")
    separate = None
    if args.separate:
        ms_sep, fs, same = time_gpu_separate(swarms, steps, lanes)
        log(f"separate swarms: {ms_sep:.3f} ms for {steps} generations")
        rel = np.abs(fs.astype(np.float64) - fb) / np.maximum(np.abs(fb.astype(np.float64)), 1e-30)
        separate = {"ms_per_step": ms_sep / steps, "speedup_of_batch": ms_sep / ms,
                    "swarms_with_batch_lanes": int(same.sum()),
                    "equal_final_fG_with_batch_lanes": int(np.sum(fs[same] == fb[same])),
                    "max_rel_final_fG_diff_other": float(rel[~same].max()) if (~same).any() else 0.0,
                    "note": "each swarm run alone with the one-swarm library, "
                            "the swarms one after another on one stream"}
    byt = BYTES_PER_UPDATE * total
    achieved = byt / (ms_per_step / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(bw, (1, steps))}
    cpu = None
    if args.cpu_gens is None or args.cpu_gens > 0:
        gens = args.cpu_gens or 1
        updates1, csec1, _ = time_oracle_batch(swarms, gens)
        log(f"cpu oracle, one thread: {csec1:.2f} s for {updates1} updates")
        nth = host_threads()
        gens_n = max(gens, gens * nth // 8)
        updates, csec, used = time_oracle_batch(swarms, gens_n, nth)
        log(f"cpu oracle, {used} threads: {csec:.2f} s for {updates} updates")
        cpu = {"value": updates / csec, "unit": "particle-var updates/s", "cores": used,
               "kind": "oracle",
               "sample": f"{gens_n} generation(s) of each of the {bw.count} swarms of {bw.name} "
                         f"after initialisation, FP64 oracle on {used} threads ({csec:.2f} s); "
                         f"one thread: {gens} generation(s) ({csec1:.2f} s)",
               "single_thread": {"value": updates1 / csec1, "cores": 1}}
    rec = {
        "metric": "particle-var updates/s incl. fitness",
        "value": total * steps / sec,
        "unit": "particle-var updates/s",
        "n_gpus": 1,
        "steps": steps,
        # the tuner's timed generations
        "warmup": len(TUNE_CANDIDATES) * len(TUNE_WAVES) * args.tune_gens,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": bw.name, "objective": bw.kind, "swarms": bw.count,
                   "variables": total, "generations": steps, "mapping_rule": cpl,
                   "waves_per_workgroup": waves, "workgroups_per_launch": tiles,
                   "graph_block": 50},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if separate is not None:
        rec["separate_swarms"] = separate
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
