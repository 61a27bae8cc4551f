#!/usr/bin/env python3
"""Benchmark of the 2D PIC space-charge step on one MI355X.

A step is one pass of the whole hot path over the beam: kick with the field
of the previous space-charge location, push through the ring elements up to
the next one, deposit the charge, solve the open-boundary Poisson equation
and form the field.  The default workload is the production shape: 1e6
Gaussian particles, a 128 x 128 grid over +-6 sigma, one turn = 100
block-diagonal 4x4 transfer maps, 10 thin sextupoles and 100 space-charge
steps, all in FP64.  Inputs are seeded synthetic data resident in HBM before
the timed region starts.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(the fused particle pass, timed live with HIP events on the library's stream)
and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

K and W are lower bounds in space-charge steps: both are rounded up to whole
turns (a track call runs whole turns), the timed region to at least ten turns
of the production ring so that replays of the captured turn graph dominate it;
the line reports the steps actually timed and the ones requested.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = ("particle-steps/sec (push+deposit+solve+kick), 1e6 particles, 128\u00b2 grid; "
          "% HBM peak")
HBM_PEAK_GBS = 8000.0
BYTES_PER_PARTICLE_STEP = 64  # read + write x, px, y, py in FP64
BYTES_PER_WEIGHT = 4          # + the FP32 line-density kick weight (2.5D long bunch)
BYTES_PER_LONGITUDINAL = 24   # + read sigma, p_sigma and write sigma (thick elements, 6D)
FP64_PEAK_TFLOPS = 78.6       # MI355X vector FP64
# FP64 operations per particle (a fused multiply-add counts 2, sqrt and
# division 1) of the pass's arithmetic: gather + kick and the deposit's cell
# and weights, plus each element of the pass
FLOPS_KICK, FLOPS_DEPOSIT, FLOPS_CHROMA = 35, 14, 3
# the line density: line weights at the kick and the deposit, the two table
# gathers, the potential gather and the longitudinal kick
FLOPS_LINE = 32
BYTES_LINE_KICK = 8           # + write p_sigma (the longitudinal kick)



def stream_time_us(stream, fn, reps: int) -> float:
    """Average GPU time per call of fn (which enqueues work on `stream`) over
    reps calls timed with HIP events.  A bounded sleep kernel ahead of the
    first event keeps the GPU busy while the host enqueues every call, so the
    host's cost per call leaves no gaps between the kernels; the sleep is
    lengthened (at most three times) until it outlasts the enqueueing."""
    import torch

    for _ in range(3):
        fn()
    cycles = int(reps * 60e-6 * 2.0e9)
    for _ in range(4):
        torch.cuda.synchronize()
        ready = torch.cuda.Event()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            torch.cuda._sleep(cycles)
        ready.record(stream)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        covered = not ready.query()
        torch.cuda.synchronize()
        if covered:
            break
        cycles *= 4
    return t0.elapsed_time(t1) * 1e3 / reps

def element_flops(e, inputs) -> int:
    k, m = int(e["kind"]), e["p"]
    if k == inputs.LIN2X2:
        return 12
    if k == inputs.LIN4X4:
        return 28
    if k == inputs.SEXT_THIN:
        return 8
    if k == inputs.QUAD_THICK:
        return 105 if m[0] != 0.0 else 16
    if k == inputs.SEXT_THICK:
        return 15 if m[0] == 0.0 else 6 + 60 * int(m[3])
    return 0
PROFILE_TRAFFIC = ROOT / "profiles" / "pass_traffic_production.json"
PASS_SOURCE = ROOT / "paper_2010_11540_amd" / "csrc" / "particles.hip"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed SC steps, at least; rounded up to whole turns and to the "
                         "workload's minimum (default: 20 turns of production, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed SC steps before timing, at least; rounded up to whole turns, "
                         "two at the least (default: 2 turns)")
    ap.add_argument("--workload", default="production",
                    choices=["production", "small", "large", "batch", "thick", "line"],
                    help="production (the metric): 1e6 Gaussian, 128^2; large: 1e7 KV long "
                         "bunch with line-density kick weights, 256^2; batch: 64-beam tune scan")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--gather", default="cic", choices=["cic", "bspline"],
                    help="kick field: cloud-in-cell gather of the node field, or the gradient of "
                         "the bicubic B-spline surface of the node potential")
    ap.add_argument("--solver", default="open", choices=["open", "pipe"],
                    help="open-boundary convolution, or the grounded rectangular pipe")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels directly, no HIP graph")
    ap.add_argument("--pass-threads", type=int, default=0)
    ap.add_argument("--pass-blocks", type=int, default=0)
    ap.add_argument("--pass-reps", type=int, default=200, help="standalone pass launches timed")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="wall-clock budget of each CPU oracle sample (all host threads, then one)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 64 MiB device-to-device copy 20 times (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="only time plain device streams (copies of 320 MiB and 1 GiB, and an "
                         "in-place scale of four 256 MiB arrays): the read+write bandwidth HBM "
                         "delivers in practice, beside the 8 TB/s peak")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024 // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 8, "bytes_written": n * 8,
                                           "launches": 20}}), flush=True)


def stream_ceiling():
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    for mib in (320, 1024):
        n = mib * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        us = stream_time_us(stream, lambda: dst.copy_(src), 50)
        out[f"copy_{mib}MiB"] = {"us": round(us, 2), "GBps": round(2 * n * 8 / (us * 1e-6) / 1e9, 1)}
        del src, dst
    n = 256 * (1 << 20) // 8
    xs = [torch.rand(n, dtype=torch.float64, device="cuda") for _ in range(4)]

    def scale_all():
        for x in xs:
            x.mul_(1.0)

    us = stream_time_us(stream, scale_all, 20)
    out["scale_4x256MiB"] = {"us": round(us, 2), "GBps": round(8 * n * 8 / (us * 1e-6) / 1e9, 1)}
    print(json.dumps({"stream_ceiling": out, "peak_GBps": HBM_PEAK_GBS}), flush=True)


def code_digest(text: str) -> str:
    """Digest of a source's code: // comments, line continuations and all
    whitespace left out, so that editing a comment or re-wrapping a line does
    not mark a measurement stale."""
    lines = (l.split("//")[0].rstrip().rstrip("\\") for l in text.splitlines())
    code = "".join("".join(l.split()) for l in lines)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def source_digest() -> str:
    return code_digest(PASS_SOURCE.read_text())


def measured_traffic(n_particles: int):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source and this particle count."""
    try:
        d = json.loads(PROFILE_TRAFFIC.read_text())
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != source_digest() or d.get("particles") != n_particles:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w, seconds: float, solver: str = "open", gather: str = "cic"):
    """The oracle on the host cores, on every thread and on one: the ring's
    first space-charge steps on the whole beam, repeated until `seconds` of
    wall time each."""
    import numpy as np

    import oracle
    from paper_2010_11540_amd import inputs

    lat = w["lattice"]
    sc_idx = np.nonzero(lat["kind"] == inputs.SC)[0]
    chunk_steps = min(5, len(sc_idx))
    chunk = lat[: sc_idx[chunk_steps - 1] + 1]
    parts = inputs.copy_parts(w["parts"])

    def run_chunk():
        if "line" in w:
            oracle.track_line(parts, w["grid"], w["line"], chunk, 1)
        else:
            oracle.track(parts, w["grid"], chunk, 1, solver=solver, gather=gather)
        return w["n"] * chunk_steps

    full, one = cpu_both(run_chunk, seconds)
    return {
        "value": full["value"],
        "unit": "particle-steps/s",
        "cores": full["threads"],
        "kind": "oracle",
        "sample": (f"the first {chunk_steps} SC steps of the turn on all {w['n']} particles of the "
                   f"{w['name']} workload, repeated: {full['particle_steps'] // w['n']} steps in "
                   f"{full['wall_s']:.1f} s on {full['threads']} threads, "
                   f"{one['particle_steps'] // w['n']} steps in {one['wall_s']:.1f} s on 1"),
        "value_1thread": one["value"],
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "note": CPU_NOTE,
    }


WORKLOAD_TEXT = {
    "production": ("production 2D PIC: 1e6 Gaussian particles, 128x128 grid, per turn 100 4x4 "
                   "maps + 10 thin sextupoles + 100 SC steps"),
    "small": "small 2D PIC: 1e4 Gaussian particles, 64x64 grid, 16 SC steps/turn",
    "large": ("large 2.5D PIC: 1e7 KV 2:1 long-bunch particles with 128-bin line-density kick "
              "weights, 256x256 grid, 200 SC steps/turn"),
    "line": ("long-bunch 6D PIC: 1e6 Gaussian particles (x, px, y, py, sigma, p_sigma), 128x128 "
             "grounded pipe, 128-node line density of sigma recomputed every SC step "
             "(transverse kick scaled by lambda/lambda_peak, longitudinal kick), per turn 100 thick "
             "FODO cells, 100 SC steps"),
    "thick": ("6D thick-element PIC: 1e6 Gaussian particles (x, px, y, py, sigma, p_sigma), "
              "128x128 grid, per turn 100 FODO cells of 3 chromatic thick quadrupoles + 2 SABA2 "
              "thick sextupoles + 4 drifts, 100 SC steps"),
    "batch": ("tune scan: 64 independent Gaussian beams of 1e4..5e5 particles (8.1e6 in all) on "
              "64x64 / 128x128 grids, tunes on an 8x8 lattice in [4.05, 4.45]^2, 16 SC steps/turn"),
}


# Whole turns timed and warmed up.  A track call launches its first turn
# directly and replays the captured graph of a steady turn for the others, so
# the timed call needs many turns for the replays to dominate it; the warm-up
# call (two turns at least) captures that graph.
MIN_TIMED_TURNS = {"production": 10, "batch": 5, "small": 10}
DEFAULT_TIMED_TURNS = {"production": 20}
MIN_WARMUP_TURNS = 2


def resolve_turns(workload: str, steps, warmup, steps_per_turn: int) -> dict:
    """Turns to time and to warm up for requested SC step counts.  Each
    request is a lower bound: rounded up to whole turns and to the workload's
    minimum (None takes the default).  Any integer is accepted."""
    spt = max(1, int(steps_per_turn))
    min_timed = MIN_TIMED_TURNS.get(workload, 2)
    if steps is None:
        timed = DEFAULT_TIMED_TURNS.get(workload, 20)
    else:
        timed = max(min_timed, math.ceil(max(0, int(steps)) / spt))
    if warmup is None:
        warm = MIN_WARMUP_TURNS
    else:
        warm = max(MIN_WARMUP_TURNS, math.ceil(max(0, int(warmup)) / spt))
    return {"timed_turns": timed, "warmup_turns": warm, "steps": timed * spt,
            "warmup": warm * spt, "steps_requested": steps, "warmup_requested": warmup,
            "steps_per_turn": spt}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine() or "unknown"


def timed_rate(run_chunk, seconds: float) -> tuple[float, int, float]:
    """Call run_chunk() (which returns the particle-steps it did) until
    `seconds` of wall time have passed: (particle-steps/s, particle-steps,
    seconds)."""
    done = 0
    t0 = time.perf_counter()
    while True:
        done += run_chunk()
        el = time.perf_counter() - t0
        if el >= seconds:
            return done / el, done, el


# Particles lost on the way take no further part, so the metric counts the
# alive ones: value = sum over timed steps of the alive count / wall time.
# Lost flags are sticky, so the count after the timed region, times the steps,
# is a lower bound on that sum, and exact when nothing was lost meanwhile.
ALIVE_NOTE = ("sum over the timed steps of the particles alive, taken as steps x alive_after: a "
              "lower bound, exact when alive_before == alive_after")

CPU_NOTE = ("the oracle is plain FP64 C with OpenMP over particles and target nodes; its open-"
            "boundary solve is the direct sum of the Green's function over every charged node "
            "(O(nodes^2) per step, no FFT), which takes most of its time")


def cpu_both(run_chunk, seconds: float) -> tuple[dict, dict]:
    """The oracle's rate on every host thread, then on one thread."""
    import oracle

    oracle.lib()
    threads = oracle.num_threads()
    v_all, done_all, el_all = timed_rate(run_chunk, seconds)
    oracle.set_num_threads(1)
    try:
        v_one, done_one, el_one = timed_rate(run_chunk, seconds)
    finally:
        oracle.set_num_threads(threads)
    return ({"value": v_all, "threads": threads, "particle_steps": done_all, "wall_s": el_all},
            {"value": v_one, "threads": 1, "particle_steps": done_one, "wall_s": el_one})


def cpu_baseline_batch(w, seconds: float):
    """The oracle on the host cores, on every thread and on one: each beam of
    the tune scan in turn through its first 5 space-charge steps, until
    `seconds` of wall time each."""
    import numpy as np

    import oracle
    from paper_2010_11540_amd import inputs

    state = {"k": 0, "beams": 0}

    def run_chunk():
        k = state["k"]
        a, b = int(w["offsets"][k]), int(w["offsets"][k + 1])
        lat = w["lattices"][k]
        sc_idx = np.nonzero(lat["kind"] == inputs.SC)[0]
        chunk = lat[: sc_idx[4] + 1]
        parts = {key: v[a:b].copy() for key, v in w["parts"].items()}
        oracle.track(parts, w["grids"][k], chunk, 1)
        state["k"] = (k + 1) % len(w["grids"])
        state["beams"] += 1
        return (b - a) * 5

    full, one = cpu_both(run_chunk, seconds)
    return {
        "value": full["value"],
        "unit": "particle-steps/s",
        "cores": full["threads"],
        "kind": "oracle",
        "sample": (f"the first 5 SC steps of the tune scan's beams one after another: "
                   f"{full['particle_steps']} particle-steps in {full['wall_s']:.1f} s on "
                   f"{full['threads']} threads, {one['particle_steps']} in {one['wall_s']:.1f} s "
                   f"on 1 ({state['beams']} beams in all)"),
        "value_1thread": one["value"],
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "note": CPU_NOTE,
    }


def run_batch(args):
    import torch

    from paper_2010_11540_amd import inputs, scpic

    w = inputs.batch_workload()
    steps_per_turn = 16
    plan = resolve_turns("batch", args.steps, args.warmup, steps_per_turn)
    b = scpic.Batch(w["grids"], w["offsets"], args.precision)
    d = scpic.to_device(w["parts"])
    torch.cuda.synchronize()
    threads, per_cu = b.autotune(d, w["lattices"], trial_turns=2)
    print(f"[bench] autotuned pass shape: {threads} threads, {per_cu} workgroups per CU",
          file=sys.stderr, flush=True)
    b.track(d, w["lattices"], plan["warmup_turns"])
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({plan['warmup']} steps)", file=sys.stderr, flush=True)
    n = w["n"]
    alive_before = int((d["lost"] == 0).sum().item())
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    b.track(d, w["lattices"], plan["timed_turns"])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    print(f"[bench] timed {plan['steps']} steps: {wall * 1e3:.1f} ms wall, {gpu_ms:.1f} ms events",
          file=sys.stderr, flush=True)
    alive = int((d["lost"] == 0).sum().item())
    cpu = None
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline_batch(w, args.cpu_seconds)
    out = {
        "metric": "particle-steps/s (push+deposit+solve+kick)",
        "value": alive * plan["steps"] / wall,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": plan["steps"],
        "warmup": plan["warmup"],
        "steps_requested": plan["steps_requested"],
        "warmup_requested": plan["warmup_requested"],
        "ms_per_step": wall * 1e3 / plan["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 coords / f32 field",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["batch"], "particles": n, "beams": len(w["grids"]),
                   "sc_steps_per_turn": steps_per_turn, "precision": args.precision,
                   "graph": True, "pass_threads": threads, "pass_workgroups_per_cu": per_cu,
                   "alive_before": alive_before, "alive_after": alive,
                   "value_counts": ALIVE_NOTE, "gpu_event_ms": round(gpu_ms, 3)},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    b.close()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): "
              "the space-charge loop is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2010_11540_amd import inputs, scpic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.stream_ceiling:
        stream_ceiling()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch":
        run_batch(args)
        return
    w = inputs.workload(args.workload)
    lat = w["lattice"]
    steps_per_turn = int((lat["kind"] == inputs.SC).sum())
    plan = resolve_turns(args.workload, args.steps, args.warmup, steps_per_turn)
    n = w["n"]
    ctx = scpic.Context(w["grid"], args.precision)
    if "solver" in w:
        args.solver = w["solver"]
    if args.solver == "pipe":
        ctx.set_option(scpic.OPT_SOLVER, scpic.SOLVER_PIPE)
    if "line" in w:
        ctx.set_line_density(w["line"])
    if args.gather == "bspline":
        ctx.set_option(scpic.OPT_GATHER, scpic.GATHER_BSPLINE)
    if args.no_graph:
        ctx.set_option(scpic.OPT_USE_GRAPH, 0)
    if args.pass_threads:
        ctx.set_option(scpic.OPT_PASS_THREADS, args.pass_threads)
    if args.pass_blocks:
        ctx.set_option(scpic.OPT_PASS_BLOCKS, args.pass_blocks)
    d = scpic.to_device(w["parts"])
    torch.cuda.synchronize()

    ctx.track(d, lat, plan["warmup_turns"])
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({plan['warmup']} steps)", file=sys.stderr, flush=True)
    alive_before = int((d["lost"] == 0).sum().item())

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.track(d, lat, plan["timed_turns"])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    print(f"[bench] timed {plan['steps']} steps: {wall * 1e3:.1f} ms wall, {gpu_ms:.1f} ms events",
          file=sys.stderr, flush=True)
    seconds = wall
    alive = int((d["lost"] == 0).sum().item())
    value = alive * plan["steps"] / seconds

    # dominant kernel: the fused pass (kick + the elements of the turn's first
    # segment + deposit), timed alone on the same stream over a copy of the beam
    d2 = {k: v.clone() for k, v in d.items()}
    first_sc = int(np.nonzero(lat["kind"] == inputs.SC)[0][0])
    one_map = lat[:first_sc]
    kappa = float(lat["p"][lat["kind"] == inputs.SC][0, 0])
    scale = 1.0 / ((1 << 24) * n)
    for _ in range(5):
        ctx.pass_(d2, True, kappa, one_map, True)
        ctx.reduce_solve(scale)
    torch.cuda.synchronize()
    pass_us = stream_time_us(stream, lambda: ctx.pass_(d2, True, kappa, one_map, True),
                             args.pass_reps)
    grid_us = stream_time_us(stream, lambda: ctx.reduce_solve(scale), args.pass_reps)

    six = "sigma" in d and bool(np.isin(one_map["kind"], (inputs.QUAD_THICK, inputs.SEXT_THICK)).any())
    line_on = "line" in w
    six = six or line_on
    unit_bytes = (BYTES_PER_PARTICLE_STEP + (BYTES_PER_WEIGHT if "w" in d else 0)
                  + (BYTES_PER_LONGITUDINAL if six else 0) + (BYTES_LINE_KICK if line_on else 0))
    achieved = unit_bytes * n / (pass_us * 1e-6) / 1e9
    seg = {"production": "4x4 map", "thick": "FODO cell of thick elements",
           "line": "FODO cell of thick elements, line density"}.get(args.workload, "2x2 map")
    # the library streams the coordinates of four-dimensional CIC passes over
    # arrays above 128 MiB (non-temporal loads and stores)
    array_bytes = n * (8 * sum(k in d for k in ("x", "px", "y", "py", "sigma", "psigma"))
                       + (4 if "w" in d else 0) + (1 if "lost" in d else 0))
    streamed = not six and args.gather == "cic" and array_bytes > (128 << 20)
    roofline = {
        "bound": "hbm",
        "kernel": (f"k_pass{'_line' if line_on else ('_bspline' if args.gather == 'bspline' else '')}<"
                   f"{'double' if args.precision == 'fp64' else 'float'},kick,deposit"
                   f"{',six' if six and not line_on else ''}{',stream' if streamed else ''}> "
                   f"(gather+kick, {seg}, CIC deposit, flush)"),
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": (measured_traffic(n) if args.workload == "production" and args.gather == "cic"
                    else None),
        "algorithmic_bytes_per_launch": unit_bytes * n,
        "avg_launch_us": round(pass_us, 3),
        "grid_phase_us": round(grid_us, 3),
    }
    if six:
        # thick elements make the pass arithmetic-bound: FP64 roofline, with
        # the HBM figures kept beside it
        flops = (FLOPS_KICK + FLOPS_DEPOSIT + FLOPS_CHROMA + (FLOPS_LINE if line_on else 0)
                 + sum(element_flops(e, inputs) for e in one_map))
        tflops = flops * n / (pass_us * 1e-6) / 1e12
        roofline.update({
            "bound": "alu", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
            "flops_per_particle": flops, "hbm_achieved_gbs": round(achieved, 1),
            "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)})
    # the pass's two particle stages alone: the push (the segment's elements,
    # no kick or deposit) and the interpolation + kick (no elements, no
    # deposit), each one kernel on the same stream
    no_el = lat[:0]
    push_us = stream_time_us(stream, lambda: ctx.pass_(d2, False, 0.0, one_map, False),
                             args.pass_reps)
    kick_us = stream_time_us(stream, lambda: ctx.pass_(d2, True, kappa, no_el, False),
                             args.pass_reps)
    ext = BYTES_PER_WEIGHT if "w" in d else 0
    push_bytes = (BYTES_PER_PARTICLE_STEP + (BYTES_PER_LONGITUDINAL if "sigma" in d and six else 0)) * n
    # read x, y, px, py and write px, py; the line kick also reads sigma, p_sigma, writes p_sigma
    kick_bytes = (48 + ext + (24 if "line" in w else 0)) * n
    components = {
        "push": {"us": round(push_us, 3), "bytes": push_bytes,
                 "GBps": round(push_bytes / (push_us * 1e-6) / 1e9, 1),
                 "frac": round(push_bytes / (push_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "kick": {"us": round(kick_us, 3), "bytes": kick_bytes,
                 "GBps": round(kick_bytes / (kick_us * 1e-6) / 1e9, 1),
                 "frac": round(kick_bytes / (kick_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "note": ("each stage alone, one kernel per launch, launches back to back, algorithmic "
                 "bytes; a beam below the 256 MB last-level cache can exceed the HBM figure"),
    }
    del d2

    cpu = None
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_seconds, args.solver, args.gather)

    out = {
        "metric": METRIC if args.workload == "production" else
                  "particle-steps/s (push+deposit+solve+kick)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": plan["steps"],
        "warmup": plan["warmup"],
        "steps_requested": plan["steps_requested"],
        "warmup_requested": plan["warmup_requested"],
        "ms_per_step": seconds * 1e3 / plan["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 coords / f32 field",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT[args.workload],
            "particles": n,
            "grid": f"{w['grid']['nx']}x{w['grid']['ny']}",
            "sc_steps_per_turn": steps_per_turn,
            "precision": args.precision,
            "solver": args.solver,
            "gather": args.gather,
            "graph": not args.no_graph,
            "alive_before": alive_before,
            "alive_after": alive,
            "value_counts": ALIVE_NOTE,
            "gpu_event_ms": round(gpu_ms, 3),
        },
        "step_hbm_frac": round(BYTES_PER_PARTICLE_STEP * value / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roofline,
        "stages": components,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
