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
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

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
                    help="timed SC steps, a multiple of the steps per turn (default: 1000 for "
                         "production, 20 turns otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed SC steps before timing (default: 200 for production, 2 turns "
                         "otherwise)")
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
    ap.add_argument("--cpu-seconds", type=float, default=6.0,
                    help="wall-clock budget of the CPU oracle sample")
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
    """The oracle on the host cores: the production lattice's first space-charge
    steps on the full beam, repeated until `seconds` of wall time."""
    import numpy as np

    import oracle
    from paper_2010_11540_amd import inputs

    lat = w["lattice"]
    sc_idx = np.nonzero(lat["kind"] == inputs.SC)[0]
    chunk_steps = min(5, len(sc_idx))
    chunk = lat[: sc_idx[chunk_steps - 1] + 1]
    parts = inputs.copy_parts(w["parts"])
    oracle.lib()
    steps = 0
    t0 = time.perf_counter()
    while True:
        if "line" in w:
            oracle.track_line(parts, w["grid"], w["line"], chunk, 1)
        else:
            oracle.track(parts, w["grid"], chunk, 1, solver=solver, gather=gather)
        steps += chunk_steps
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": w["n"] * steps / el,
        "unit": "particle-steps/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} SC steps (first {chunk_steps} segments of the turn, repeated) on all "
                  f"{w['n']} particles of the {w['name']} workload, {el:.1f} s wall",
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


def default_steps(args, steps_per_turn: int):
    if args.steps is None:
        args.steps = 1000 if args.workload == "production" else 20 * steps_per_turn
    if args.warmup is None:
        args.warmup = 200 if args.workload == "production" else 2 * steps_per_turn


def cpu_baseline_batch(w, seconds: float):
    """The oracle on the host cores: each beam of the tune scan in turn through
    its first 5 space-charge steps, until `seconds` of wall time."""
    import numpy as np

    import oracle
    from paper_2010_11540_amd import inputs

    oracle.lib()
    done = 0
    beams = 0
    t0 = time.perf_counter()
    k = 0
    while True:
        a, b = int(w["offsets"][k]), int(w["offsets"][k + 1])
        lat = w["lattices"][k]
        sc_idx = np.nonzero(lat["kind"] == inputs.SC)[0]
        chunk = lat[: sc_idx[4] + 1]
        parts = {key: v[a:b].copy() for key, v in w["parts"].items()}
        oracle.track(parts, w["grids"][k], chunk, 1)
        done += (b - a) * 5
        beams += 1
        k = (k + 1) % len(w["grids"])
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": done / el,
        "unit": "particle-steps/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"first 5 SC steps of {beams} beams of the tune scan (one after another), "
                  f"{done} particle-steps, {el:.1f} s wall",
    }


def run_batch(args):
    import torch

    from paper_2010_11540_amd import inputs, scpic

    w = inputs.batch_workload()
    steps_per_turn = 16
    default_steps(args, steps_per_turn)
    if args.steps % steps_per_turn or args.warmup % steps_per_turn:
        print(f"--steps and --warmup must be multiples of {steps_per_turn} (one turn)",
              file=sys.stderr)
        sys.exit(2)
    b = scpic.Batch(w["grids"], w["offsets"], args.precision)
    d = scpic.to_device(w["parts"])
    torch.cuda.synchronize()
    threads, per_cu = b.autotune(d, w["lattices"], trial_turns=2)
    print(f"[bench] autotuned pass shape: {threads} threads, {per_cu} workgroups per CU",
          file=sys.stderr, flush=True)
    if args.warmup:
        b.track(d, w["lattices"], args.warmup // steps_per_turn)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.track(d, w["lattices"], args.steps // steps_per_turn)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    print(f"[bench] timed {args.steps} steps: {wall * 1e3:.1f} ms wall, {gpu_ms:.1f} ms events",
          file=sys.stderr, flush=True)
    n = w["n"]
    alive = int((d["lost"] == 0).sum().item())
    cpu = None
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline_batch(w, args.cpu_seconds)
    out = {
        "metric": "particle-steps/s (push+deposit+solve+kick)",
        "value": n * args.steps / wall,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 coords / f32 field",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["batch"], "particles": n, "beams": len(w["grids"]),
                   "sc_steps_per_turn": steps_per_turn, "precision": args.precision,
                   "graph": True, "pass_threads": threads, "pass_workgroups_per_cu": per_cu,
                   "alive_after": alive, "gpu_event_ms": round(gpu_ms, 3)},
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
    default_steps(args, steps_per_turn)
    if args.steps % steps_per_turn or args.warmup % steps_per_turn:
        print(f"--steps and --warmup must be multiples of {steps_per_turn} (one turn)",
              file=sys.stderr)
        sys.exit(2)
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

    if args.warmup:
        ctx.track(d, lat, args.warmup // steps_per_turn)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.track(d, lat, args.steps // steps_per_turn)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    print(f"[bench] timed {args.steps} steps: {wall * 1e3:.1f} ms wall, {gpu_ms:.1f} ms events",
          file=sys.stderr, flush=True)
    seconds = wall
    value = n * args.steps / seconds
    alive = int((d["lost"] == 0).sum().item())

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
        "metric": "particle-steps/s (push+deposit+solve+kick)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": seconds * 1e3 / args.steps,
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
            "alive_after": alive,
            "gpu_event_ms": round(gpu_ms, 3),
        },
        "roofline": roofline,
        "stages": components,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
