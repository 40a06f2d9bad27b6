"""Throughput of the IFDLBM time step on one MI355X.

Workload (one "step" = one time step of every cavity): the seeded batch of
256 lid-driven isosceles-trapezoid cavities of uneven size and parameters
(sides 65/129/257/513, Re 100-5000 log-uniform, n 0.5-1.5, theta 40-90 deg,
lid 0.1, CFL 0.5).  By default the distributions are stored in FP32 with
stochastic rounding and updated in FP32 arithmetic, with the final sum of
each update in FP64 (--precision selects the other modes); FP64 residual sums
of Eq. (2.19) every 100 steps; all cavities in one launch per step, replayed
from captured HIP graphs of 100 steps.  With fewer than 100 timed steps the
graph and the residual interval shrink to the timed count, so that the timed
region is whole graph replays, each with one residual step; the JSON line
records what the timed region ran.  Inputs start resident in HBM (Step 1 on
the device).  Printed on one JSON line: MLUPS, the roofline record of the
step kernel (algorithmic bytes per launch over its average duration, from HIP
events on the stream the library launches on), the same batch in FP64 with
one launch per cavity and no graph ("plain FP64") and in one launch per step
("batched FP64"), the speedups over both, the other storage modes, and the
serial CPU oracle timed on a bounded sample of the batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, FP32-batched vs plain FP64 on GPU at ≤1e-5 vs oracle"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4   # wave64 VALU instructions per ns: 256 CUs, 4 SIMD16 each, 2.4 GHz
WORKLOAD = ("256-cavity uneven batch: sides {65,129,257,513}, Re log-uniform [100,5000], n uniform [0.5,1.5], "
            "theta uniform [40,90] deg, lid 0.1, CFL 0.5, central weight 0.75; one launch per step for all cavities; "
            "timed: %s")
# storage of the distributions and arithmetic type of each precision mode
PRECISION = {
    "fp32srf": ("FP32, stochastic rounding; FP32 arithmetic, the final update of f-hat summed in FP64", "f32"),
    "fp32sr": ("FP32, stochastic rounding", "f64"),
    "fp32": ("FP32, round to nearest", "f32"),
    "fp32x": ("FP32, round to nearest", "f64"),
    "fp16dev": ("FP16 of g_k / w_k", "f32"),
    "fp64": ("FP64", "f64"),
}


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


# Kernel sources whose content the measured traffic belongs to: the traffic
# record in profiles/ is used only while these files and the compiler flags
# of step_fused.hip are unchanged.
KERNEL_SOURCES = ["paper_2306_07603_amd/csrc/step_fused.hip", "paper_2306_07603_amd/csrc/lbm_device.h",
                  "paper_2306_07603_amd/csrc/ifdlbm_internal.h"]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_fused_traffic_batch256.txt")


def kernel_source_digest() -> str:
    import hashlib
    from paper_2306_07603_amd import _build
    h = hashlib.sha256()
    h.update(repr(_build.FILE_FLAGS.get("step_fused.hip", [])).encode())
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_record(precision: str, what: str, segment_rows):
    """A per-launch figure of the step kernel at `segment_rows`-row segments,
    recorded in profiles/ from rocprofv3 counter passes: what = "bytes"
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a
    plain copy of known size) or "valu_insts" (SQ_INSTS_VALU, wavefront
    instructions).  None when the record is absent, was taken on other kernel
    sources or holds no figure for that segment length."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = {}
    with open(TRAFFIC_RECORD) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_sources_sha256") != kernel_source_digest():
        return None
    if not segment_rows:
        return None
    key = "%s_per_launch_%s_seg%d" % (what, precision, segment_rows)
    return float(rec[key]) if key in rec else None


def binding_limit(hbm_frac: float, valu):
    """The limit the kernel runs into: "valu" when the VALU issue fraction of the
    same launches exceeds the memory fraction `hbm_frac`, else "hbm"; None
    without a VALU figure.  The memory fraction is the measured traffic rate
    over the device-copy rate of the same run when both are known, else the
    algorithmic rate over the HBM peak."""
    if not valu:
        return None
    return "valu" if valu["frac"] > hbm_frac else "hbm"


def time_steps(M, h, stream, steps: int, warmup: int):
    import torch
    M.ifdlbm_step(h, warmup)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    M.ifdlbm_step(h, steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(end)


def cpu_baseline(specs, steps: int):
    """The serial FP64 oracle on one cavity of each side of the batch."""
    import oracle as O
    picks = []
    for side in (65, 129, 257, 513):
        for s in specs:
            if s.n_xi == side:
                picks.append(s)
                break
    nodes = 0
    t0 = time.perf_counter()
    for s in picks:
        p = O.Params(nx=s.n_xi, ny=s.n_eta, re=s.re, n=s.n, theta_deg=s.theta_deg, u_lid=s.u_lid)
        F, L = O.init(p)
        O.run(p, F, L, steps)
        nodes += s.n_xi * s.n_eta * steps
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": nodes / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": "serial FP64 oracle, %d steps of one cavity of each side (65, 129, 257, 513) of the batch, "
                      "%.1f s" % (steps, dt)}


def copy_ceiling(stream, reps: int = 10) -> dict:
    """Rate of a plain device copy of 2 GiB (torch copy_, read + write bytes over
    the HIP-event time on `stream`): the practical ceiling of a stream that reads
    and writes each byte once, on the box the step was timed on."""
    import torch
    n = (2 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        b.copy_(a)
    end.record(stream)
    end.synchronize()
    gbs = 2.0 * n * 4 * reps / (start.elapsed_time(end) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"achieved": gbs, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "what": "device copy of 2 GiB, read + write bytes over HIP-event time, %d copies" % reps}


def copy_calibration() -> int:
    """A device-to-device copy of 2 GiB, three times: under rocprofv3 --pmc the
    FETCH_SIZE and WRITE_SIZE counters of a copy of known size give the scale
    from counter units to bytes on this device."""
    import torch
    n = (2 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "copies": 3}))
    return 0


def timed_schedule(steps: int, warmup: int, graph_steps: int, residual_every: int):
    """Graph size, residual interval and warm-up count of a run of `steps`
    timed steps: with fewer timed steps than a graph holds, the graph and the
    residual interval shrink to the timed count (rounded down to even, as the
    library requires), and the warm-up rounds up to whole graphs, so that the
    timed region starts at a graph boundary."""
    if graph_steps > 0 and steps < graph_steps:
        graph_steps = max(2, steps - steps % 2)
        residual_every = graph_steps
    if graph_steps > 0:
        warmup = -(-warmup // graph_steps) * graph_steps
    return graph_steps, residual_every, warmup


def executed(start: int, steps: int, graph_steps: int, residual_every: int) -> dict:
    """What ifdlbm_step(steps) runs from step count `start`: graph replays
    cover whole graphs from a multiple of graph_steps, the rest is eager
    launches; residual steps are those whose count is a multiple of
    residual_every (the library's schedule)."""
    G = graph_steps
    lead = min((G - start % G) % G, steps) if G > 0 else steps
    replays = (steps - lead) // G if G > 0 else 0
    eager = steps - replays * G
    residual = (start + steps) // residual_every - start // residual_every
    return {"graph_replays": replays, "graph_steps": G, "eager_steps": eager, "residual_steps": residual,
            "residual_every": residual_every}


def describe(ex: dict) -> str:
    parts = []
    if ex["graph_replays"]:
        parts.append("%d replays of a %d-step HIP graph" % (ex["graph_replays"], ex["graph_steps"]))
    if ex["eager_steps"]:
        parts.append("%d eager steps" % ex["eager_steps"])
    parts.append("%d steps with the FP64 residual sums of Eq. (2.19)" % ex["residual_steps"])
    return ", ".join(parts)


def run_mode(M, cav, stream, prec: str, kernel: str, steps: int, warmup: int, **opt):
    """MLUPS of `steps` steps of the batch in another mode (fresh handle)."""
    o = M.ifdlbm_default_options(precision=prec, kernel=kernel, hip_stream=stream.cuda_stream, **opt)
    h = M.ifdlbm_create(cav, o)
    nodes = M.ifdlbm_info(h)["nodes"]
    wall, _ = time_steps(M, h, stream, steps, warmup)
    h.close()
    return nodes * steps / wall / 1e6, wall * 1e3 / steps


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--kernel", default="fused", choices=["fused", "staged"])
    ap.add_argument("--precision", default="fp32srf", choices=["fp32srf", "fp32sr", "fp32", "fp32x", "fp16dev", "fp64"])
    ap.add_argument("--residual-every", type=int, default=100)
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--autotune-steps", type=int, default=40,
                    help="steps per trial of the segment-length autotuner before timing (0: automatic choice)")
    ap.add_argument("--segment-rows", type=int, default=0,
                    help="force the fused kernel's row-segment length (skips the autotuner; for profiling runs)")
    ap.add_argument("--plain-steps", type=int, default=100, help="steps of the plain FP64 comparison run (0: skip)")
    ap.add_argument("--other-steps", type=int, default=300,
                    help="steps of each other mode (batched FP64 and the other storage modes) (0: skip)")
    ap.add_argument("--cpu-steps", type=int, default=100, help="steps of the CPU oracle sample (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy three times (scale for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (cavities are independent; "
              "the batch would shard across GPUs with no communication).", file=sys.stderr)
        return 2

    import torch
    import paper_2306_07603_amd as M
    from paper_2306_07603_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    # a stream of our own (default priority): torch's default stream is the null
    # stream, and the events must be recorded where the library launches
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    specs = W.batch_sweep()
    cav = [M.Cavity(**s.__dict__) for s in specs]
    pr = torch.cuda.get_device_properties(0)
    device = {"name": pr.name, "arch": getattr(pr, "gcnArchName", ""), "compute_units": pr.multi_processor_count,
              "memory_gib": round(pr.total_memory / 2**30, 1)}

    graph_steps, residual_every, warmup_run = timed_schedule(args.steps, args.warmup, args.graph_steps,
                                                             args.residual_every)
    opt = M.ifdlbm_default_options(precision=args.precision, kernel=args.kernel, residual_every=residual_every,
                                   graph_steps=graph_steps, batched=1, hip_stream=stream.cuda_stream,
                                   segment_rows=args.segment_rows)
    h = M.ifdlbm_create(cav, opt)
    seg_rows = args.segment_rows or None
    if args.autotune_steps > 0 and not args.segment_rows and args.kernel == "fused":
        seg_rows, tuned_ms = M.ifdlbm_autotune(h, args.autotune_steps)
        log("autotune: %d-row segments, %.3f ms/step in its trials" % (seg_rows, tuned_ms))
    info = M.ifdlbm_info(h)
    log("created %d cavities, %d nodes per step, %d work items" % (info["n_cavities"], info["nodes"], info["work_items"]))
    ex = executed(warmup_run, args.steps, graph_steps, residual_every)   # the autotuner restores the step count
    wall, ev_ms = time_steps(M, h, stream, args.steps, warmup_run)
    ru, rp = M.ifdlbm_get_residuals(h)
    import numpy as np
    bad = [int(c) for c in np.nonzero(~(np.isfinite(ru) & np.isfinite(rp)))[0]]
    diverged = len(bad)
    if diverged:
        log("WARNING: %d cavities have non-finite residuals: %s" % (diverged, ", ".join(
            "%d (side %d, Re %.0f, n %.3f, theta %.2f)" % (c, specs[c].n_xi, specs[c].re, specs[c].n, specs[c].theta_deg)
            for c in bad)))
    nodes = info["nodes"]
    mlups = nodes * args.steps / wall / 1e6
    launches = args.steps * info["launches_per_step"]
    # HIP-event time of the timed region per launch of the step kernel: it also holds the one-thread seed kernel
    # of each graph replay or eager call and the residual reduction of each residual step (a few microseconds
    # against hundreds per launch)
    kernel_ms = ev_ms / launches
    alg_bytes = nodes * info["alg_bytes_per_node"]
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    log(args.precision + " batched: %.1f MLUPS, %.3f ms/step, %.3f ms per launch (events), %.0f GB/s; timed: %s" % (
        mlups, wall * 1e3 / args.steps, kernel_ms, achieved, describe(ex)))
    # the vector-ALU issue rate of the same launches: SQ_INSTS_VALU per launch (counter record) over the
    # measured launch time, against 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
    insts = measured_record(args.precision, "valu_insts", seg_rows)
    valu = None
    if insts:
        rate = insts / (kernel_ms * 1e-3) / 1e9
        valu = {"achieved": rate, "peak": VALU_PEAK_GINST, "unit": "G wave64 VALU instructions/s",
                "frac": rate / VALU_PEAK_GINST, "insts_per_launch": insts}
    h.close()
    # the memory side of the same launches: the recorded L2-egress bytes per launch over the measured launch
    # time, against the rate a plain device copy reaches on this machine
    copy = copy_ceiling(stream)
    log("device copy: %.0f GB/s" % copy["achieved"])
    traffic = measured_record(args.precision, "bytes", seg_rows)
    traffic_gbs = traffic / (kernel_ms * 1e-3) / 1e9 if traffic else None
    mem_frac = traffic_gbs / copy["achieved"] if traffic_gbs else achieved / HBM_PEAK_GBS

    plain = None
    if args.plain_steps > 0:
        # FP64, one launch per cavity and per step, no graph; each cavity's launch takes the row-segment length
        # that fills the GPU with that cavity alone (the library's rule for unbatched launches)
        v64, ms64 = run_mode(M, cav, stream, "fp64", args.kernel, args.plain_steps, min(args.warmup, 20),
                             residual_every=residual_every, graph_steps=0, batched=0)
        plain = {"value": v64, "unit": "MLUPS", "ms_per_step": ms64, "steps": args.plain_steps,
                 "config": "same batch, FP64, one launch per cavity per step with its own segment length, no graph"}
        log("fp64 plain: %.1f MLUPS" % v64)

    other = {}
    if args.other_steps > 0:
        for prec in ("fp64", "fp32srf", "fp32sr", "fp32", "fp16dev"):
            if prec == args.precision:
                continue
            gs, re_, wu = timed_schedule(args.other_steps, min(args.warmup, 50), args.graph_steps, args.residual_every)
            v, ms = run_mode(M, cav, stream, prec, args.kernel, args.other_steps, wu, residual_every=re_,
                             graph_steps=gs, batched=1)
            other[prec] = {"value": v, "unit": "MLUPS", "ms_per_step": ms, "storage": PRECISION[prec][0],
                           "dtype": PRECISION[prec][1], "steps": args.other_steps,
                           "alg_bytes_per_node": {"fp64": 160.0, "fp16dev": 44.0}.get(prec, 80.0)}
            log("%s batched: %.1f MLUPS" % (prec, v))

    cpu = cpu_baseline(specs, args.cpu_steps) if args.cpu_steps > 0 else None
    if cpu:
        log("cpu oracle: %.3f MLUPS" % cpu["value"])

    fp64_batched = other.get("fp64")
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": PRECISION[args.precision][1], "data": "synthetic",
        "config": {"workload": WORKLOAD % describe(ex), "cavities": len(specs), "nodes_per_step": nodes,
                   "kernel": args.kernel, "precision": args.precision, "storage": PRECISION[args.precision][0],
                   "diverged_cavities": diverged, "diverged_indices": bad, "warmup_steps_run": warmup_run,
                   "segment_rows": seg_rows, "autotune_steps": args.autotune_steps, **ex},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_counters": "FETCH_SIZE + WRITE_SIZE per launch, scaled by a plain copy: bytes between "
                                         "L2 and the memory fabric, Infinity Cache hits included",
                     "traffic_gbs": traffic_gbs,
                     "traffic_frac_of_copy": traffic_gbs / copy["achieved"] if traffic_gbs else None,
                     "copy_ceiling": copy,
                     "event_ms_per_launch": kernel_ms, "alg_bytes_per_launch": alg_bytes,
                     "alg_bytes_per_node": info["alg_bytes_per_node"], "valu": valu,
                     "binding": binding_limit(mem_frac, valu)},
        "fp64_plain": plain,
        "fp64_batched": fp64_batched,
        "other_modes": other or None,
        "speedup_vs_fp64_plain": (mlups / plain["value"]) if plain else None,
        "speedup_vs_fp64_batched": (mlups / fp64_batched["value"]) if fp64_batched else None,
        "cpu_baseline": cpu,
        "device": device,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
