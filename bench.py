"""Throughput of the coupled flow + thermal lattice update on one MI355X.

One step = the whole per-time-step update over the workload, driven through
the C ABI: for many particles the particle pass (particle update, neighbour
repulsion, per-tile lists), then one launch of the fused step kernel (solid
fractions, both lattices, momentum exchange); for few particles the step
kernel alone.  The headline workload is the largest single-GPU
configuration, the 1536 x 1536 cavity holding 2048 settling cold disks of
diameter 16; the headline value is its FP64 throughput in MLUPS (every
cell counts).  The same line reports the FP32 / FP16-shifted /
BF16-shifted forms, the step kernel's achieved HBM bandwidth against the
8 TB/s peak, the bandwidth of a plain device copy, the 200 x 4000
single-disk channel (its working set fits the 256 MB Infinity Cache), the
channel's physics on 16 M cells, the 256-domain batch, the two
three-dimensional workloads (FP64 and the FP32 storage form), and the FP64
CPU oracle timed on a bounded sample of the headline workload on the host
cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled flow+thermal MLUPS & %HBM roofline, FP64 vs FP32 vs FP16-shifted"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell and step: both D2Q9 population sets read once
# and written once, plus the [df_s/dt] carrier read and written once.
BYTES_PER_CELL = {"fp64": 2 * 18 * 8 + 2 * 8, "fp32": 2 * 18 * 4 + 2 * 4,
                  "fp16s": 2 * 18 * 2 + 2 * 4, "bf16s": 2 * 18 * 2 + 2 * 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f16 storage, f32 arithmetic",
         "bf16s": "bf16 storage, f32 arithmetic"}
# the step kernel and its launch shape (tile mapping, grid) come from these
KERNEL_SOURCES = ["paper_2410_23802_amd/csrc/vlb_device.h",
                  "paper_2410_23802_amd/csrc/vlb_kernels.hip",
                  "paper_2410_23802_amd/csrc/vlb_internal.h",
                  "paper_2410_23802_amd/csrc/vlb_api.hip",
                  "paper_2410_23802_amd/build.py"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as fh:
            h.update(code_only(fh.read(), p.endswith(".py")).encode())
    return h.hexdigest()[:16]


def code_only(text: str, python: bool) -> str:
    """The source without its comments and blank-space differences, so that
    an edit of comments alone keeps the hash (it changes no kernel)."""
    if python:
        text = re.sub(r"#[^\n]*", "", text)
    else:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
    return " ".join(text.split())


def measured_traffic(workload: str, precision: str):
    """HBM bytes per step-kernel launch (FETCH_SIZE + WRITE_SIZE, each
    scaled by what it reads for a copy of known size) from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_k_step_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    ent = rec.get("per_precision", {}).get(precision)
    return None if ent is None else ent.get("bytes_per_launch")


def run_gpu(vlb, d, ps, precision, steps, warmup):
    """K steps with nothing else on the stream give the throughput; then K
    more steps with every launch of the step kernel bracketed by HIP events
    (recorded by the dispatch, on the context stream) give its average
    duration for the roofline."""
    import torch
    dom = vlb.Domain(d, ps, precision).init()
    if warmup:
        dom.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps)                        # returns after the stream drained
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom.timing(True)
    dom.timing_read()                      # reset the event pairs
    dom.step(steps)
    ker_ms, nker = dom.timing_read()
    dom.timing(False)
    # the same memory pattern without the arithmetic: the ceiling
    probe_ms = dom.stream_probe(min(steps, 100)) * 1e-3
    p = dom.particles()
    dom.close()
    cells = d["nx"] * d["ny"]
    wall = t1 - t0
    return {
        "mlups": cells * steps / wall / 1e6,
        "ms_per_step": wall * 1e3 / steps,
        "lattice_ms": ker_ms / max(nker, 1),
        "launches": nker,
        "probe_ms": probe_ms,
        "particle_y": float(p["y"][0]) if len(p) else None,
    }


WORKLOADS = {
    "c3_dense": "1536 x 1536 cavity, 2048 cold disks of D = 16 settling "
                "(list form: particle pass + step kernel)",
    "c2_channel": "200 x 4000 channel, one cold disk of D = 20 (scan form; "
                  "working set within the 256 MB Infinity Cache below FP64)",
    "c2_channel_1000x16000": "the channel's physics on 1000 x 16000 cells "
                             "(working sets 1.3-4.9 GB, HBM-bound)",
}


def make_workload(name):
    import workloads as W
    if name == "c3_dense":
        return W.c3_dense()
    if name == "c2_channel":
        return W.c2_channel()
    if name == "c2_channel_1000x16000":
        return W.c2_channel(nx=1000, ny=16000)
    raise KeyError(name)


def run_workload(vlb, name, precs, steps, warmup):
    """Every storage form of one workload: whole-step MLUPS, and the step
    kernel's event-timed duration against its algorithmic bytes and against
    the memory-pattern probe of the same cells in the same tile order."""
    d, ps = make_workload(name)
    cells = d["nx"] * d["ny"]
    out = {}
    for prec in precs:
        r = run_gpu(vlb, d, ps, prec, steps, warmup)
        gbs = BYTES_PER_CELL[prec] * cells / (r["lattice_ms"] * 1e-3) / 1e9
        ceil = BYTES_PER_CELL[prec] * cells / (r["probe_ms"] * 1e-3) / 1e9
        r.update(achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS, ceiling_GBs=ceil)
        out[prec] = r
        print(f"# {name} {prec}: {r['mlups']:.0f} MLUPS, "
              f"{r['ms_per_step'] * 1e3:.1f} us/step, k_step "
              f"{r['lattice_ms'] * 1e3:.1f} us -> {gbs:.0f} GB/s "
              f"({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak; pattern "
              f"ceiling {ceil:.0f} GB/s)", file=sys.stderr, flush=True)
    return d, ps, out


def form_key(prec):
    return DTYPE[prec].split(" ")[0] + ("-shifted" if prec.endswith("s") else "")


def forms_block(res, precs):
    return {form_key(p): {
        "mlups": round(res[p]["mlups"], 1),
        "ms_per_step": round(res[p]["ms_per_step"], 5),
        "k_step_us": round(res[p]["lattice_ms"] * 1e3, 2),
        "rest_of_step_us": round((res[p]["ms_per_step"]
                                  - res[p]["lattice_ms"]) * 1e3, 2),
        "achieved_GBs": round(res[p]["achieved_GBs"], 1),
        "frac_hbm": round(res[p]["frac"], 4),
        "pattern_ceiling_GBs": round(res[p]["ceiling_GBs"], 1),
        "frac_of_pattern_ceiling": round(res[p]["achieved_GBs"]
                                         / res[p]["ceiling_GBs"], 4),
        "bytes_per_cell": BYTES_PER_CELL[p],
    } for p in precs}


def run_batch(vlb, steps, warmup):
    """The 256 uneven single-particle domains in FP32: one autotuned batch
    (one launch per step, graph replay) against the same domains run one at
    a time, each for the same steps.  Aggregate MLUPS = all cells x steps /
    wall time."""
    import torch
    import workloads as W
    cases = W.c5_batch()
    b = vlb.Batch(cases, "fp32").init()
    tune = b.autotune(3)
    cells = b.cells
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    batch_s = time.perf_counter() - t0
    b.close()
    batched = cells * steps / batch_s / 1e6
    seq = 0.0
    for d, ps in cases:
        dom = vlb.Domain(d, ps, "fp32").init()
        dom.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dom.step(steps)
        seq += time.perf_counter() - t0
        dom.close()
    single = cells * steps / seq / 1e6
    print(f"# batch: {len(cases)} domains, {cells} cells: {batched:.0f} MLUPS "
          f"batched vs {single:.0f} one at a time ({batched / single:.2f}x); "
          f"tuning {tune}", file=sys.stderr, flush=True)
    return {"workload": "c5_batch", "domains": len(cases), "cells": cells,
            "precision": "fp32 storage and arithmetic, fp64 particle sums",
            "steps": steps, "mlups_batched": round(batched, 1),
            "ms_per_step_batched": round(batch_s * 1e3 / steps, 4),
            "mlups_one_at_a_time": round(single, 1),
            "speedup": round(batched / single, 3),
            # algorithmic bytes (every cell's populations read and written
            # once) over the batched step time, against 8 TB/s
            "achieved_GBs": round(cells * BYTES_PER_CELL["fp32"] * steps
                                  / batch_s / 1e9, 1),
            "frac_hbm": round(cells * BYTES_PER_CELL["fp32"] * steps
                              / batch_s / 1e9 / HBM_PEAK_GBS, 4),
            "tuning": {k: (round(v, 2) if isinstance(v, float) else v)
                       for k, v in tune.items()}}


# Algorithmic bytes per cell and step in three dimensions (FP64): the 19
# flow and 7 energy populations read once and written once, and the
# [df_s/dt] carrier read and written once.
# (19 + 7) populations and the carrier, read and written: FP64 and the FP32
# storage form (whose arithmetic is FP64 too)
BYTES_PER_CELL3 = {"fp64": 2 * (19 + 7) * 8 + 2 * 8,
                   "fp32": 2 * (19 + 7) * 4 + 2 * 4}
WORKLOADS3 = {
    "c6_sphere_channel3": "80 x 80 x 320 channel, one cold sphere of D = 16 "
                          "settling (D3Q19 flow, D3Q7 energy, FP64)",
    "c7_spheres_box3": "96^3 box, 64 cold spheres of D = 12 settling "
                       "(D3Q19 flow, D3Q7 energy, FP64)",
}


def run_3d(vlb, steps, warmup):
    """The three-dimensional path on both workloads, FP64 (the top-level
    keys) and the FP32 storage form ("fp32"): whole-step MLUPS and the
    lattice step kernel's event-timed duration against its algorithmic
    bytes."""
    import torch
    import workloads as W
    out = {}
    for name, what in WORKLOADS3.items():
        d, ps = getattr(W, name)()
        cells = d["nx"] * d["ny"] * d["nz"]
        res = {}
        for prec in ("fp64", "fp32"):
            dom = vlb.Domain3(d, ps, precision=prec).init()
            dom.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dom.step(steps)
            wall = time.perf_counter() - t0
            dom.timing(True)
            dom.timing_read()
            dom.step(steps)
            ms, n = dom.timing_read()
            dom.timing(False)
            dom.close()
            k_ms = ms / max(n, 1)
            bpc = BYTES_PER_CELL3[prec]
            gbs = bpc * cells / (k_ms * 1e-3) / 1e9
            res[prec] = {"mlups": round(cells * steps / wall / 1e6, 1),
                         "ms_per_step": round(wall * 1e3 / steps, 4),
                         "k3_step_us": round(k_ms * 1e3, 2),
                         # the sphere pass and the geometry passes (exact
                         # sphere-cell volumes, FP64-bound)
                         "rest_of_step_us": round(
                             wall * 1e6 / steps - k_ms * 1e3, 2),
                         "achieved_GBs": round(gbs, 1),
                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_cell": bpc}
            print(f"# 3-D {name} {prec}: {res[prec]['mlups']} MLUPS, k3_step "
                  f"{k_ms * 1e3:.1f} us -> {gbs:.0f} GB/s", file=sys.stderr,
                  flush=True)
        out[name] = {"workload": what, "cells": cells, "spheres": len(ps),
                     **res["fp64"], "fp32": res["fp32"]}
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _oracle_rate(O, d, ps, threads, target_s):
    """MLUPS of the oracle on `threads` threads: one untimed step, then as
    many steps as take about target_s seconds."""
    O.set_threads(threads)
    o = O.Oracle(d, ps).init()
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    n = max(1, int(target_s / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    o.close()
    return d["nx"] * d["ny"] * n / dt / 1e6, n, dt


def cpu_baseline(d, ps, workload, target_s=20.0):
    """The FP64 oracle as it stands, on a bounded sample of the same
    workload, on up to 16 host threads (and, for reference, on one)."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    threads = min(os.cpu_count() or 1, 16)
    v, n, dt = _oracle_rate(O, d, ps, threads, target_s)
    v1, n1, dt1 = _oracle_rate(O, d, ps, 1, target_s / 4)
    return {"value": round(v, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{workload}: {d['nx']}x{d['ny']} cells, {len(ps)} "
                      f"particles, {n} steps after one untimed step, FP64, "
                      f"{threads} OpenMP threads, {dt:.1f} s, on {_cpu_model()}",
            "value_1_thread": round(v1, 3),
            "sample_1_thread": f"{n1} steps on 1 thread, {dt1:.1f} s"}


def copy_bandwidth(torch, nbytes, reps=10):
    """A plain device-to-device copy of nbytes (reads and writes nbytes
    each): a few untimed copies, then `reps` timed with events on the
    current stream.  Returns the achieved read + write GB/s, the bandwidth
    the chip delivers to the simplest stream.  Under a counter run these
    copies also calibrate FETCH_SIZE / WRITE_SIZE against bytes known to
    move."""
    n = max(1, nbytes // 4)
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    gbs = 2 * 4 * n / (ms * 1e-3) / 1e9
    print(f"# copy: {4 * n} bytes in {ms * 1e3:.1f} us -> {gbs:.0f} GB/s",
          file=sys.stderr, flush=True)
    return {"bytes": 4 * n, "us": round(ms * 1e3, 1), "GBs": round(gbs, 1),
            "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--precisions", default="fp64,fp32,fp16s,bf16s")
    ap.add_argument("--workload", default="c3_dense", choices=tuple(WORKLOADS),
                    help="headline workload (default: the 2048-disk cavity)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-domains measurement")
    ap.add_argument("--no-channel", action="store_true",
                    help="skip the 200 x 4000 channel measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 16 M-cell channel measurement")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the three-dimensional measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library steps one domain per GPU and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_23802_amd import vlb
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if not os.path.exists(vlb.LIB_PATH):
        from paper_2410_23802_amd import build as hb
        hb.build()
    torch.cuda.set_device(0)
    copy = copy_bandwidth(torch, 1 << 30)

    workload = args.workload
    precs = [p for p in args.precisions.split(",") if p]
    # untimed: bring the GPU to its working clocks (about half a second of
    # steps) so the first form timed is not measured on a cold device
    d, ps = make_workload(workload)
    dom = vlb.Domain(d, ps, precs[0]).init()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.5:
        dom.step(20)
    dom.close()
    d, ps, res = run_workload(vlb, workload, precs, args.steps, args.warmup)
    cells = d["nx"] * d["ny"]
    head = res[precs[0]]
    traffic = measured_traffic(workload, precs[0])
    line = {
        "metric": METRIC,
        "value": round(head["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[precs[0]],
        "data": "synthetic",
        "config": {"workload": workload, "description": WORKLOADS[workload],
                   "nx": d["nx"], "ny": d["ny"], "particles": len(ps),
                   "particle_diameter": 2 * ps[0]["radius"],
                   "lattices": "D2Q9 flow + D2Q9 energy, MRT",
                   "precision": precs[0]},
        "roofline": {
            "bound": "hbm",
            "achieved": round(head["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(head["frac"], 4),
            "traffic": traffic,
            "kernel": "k_step",
            "bytes_per_cell": BYTES_PER_CELL[precs[0]],
            "cells_per_launch": cells,
            "avg_launch_us": round(head["lattice_ms"] * 1e3, 2),
            "pattern_ceiling_GBs": round(head["ceiling_GBs"], 1),
            "frac_of_pattern_ceiling": round(head["achieved_GBs"]
                                             / head["ceiling_GBs"], 4),
            "copy_GBs": copy["GBs"],
            "frac_of_copy": round(head["achieved_GBs"] / copy["GBs"], 4),
        },
        "precisions": forms_block(res, precs),
        "copy": copy,
    }
    if not args.no_channel and workload != "c2_channel":
        _, _, r2 = run_workload(vlb, "c2_channel", precs, args.steps,
                                args.warmup)
        line["channel"] = {"workload": "c2_channel",
                           "description": WORKLOADS["c2_channel"],
                           **forms_block(r2, precs)}
    if not args.no_large and workload != "c2_channel_1000x16000":
        _, _, r3 = run_workload(vlb, "c2_channel_1000x16000", precs,
                                min(args.steps, 50), 4)
        line["large"] = {"workload": "c2_channel_1000x16000",
                         "description": WORKLOADS["c2_channel_1000x16000"],
                         **forms_block(r3, precs)}
    if not args.no_batch:
        line["batch"] = run_batch(vlb, min(args.steps, 100), 4)
    if not args.no_3d:
        line["three_d"] = run_3d(vlb, min(args.steps, 100), 4)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(d, ps, workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
