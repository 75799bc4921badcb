#!/usr/bin/env python
"""Zone-updates per second of the AMR MHD hot path on one MI355X.

One step = one root step of the whole hierarchy: CFL reduction, ghost
exchange, prolongation, the advance of every level (level l takes 2^l
substeps), restriction with flux/EMF correction and same-level
synchronisation.  A zone-update is one interior cell of one patch advanced
one substep of its level (redundant extended-ghost updates are not counted).

Prints one JSON line.  Inputs are seeded synthetic states resident in HBM
before the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_TFLOPS = 78.6        # 256 CU x 128 FP32 FMA-flops/clk (unpacked) x 2.4 GHz
FP64_VALU_TFLOPS = 78.6

# Algorithmic words moved per processed entry of each kernel class (reads + writes of
# distinct values, neighbour re-reads not counted); see DESIGN.md "Kernels and rooflines".
WORDS_PER_UNIT = {
    "prim": 8 + 11,      # U (5) + one face per axis (3) in; w (8) + cell EMF (3) out
    "bhalf": 6 + 3,      # 3 faces + 3 cell EMFs in; 3 half-step faces out
    "pred": 8 + 4 + 3 + 8 + 3,  # w, rho and m, half-step faces in; increment (8) + reference EMF (3) out
    "flux": 17 + 7,      # w (8), increment (8), half-step normal field in; 5 fluxes + 2 face EMFs out
    "edge": 5 + 1,       # 2 face EMFs, 2 mass fluxes, reference EMF in; edge EMF out
    "update": 26 + 8,    # U (5), fluxes (15), faces (3), edge EMFs (3) in; 8 out
    "copy": 2,           # one element in, one out
    "primhalf": 1,       # fused prim/bhalf/pred: the library reports its algorithmic words directly
}

# HBM bytes per launch of the dominant kernel measured with rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a
# 512 MiB copy's readings), keyed by (workload, precision, kernel class); valid only for the kernel sources whose
# hash is stored beside it, null otherwise.
MEASURED_TRAFFIC = {
    ("two_level", "fp32", "flux"): {"bytes_per_launch": 716.4e6, "sources": "d673f467b369686f:2e7a3d55329dfdaa"},
}


def sources_hash():
    import hashlib
    out = []
    for f in ("kernels.hip", "amrx_internal.h"):
        with open(os.path.join(ROOT, "paper_1112_1710_amd", "csrc", f), "rb") as fh:
            out.append(hashlib.sha256(fh.read()).hexdigest()[:16])
    return ":".join(out)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="two_level", choices=["two_level", "uniform256", "uniform32", "deep"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_mixed", "fp64"])
    ap.add_argument("--mode", default="graph", choices=["plain", "batched", "graph", "persistent", "concurrent"])
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="after the timed steps, copy a 512 MiB buffer once (reference dispatch for HBM counters)")
    ap.add_argument("--plain-steps", type=int, default=4, help="steps of the FP64 per-patch-launch comparison")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--staged", action="store_true", help="run the first three advance stages as separate kernels")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile of the fused kernel")
    return ap.parse_args()


def workload(name):
    from workloads import hierarchies as H
    from workloads.fields import Blast, SmoothField
    if name == "two_level":
        return H.two_level(), SmoothField(1112), "two-level 128^3 root + 512 refined patches (ratio 2), smooth field"
    if name == "uniform256":
        return H.single_patch(256), SmoothField(1710), "single periodic 256^3 patch, smooth field"
    if name == "uniform32":
        return H.single_patch(32), SmoothField(1112), "single periodic 32^3 patch, smooth field"
    spec, centre, _ = H.deep_blast_target()
    return spec, Blast(centre), "deep 8-level hierarchy (64^3 root, ~40M cells), off-centre blast"


def timed_steps(h, mode, steps, warmup, torch):
    for _ in range(warmup):
        h.step(mode)
    torch.cuda.synchronize()
    h.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        h.step(mode)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.timing(False)
    return (t1 - t0) / steps, h.timing_read()


def cpu_baseline():
    """The oracle, as it stands, on a scaled-down instance of the two-level recipe (one root step)."""
    from oracle import amr
    from workloads import hierarchies as H
    from workloads.fields import SmoothField
    spec = H.two_level(root=32, count=32)
    o = amr.build(spec, SmoothField(1112))
    t0 = time.perf_counter()
    o.root_step()
    el = time.perf_counter() - t0
    zu = spec.zone_updates_per_root_step()
    return {"value": zu / el, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one root step of the two-level recipe scaled to a 32^3 root + {len(spec.patches) - 1} "
                      f"refined patches ({zu} zone-updates, {el:.1f} s, single-threaded NumPy float64)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.stderr.write("bench.py measures one GPU only: this build has no multi-GPU path "
                         "(run with --gpus 1).\n")
        sys.exit(2)
    import torch

    from paper_1112_1710_amd import BATCHED, CONCURRENT, FP32, FP32_MIXED, FP64, GRAPH, PERSISTENT, PLAIN, Hierarchy
    from paper_1112_1710_amd.binding import TUNE_FUSED
    prec = {"fp32": FP32, "fp32_mixed": FP32_MIXED, "fp64": FP64}[args.precision]
    mode = {"plain": PLAIN, "batched": BATCHED, "graph": GRAPH, "persistent": PERSISTENT,
            "concurrent": CONCURRENT}[args.mode]
    spec, field, desc = workload(args.workload)
    zu = spec.zone_updates_per_root_step()

    h = Hierarchy(spec, prec)
    h.set_field(field)
    tiles = None
    if args.staged:
        h.tune_set(TUNE_FUSED, 0)
    elif not args.no_autotune:
        from paper_1112_1710_amd.autotune import autotune
        tiles = {lvl: v[1] for lvl, v in autotune(h).items()}
    sec, timing = timed_steps(h, mode, args.steps, args.warmup, torch)
    value = zu / sec
    work = h.step_work()
    if mode in (GRAPH, PERSISTENT, CONCURRENT):
        # kernels inside a replayed graph or the persistent kernel are not bracketed by events: take the per-kernel
        # launch times from an instrumented batched pass of the same steps
        _, timing = timed_steps(h, BATCHED, args.steps, 1, torch)

    # dominant kernel class and its roofline
    dom = max(timing, key=lambda k: timing[k][0])
    ms_total, nlaunch = timing[dom]
    units_per_step, launches_per_step = work[dom]
    word = 8 if prec == FP64 else 4
    roof = None
    if dom in WORDS_PER_UNIT and nlaunch:
        bytes_per_launch = units_per_step * WORDS_PER_UNIT[dom] * word / max(launches_per_step, 1)
        avg_ms = ms_total / nlaunch
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        meas = MEASURED_TRAFFIC.get((args.workload, args.precision, dom))
        traffic = None
        if meas is not None and meas["sources"] == sources_hash():
            traffic = round(meas["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9, 1)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": int(bytes_per_launch),
                "traffic_bytes_per_launch": None if traffic is None else int(meas["bytes_per_launch"])}
    per_class = {k: round(v[0] / args.steps, 4) for k, v in timing.items() if v[1]}
    del h
    torch.cuda.empty_cache()
    if args.pmc_calibration:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    out = {
        "metric": "zone-updates/sec per MI355X (FP32 batched vs FP64 plain) at stated rel-L1; % HBM roof",
        "value": round(value, 1),
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_mixed": "f32+f64", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "patches": len(spec.patches), "levels": spec.levels(),
                   "cells": spec.cells(), "zone_updates_per_step": zu, "precision": args.precision,
                   "schedule": args.mode,
                   "first_stages": "staged" if args.staged or tiles is None else tiles,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernel_ms_per_step": per_class,
    }

    if not args.skip_plain:
        hp = Hierarchy(spec, FP64)
        hp.set_field(field)
        psec, _ = timed_steps(hp, PLAIN, args.plain_steps, 1, torch)
        out["fp64_plain_value"] = round(zu / psec, 1)
        out["speedup_vs_fp64_plain"] = round(value / (zu / psec), 3)
        del hp
        torch.cuda.empty_cache()

    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
