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
import functools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# vector ALU peaks: 256 CU x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  FP32 reaches 157.3 TFLOP/s only with
# packed two-wide FP32 instructions, which the kernels here do not use; FP64 runs at the same 78.6.
VALU_PEAK_TFLOPS = 78.6

# Kernel classes bound by vector arithmetic rather than HBM, with their algorithmic floating-point operations per
# processed entry: the arithmetic of the oracle's formulas for that stage, each piece of the method computed once
# (add, subtract, multiply, divide, square root, min/max one each per element; signs, absolute values,
# comparisons and selects free), counted on the oracle itself by tests/test_flop_counts.py.
# flux, per face: the two face states formed from the primitives, slopes and increment and converted back (124),
# and HLLD with every region's state and flux evaluated (394); the limited slopes, which the kernel recomputes at
# each face, are priced once, in the Hancock stage.
ALU_BOUND = {"flux": 518}
# The fused first stages (class primhalf), priced per cell of the regions they cover: primitives and cell EMFs
# (34 per cell of the update region grown by 2), the half-step face field (33), the Hancock increments (708: the
# limited slopes and two physical fluxes per axis) and the half-step reference EMF (26), per cell of the region
# grown by 1.
PRIMHALF_FLOPS = {"grown2": 34, "grown1": 33 + 708 + 26}

# Algorithmic words moved per processed entry of each kernel class (reads + writes of
# distinct values, neighbour re-reads not counted).
WORDS_PER_UNIT = {
    "prim": 8 + 11,      # U (5) + one face per axis (3) in; w (8) + cell EMF (3) out
    "bhalf": 6 + 3,      # 3 faces + 3 cell EMFs in; 3 half-step faces out
    "pred": 8 + 4 + 3 + 8 + 3,  # w, rho and m, half-step faces in; increment (8) + reference EMF (3) out
    "flux": 17 + 7,      # w (8), increment (8), half-step normal field in; 5 fluxes + 2 face EMFs out
    "edge": 5 + 1,       # 2 face EMFs, 2 mass fluxes, reference EMF in; edge EMF out
    "update": 26 + 8,    # U (5), fluxes (15), faces (3), edge EMFs (3) in; 8 out
    "copy": 2,           # one element in, one out
    "primhalf": 1,       # fused prim/bhalf/pred: the library reports its algorithmic words directly
    "edgeupd": 1,        # fused edge/update: likewise
}

# HBM bytes per launch of the dominant kernel measured with rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a
# 512 MiB copy's readings), keyed by (workload, precision, kernel class); valid only for the kernel sources whose
# hash is stored beside it and, for the fused first stages, for the same set of fused levels (which sets the
# launches the average runs over), null otherwise.
MEASURED_TRAFFIC = {
    ("deep", "fp32", "primhalf"): [
        {"bytes_per_launch": 2.827e9, "fused_levels": [4, 5, 6, 7], "sources": "587fb17101c0194d:af5e83b69d950ea5"},
        {"bytes_per_launch": 2.747e9, "fused_levels": [3, 4, 5, 6, 7], "sources": "587fb17101c0194d:af5e83b69d950ea5"},
    ],
}

# Fraction of the dominant kernel's vector-ALU issue slots used (SQ_INSTS_VALU against 256 CUs x one
# wave-instruction per cycle x 2.4 GHz over its mean duration), from rocprofv3 counters, same validity rule.
MEASURED_VALU_ISSUE = {
    ("deep", "fp32", "primhalf"): {"frac": 0.67, "sources": "587fb17101c0194d:af5e83b69d950ea5"},
    ("deep", "fp32", "flux"): {"frac": 0.79, "sources": "587fb17101c0194d:af5e83b69d950ea5"},
}


def measured_traffic(workload, precision, kernel_class, fused_levels):
    """The stored counter reading of a kernel class that applies to a run: same workload, precision and
    kernel sources and, where the reading names them, the same fused levels; None if there is none."""
    for m in MEASURED_TRAFFIC.get((workload, precision, kernel_class), []):
        if m["sources"] == sources_hash() and m.get("fused_levels", sorted(fused_levels)) == sorted(fused_levels):
            return m
    return None


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
    ap.add_argument("--workload", default="deep",
                    choices=["two_level", "uniform256", "uniform32", "deep", "lowbeta", "iso_two_level"])
    ap.add_argument("--report-steps", type=int, default=3,
                    help="root steps of the low-beta precision report (workload lowbeta)")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp32_mixed", "fp64"],
                    help="default fp32 (fp32_mixed for the low-beta workload)")
    ap.add_argument("--mode", default="graph", choices=["plain", "batched", "graph", "persistent", "concurrent",
                                                         "layered"])
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="after the timed steps, copy a 512 MiB buffer once (reference dispatch for HBM counters)")
    ap.add_argument("--plain-steps", type=int, default=2, help="steps of the FP64 per-patch-launch comparison")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-precision", action="store_true",
                    help="skip the FP32-with-targeted-FP64 timing and the per-step rel-L1 report")
    ap.add_argument("--skip-secondary", action="store_true",
                    help="skip the two-level secondary line of the deep workload")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--cpu-patches", type=int, default=24,
                    help="patches of the oracle's single-core sample (the pool runs two per worker)")
    ap.add_argument("--staged", action="store_true", help="run every advance stage as a separate kernel")
    ap.add_argument("--regrid-eps", type=float, default=None,
                    help="after the timed steps, time one regrid of the finest level with this flag threshold")
    ap.add_argument("--regrid-from", type=int, default=None,
                    help="with --regrid-eps: regrid every level from this one up, coarse to fine, instead of the "
                         "finest level alone")
    ap.add_argument("--regrid-every", type=int, default=None,
                    help="with --regrid-eps: a separate timed run of --steps root steps that regrids after every "
                         "K root steps inside the loop (levels from --regrid-from, default the finest)")
    ap.add_argument("--ghosts", default="extended", choices=["extended", "time"],
                    help="later-substep ghost data of refined patches: extended ghost regions (default) or the "
                         "coarse time derivative")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile of the fused kernel")
    ap.add_argument("--pair", action="store_true",
                    help="share launches between a level's advance and the finer level's first substep")
    return ap.parse_args()


# physics of each workload other than ideal MHD: (physics, isothermal sound speed)
WORKLOAD_PHYSICS = {"iso_two_level": ("isothermal", 1.0)}


@functools.lru_cache(maxsize=None)
def workload(name):
    from workloads import hierarchies as H
    from workloads.fields import Blast, SmoothField
    if name == "two_level":
        return H.two_level(), SmoothField(1112), "two-level 128^3 root + 512 refined patches (ratio 2), smooth field"
    if name == "uniform256":
        return H.single_patch(256), SmoothField(1710), "single periodic 256^3 patch, smooth field"
    if name == "uniform32":
        return H.single_patch(32), SmoothField(1112), "single periodic 32^3 patch, smooth field"
    if name == "iso_two_level":
        from workloads.fields import Isothermal
        return (H.two_level(), Isothermal(SmoothField(1112)),
                "two-level 128^3 root + 512 refined patches, isothermal hydro (c_s = 1), smooth field")
    if name == "lowbeta":
        from workloads.fields import low_beta
        return H.two_level(), low_beta(5), "two-level 128^3 root + 512 refined patches, low beta (1e-3), 1% density noise"
    spec, centre, _ = H.deep_blast_target()
    return spec, Blast(centre), "deep 8-level hierarchy (64^3 root, ~40M cells), off-centre blast"


def _patch_fields(h, spec, pid, gamma=5.0 / 3.0):
    """Float64 interior arrays of rho, mx, my, mz, E, p and the three face fields (interior closures) of one patch."""
    import numpy as np
    G = 4
    _, lo, hi = spec.patches[pid]
    cells, faces = h.download(pid)
    n = [hi[a] - lo[a] for a in range(3)]
    sl = (slice(G, G + n[2]), slice(G, G + n[1]), slice(G, G + n[0]))
    c = [cells[m][sl].astype(np.float64) for m in range(5)]
    bc = []
    fs = []
    for d in range(3):
        f = faces[d].astype(np.float64)
        up = [slice(G, G + n[2]), slice(G, G + n[1]), slice(G, G + n[0])]
        up[2 - d] = slice(G + 1, G + n[d] + 1)
        bc.append(0.5 * (f[sl] + f[tuple(up)]))
        cl = [slice(G, G + n[2]), slice(G, G + n[1]), slice(G, G + n[0])]
        cl[2 - d] = slice(G, G + n[d] + 1)
        fs.append(f[tuple(cl)])
    pr = (gamma - 1.0) * (c[4] - 0.5 * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0]
                          - 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2))
    return c + [pr] + fs


def _interior_fields(h, spec, gamma=5.0 / 3.0):
    """Per patch: the arrays of _patch_fields."""
    return [_patch_fields(h, spec, pid, gamma) for pid in range(len(spec.patches))]


def lowbeta_report(spec, field, steps, torch):
    """Per-field relative L1 of FP32 with FP64 pressure recovery and of plain FP32 against the FP64 path (the
    FP64 GPU path, itself held to 1e-12 of the oracle), after each of `steps` root steps taken with the FP64
    path's time steps, and the conservation drift |sum U(t) - sum U(0)| / |sum U(0)| of each precision."""
    import numpy as np
    from paper_1112_1710_amd import FP32, FP32_MIXED, FP64, GRAPH, Hierarchy
    names = ("rho", "mx", "my", "mz", "E", "p", "bx", "by", "bz")

    class Rounded:
        """The field with every value rounded to float32: the FP32 runs' exact input, in float64."""

        def patch(self, level, root_n, lo, hi):
            st = field.patch(level, root_n, lo, hi)
            st.cells = st.cells.astype(np.float32).astype(np.float64)
            st.faces = [f.astype(np.float32).astype(np.float64) for f in st.faces]
            return st

    hs = {}
    for key, prec, fld in (("fp64", FP64, Rounded()), ("fp64_unrounded", FP64, field),
                           ("fp32_mixed", FP32_MIXED, field), ("fp32", FP32, field)):
        h = Hierarchy(spec, prec)
        h.set_field(fld)
        hs[key] = h
    tot0 = {k: sum(h.conservation()) for k, h in hs.items()}
    pairs = (("fp32_mixed", "fp64"), ("fp32", "fp64"), ("fp32_mixed", "fp64_unrounded"), ("fp64", "fp64_unrounded"))
    rel = {f"{a}_vs_{b}": {n: [] for n in names} for a, b in pairs}
    drift = {k: [] for k in hs}
    for _ in range(steps):
        dt = hs["fp64"].step(GRAPH)
        for k in ("fp64_unrounded", "fp32_mixed", "fp32"):
            hs[k].step(GRAPH, dt)
        fields = {k: _interior_fields(h, spec) for k, h in hs.items()}
        for a, b in pairs:
            got, ref = fields[a], fields[b]
            for i, n in enumerate(names):
                num = sum(float(np.sum(np.abs(g[i] - r[i]))) for g, r in zip(got, ref))
                den = sum(float(np.sum(np.abs(r[i]))) for r in ref)
                rel[f"{a}_vs_{b}"][n].append(num / den)
        del fields
        for k, h in hs.items():
            t = sum(h.conservation())
            d = [float(abs(t[q] - tot0[k][q])) for q in range(5)]
            # the momentum totals start near zero: their drift is reported in absolute terms only
            drift[k].append({"abs": d, "rel_mass": d[0] / abs(tot0[k][0]), "rel_energy": d[4] / abs(tot0[k][4])})
    for h in hs.values():
        del h
    hs.clear()
    torch.cuda.empty_cache()
    return {"steps": steps,
            "reference": "fp64 GPU path from the float32-rounded input (fp64) or from the exact input "
                         "(fp64_unrounded); the fp64 path is held to 1e-12 of the oracle",
            "rel_l1": rel,
            "conservation_drift": {k: {"per_step": v, "order": ["mass", "mx", "my", "mz", "energy"]}
                                   for k, v in drift.items()}}


def run_steps(h, mode, n):
    """`n` consecutive root steps: one hier_steps call (no host synchronisation between the steps)
    where the schedule supports it, else one synchronising hier_step per step."""
    from paper_1112_1710_amd import BATCHED, GRAPH, PLAIN
    if mode in (PLAIN, BATCHED, GRAPH):
        h.steps(n, mode)
    else:
        for _ in range(n):
            h.step(mode)


def timed_steps(h, mode, steps, warmup, torch):
    """Mean wall time of one root step over `steps` consecutive steps after `warmup` untimed ones."""
    run_steps(h, mode, warmup)
    torch.cuda.synchronize()
    h.timing(True)
    t0 = time.perf_counter()
    run_steps(h, mode, steps)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    h.timing(False)
    return total / steps, h.timing_read()


def time_regrid(h, eps, torch, min_side=4, efficiency=0.7):
    """Wall time of one regrid of the finest level: GPU flags, host buffer/nesting/clustering, the new
    hierarchy's host bookkeeping (finalize) and arenas, and its GPU initialisation from the old one."""
    import time
    from paper_1112_1710_amd.binding import Hierarchy
    from paper_1112_1710_amd.regrid import Spec
    top = h.levels - 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flags = h.flag_array(top - 1, eps)
    t1 = time.perf_counter()
    boxes = h.boxes_from_flags(top - 1, flags, min_side, efficiency)
    t2 = time.perf_counter()
    spec = Spec(root_n=tuple(h.spec.root_n),
                patches=[p for p in h.spec.patches if p[0] < top] + [(top, lo, hi) for lo, hi in boxes])
    h2 = Hierarchy(spec, h.precision, device=h.device)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    h2.init_from(h, top)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    old = sum(1 for p in h.spec.patches if p[0] == top)
    rep = {"eps": eps, "flagged_cells": int(flags.sum()), "patches_before": old, "patches_after": len(boxes),
           "cells_after": spec.cells(top), "flag_ms": round((t1 - t0) * 1e3, 2),
           "cluster_ms": round((t2 - t1) * 1e3, 2),
           "build_ms": round((t3 - t2) * 1e3, 2), "init_ms": round((t4 - t3) * 1e3, 2),
           "total_ms": round((t4 - t0) * 1e3, 2)}
    del h2
    torch.cuda.empty_cache()
    return rep


def time_regrid_levels(h, eps, from_level, torch, min_side=4, efficiency=0.7):
    """Wall time of one regrid of every level from `from_level` up, coarse to fine (per level: GPU
    flags of the new level below, host clustering, the level's hierarchy built and filled)."""
    import time
    from paper_1112_1710_amd.regrid import regrid_levels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        h2 = regrid_levels(h, eps, min_side, efficiency, from_level=from_level)
    except ValueError as e:  # nothing flagged below the first regridded level
        return {"eps": eps, "from_level": from_level, "error": str(e)}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = {}
    for lv, _, _ in h.spec.patches:
        per.setdefault(lv, [0, 0])[0] += 1
    for lv, _, _ in h2.spec.patches:
        per.setdefault(lv, [0, 0])[1] += 1
    rep = {"eps": eps, "from_level": from_level, "levels_before": h.levels, "levels_after": h2.levels,
           "patches_per_level_before_after": {str(k): v for k, v in sorted(per.items())},
           "cells_after": h2.spec.cells(), "total_ms": round((t1 - t0) * 1e3, 2)}
    del h2
    torch.cuda.empty_cache()
    return rep


def timed_evolve(h, mode, steps, every, eps, from_level, torch):
    """Wall time of `steps` root steps with regridding after every `every` of them (inside the timed
    loop), the zone-updates actually advanced (each step on the hierarchy it ran on) and the time of
    the regrids alone."""
    from paper_1112_1710_amd.regrid import regrid_levels
    torch.cuda.synchronize()
    zu = 0
    regrid_s = 0.0
    nreg = 0
    t0 = time.perf_counter()
    for k in range(steps):
        h.step(mode)
        zu += h.spec.zone_updates_per_root_step()
        if (k + 1) % every == 0:
            t1 = time.perf_counter()
            lv = h.levels - 1 if from_level is None else from_level
            try:
                h = regrid_levels(h, eps, from_level=lv)
                nreg += 1
            except ValueError:
                pass
            torch.cuda.synchronize()
            regrid_s += time.perf_counter() - t1
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return {"steps": steps, "every": every, "eps": eps, "from_level": from_level, "regrids": nreg,
            "value": round(zu / total, 1), "unit": "zone-updates/s", "seconds": round(total, 3),
            "regrid_seconds": round(regrid_s, 3), "patches_after": len(h.spec.patches)}


def primhalf_flops_per_step(h, spec, fused_levels):
    """Algorithmic flops of the fused first stages per root step: the update box of every patch of a fused
    level at each substep, grown by 2 (primitives) and by 1 (half-step faces, Hancock increments)."""
    G = 4
    tot = 0.0
    for pid, (lv, lo, hi) in enumerate(spec.patches):
        if lv not in fused_levels:
            continue
        subs = (0,) if lv == 0 else (0, 1)
        reps = 1 if lv == 0 else 2 ** (lv - 1)
        for s in subs:
            if lv == 0:
                blo, bhi = (G, G, G), tuple(G + hi[a] - lo[a] for a in range(3))
            else:
                blo, bhi = h.update_box(pid, s)
            v1 = v2 = 1
            for a in range(3):
                v1 *= bhi[a] - blo[a] + 2
                v2 *= bhi[a] - blo[a] + 4
            tot += reps * (PRIMHALF_FLOPS["grown2"] * v2 + PRIMHALF_FLOPS["grown1"] * v1)
    return tot


def extended_overhead(h, spec):
    """Cells advanced per root step (every patch's update region at each of its substeps, extended ghost
    layers included) over the zone-updates counted (interior cells only)."""
    done = 0
    for pid, (lv, lo, hi) in enumerate(spec.patches):
        subs = (0,) if lv == 0 else (0, 1)
        for s in subs:
            blo, bhi = h.update_box(pid, s)
            vol = 1
            for a in range(3):
                vol *= bhi[a] - blo[a]
            done += vol * (2 ** lv // len(subs))
    return done / spec.zone_updates_per_root_step()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_patch_task(task):
    """One sampled patch advanced by the oracle: (interior zone-updates, seconds)."""
    from oracle import amr, hydro, mhd
    name, lv, lo, hi = task
    spec, field, _ = workload(name)
    physics, cs = WORKLOAD_PHYSICS.get(name, ("mhd", 1.0))
    root = tuple(int(x) for x in spec.root_n)
    st = field.patch(lv, root, tuple(lo), tuple(hi))
    n = [hi[a] - lo[a] for a in range(3)]
    G = 4
    region = amr.update_box((G,) * 3, tuple(G + x for x in n), lv, 0)
    dx = [1.0 / (root[a] * 2 ** lv) for a in range(3)]
    box = ((G,) * 3, tuple(G + x for x in n))
    if physics == "isothermal":
        dt = 0.4 / hydro.max_signal(st.cells, dx, box, cs)
        t0 = time.perf_counter()
        hydro.advance(st.cells, st.faces, dx, dt, region, cs)
    else:
        dt = 0.4 / mhd.max_signal(st.cells, st.faces, dx, box, 5.0 / 3.0)
        t0 = time.perf_counter()
        mhd.advance(st.cells, st.faces, dx, dt, region, 5.0 / 3.0)
    return n[0] * n[1] * n[2], time.perf_counter() - t0


def cpu_baseline(name, npatch):
    """The oracle, as it stands, on a bounded sample of the benchmarked workload: one substep advance
    (the extended first-substep region on refined levels) of seeded patches drawn from every level, with
    the workload's own initial state and ghost data from the field generator.  Timed on one core, then on
    every usable host core through a process pool (forked before the GPU is touched)."""
    import multiprocessing as mp

    import numpy as np
    spec, _, _ = workload(name)
    rng = np.random.default_rng(1710)
    by_level = {}
    for lv, lo, hi in spec.patches:
        by_level.setdefault(lv, []).append((lv, lo, hi))
    levels = sorted(by_level)
    picks = []
    while len(picks) < npatch and any(by_level.values()):
        for lv in levels:
            if by_level[lv] and len(picks) < npatch:
                picks.append(by_level[lv].pop(int(rng.integers(len(by_level[lv])))))
    tasks = [(name, lv, lo, hi) for lv, lo, hi in picks]
    zu1 = sec1 = 0.0
    for t in tasks:
        z, s = _oracle_patch_task(t)
        zu1 += z
        sec1 += s
    cores = max(1, min(os.cpu_count() or 1, 16))
    pool_tasks = (tasks * (2 * cores // max(len(tasks), 1) + 1))[:2 * cores]
    with mp.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_patch_task, pool_tasks, chunksize=1)
        wall = time.perf_counter() - t0
    zup = sum(r[0] for r in res)
    sample = (f"one substep advance of {len(tasks)} seeded patches drawn from every level of the benchmarked workload "
              f"({int(zu1)} interior zone-updates), initial state and ghosts from the field generator, NumPy float64; "
              f"all cores: {len(pool_tasks)} such patch advances over a process pool; CPU: {_cpu_model()}")
    return {"value": round(zup / wall, 1), "unit": "zone-updates/s", "cores": cores, "kind": "oracle",
            "sample": sample, "single_core": {"value": round(zu1 / sec1, 1), "cores": 1, "seconds": round(sec1, 2)},
            "all_cores_seconds": round(wall, 2)}


def precision_report(spec, h32, hmix, mode, torch, physics="mhd", cs=1.0):
    """Per-field relative L1 after one root step of FP32 and of FP32 with targeted FP64 against the FP64 path
    (itself held to 1e-12 of the oracle), all three started from the FP32 run's current state with the
    FP64 path's time step; components whose vector starts in a plane (b_z of the blast) are also given
    against their vector's L1 norm."""
    import numpy as np
    from paper_1112_1710_amd import FP64, Hierarchy
    h64 = Hierarchy(spec, FP64, physics=physics, cs=cs)
    h32.synchronize()
    for pid in range(len(spec.patches)):
        cells, faces = h32.download(pid)
        h64.upload(pid, cells, faces)
        hmix.upload(pid, cells, faces)
    h64.synchronize()
    hmix.synchronize()
    dt = h64.step(mode)
    h32.step(mode, dt)
    hmix.step(mode, dt)
    names = ("rho", "mx", "my", "mz", "E", "p", "bx", "by", "bz")
    num = {"fp32": np.zeros(9), "fp32_mixed": np.zeros(9)}
    den = np.zeros(9)
    for pid in range(len(spec.patches)):
        ref = _patch_fields(h64, spec, pid)
        for key, h in (("fp32", h32), ("fp32_mixed", hmix)):
            got = _patch_fields(h, spec, pid)
            for i in range(9):
                num[key][i] += float(np.sum(np.abs(got[i] - ref[i])))
        for i in range(9):
            den[i] += float(np.sum(np.abs(ref[i])))
    gden = den.copy()
    for group in ((1, 2, 3), (6, 7, 8)):
        tot = sum(den[q] for q in group)
        for q in group:
            gden[q] = max(gden[q], tot)
    out = {"reference": "FP64 GPU path (held to 1e-12 rel-L1 of the oracle), one root step from the FP32 run's "
                        "state after the timed steps, same dt", "dt": dt}
    for key in num:
        out[key] = {n: float(f"{v:.3g}") for n, v in zip(names, num[key] / np.maximum(den, 1e-300))}
        out[key + "_vector_scaled"] = {n: float(f"{v:.3g}") for n, v in zip(names, num[key] / np.maximum(gden, 1e-300))}
    del h64
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.mode == "layered":
        args.staged = True  # the layered schedule runs the staged kernels (device-side nodes)
    if args.precision is None:
        args.precision = "fp32_mixed" if args.workload == "lowbeta" else "fp32"
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.stderr.write("bench.py measures one GPU only: the library has no multi-GPU path "
                         "(run with --gpus 1).\n")
        sys.exit(2)
    # the oracle's host timing first: its process pool forks before anything touches the GPU
    cpu = None if args.skip_cpu else cpu_baseline(args.workload, args.cpu_patches)
    import torch

    from paper_1112_1710_amd import (BATCHED, CONCURRENT, FP32, FP32_MIXED, FP64, GRAPH, LAYERED, PERSISTENT, PLAIN,
                                     Hierarchy)
    from paper_1112_1710_amd.binding import TUNE_FUSED, TUNE_FUSED_EU, TUNE_PAIR
    prec = {"fp32": FP32, "fp32_mixed": FP32_MIXED, "fp64": FP64}[args.precision]
    mode = {"plain": PLAIN, "batched": BATCHED, "graph": GRAPH, "persistent": PERSISTENT,
            "concurrent": CONCURRENT, "layered": LAYERED}[args.mode]
    spec, field, desc = workload(args.workload)
    zu = spec.zone_updates_per_root_step()

    physics, cs = WORKLOAD_PHYSICS.get(args.workload, ("mhd", 1.0))

    def prepared(precision, spec, field, physics=physics, cs=cs):
        """Hierarchy with the initial state uploaded and (unless disabled) autotuned kernels and tiles."""
        hh = Hierarchy(spec, precision, ghosts=args.ghosts, physics=physics, cs=cs)
        hh.set_field(field)
        t_first = t_eu = None
        if args.pair:
            hh.tune_set(TUNE_PAIR, 1)
        if args.staged:
            hh.tune_set(TUNE_FUSED, 0)
            hh.tune_set(TUNE_FUSED_EU, 0)
        elif not args.no_autotune:
            from paper_1112_1710_amd.autotune import autotune
            chosen = autotune(hh)
            t_first = {str(k): v[1] for k, v in chosen.items() if isinstance(k, int)}
            t_eu = {str(k[1]): v[1] for k, v in chosen.items() if not isinstance(k, int) and k[0] == "eu"}
            hh.flux_forms = {str(k[1]): v[1] for k, v in chosen.items() if not isinstance(k, int) and k[0] == "flux"}
        return hh, t_first, t_eu

    h, tiles, last = prepared(prec, spec, field)
    sec, timing = timed_steps(h, mode, args.steps, args.warmup, torch)
    value = zu / sec
    work = h.step_work()
    if mode in (GRAPH, PERSISTENT, CONCURRENT, LAYERED):
        # kernels inside a replayed graph or the persistent kernel are not bracketed by events: take the per-kernel
        # launch times from an instrumented batched pass of further consecutive steps
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
        fused_levels = {int(k) for k, v in (tiles or {}).items() if v != "staged"}
        meas = measured_traffic(args.workload, args.precision, dom, fused_levels) if args.ghosts == "extended" else None
        traffic = None
        if meas is not None:
            traffic = round(meas["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9, 1)
        hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
               "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": int(bytes_per_launch),
               "traffic_bytes_per_launch": None if traffic is None else int(meas["bytes_per_launch"])}
        # the flop prices are the MHD scheme's; the isothermal workload's kernels are reported against HBM
        if physics == "mhd" and (dom in ALU_BOUND or (dom == "primhalf" and fused_levels)):
            if dom == "primhalf":
                flops_per_launch = primhalf_flops_per_step(h, spec, fused_levels) / max(launches_per_step, 1)
            else:
                flops_per_launch = units_per_step * ALU_BOUND[dom] / max(launches_per_step, 1)
            tf = flops_per_launch / (avg_ms * 1e-3) / 1e12
            issue = MEASURED_VALU_ISSUE.get((args.workload, args.precision, dom)) if args.ghosts == "extended" else None
            issue = issue["frac"] if issue is not None and issue["sources"] == sources_hash() else None
            roof = {"bound": "alu", "achieved": round(tf, 2), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / VALU_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": dom,
                    "valu_issue_frac": issue,
                    "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": int(flops_per_launch),
                    "hbm": {k: hbm[k] for k in ("achieved", "peak", "unit", "frac", "bytes_per_launch")}}
        else:
            roof = hbm
    per_class = {k: round(v[0] / args.steps, 4) for k, v in timing.items() if v[1]}
    # the whole step against HBM: algorithmic bytes of every priced class that ran, over the step time (a lower
    # bound: restriction, corrections, sync, prolongation and CFL are not priced)
    priced = sorted(k for k in work if k in WORDS_PER_UNIT and work[k][1] > 0)
    step_bytes = sum(work[k][0] * WORDS_PER_UNIT[k] * word for k in priced)
    step_hbm = {"bytes_per_step": int(step_bytes), "achieved": round(step_bytes / sec / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(step_bytes / sec / 1e9 / HBM_PEAK_GBS, 4), "classes": priced}
    regrid_report = None
    if args.regrid_eps is not None and spec.levels() > 1 and args.regrid_every:
        regrid_report = timed_evolve(h, mode, args.steps, args.regrid_every, args.regrid_eps, args.regrid_from, torch)
    elif args.regrid_eps is not None and spec.levels() > 1:
        if args.regrid_from is None:
            regrid_report = time_regrid(h, args.regrid_eps, torch)
        else:
            regrid_report = time_regrid_levels(h, args.regrid_eps, args.regrid_from, torch)
    overhead = extended_overhead(h, spec)
    mixed = None
    if not args.skip_precision and prec == FP32 and args.workload != "lowbeta":
        hm, _, _ = prepared(FP32_MIXED, spec, field)
        msec, _ = timed_steps(hm, mode, max(args.steps // 2, 1), 1, torch)
        mixed = {"value": round(zu / msec, 1), "ms_per_step": round(msec * 1e3, 4),
                 "flux_stage": getattr(hm, "flux_forms", None),
                 "rel_l1_per_step": precision_report(spec, h, hm, mode, torch, physics, cs)}
        del hm
        torch.cuda.empty_cache()
    flux_forms = getattr(h, "flux_forms", None)
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
                   "schedule": args.mode, "ghosts": args.ghosts, "physics": physics,
                   "steps_from": "consecutive steps from the seeded initial state",
                   "first_stages": "staged" if args.staged or tiles is None else tiles,
                   "edge_update_stages": "staged" if args.staged or last is None else last,
                   "extended_ghost_overhead": round(overhead, 4),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "step_hbm": step_hbm,
        "kernel_ms_per_step": per_class,
    }
    if flux_forms:
        out["config"]["flux_stage"] = flux_forms
    if regrid_report is not None:
        out["regrid"] = regrid_report
    if mixed is not None:
        out["fp32_mixed"] = mixed
        out["rel_l1_per_step"] = mixed["rel_l1_per_step"]["fp32"]

    if not args.skip_plain:
        hp = Hierarchy(spec, FP64, ghosts=args.ghosts, physics=physics, cs=cs)
        hp.set_field(field)
        psec, _ = timed_steps(hp, PLAIN, args.plain_steps, 1, torch)
        out["fp64_plain_value"] = round(zu / psec, 1)
        out["speedup_vs_fp64_plain"] = round(value / (zu / psec), 3)
        del hp
        torch.cuda.empty_cache()

    if args.workload == "deep" and not args.skip_secondary:
        s2, f2, d2 = workload("two_level")
        zu2 = s2.zone_updates_per_root_step()
        h2, _, _ = prepared(prec, s2, f2, "mhd", 1.0)
        sec2, _ = timed_steps(h2, mode, args.secondary_steps, args.warmup, torch)
        out["secondary"] = {"workload": d2, "value": round(zu2 / sec2, 1), "unit": "zone-updates/s",
                            "ms_per_step": round(sec2 * 1e3, 4), "steps": args.secondary_steps,
                            "precision": args.precision, "schedule": args.mode}
        del h2
        torch.cuda.empty_cache()

    if args.workload == "lowbeta":
        out["lowbeta_report"] = lowbeta_report(spec, field, args.report_steps, torch)

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
