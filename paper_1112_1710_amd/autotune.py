"""Autotuner for the two fusable groups of advance stages: the first three
(primitives, half-step face field, Hancock predictor) and the last two (edge
EMFs, update).

For every level of a bound hierarchy and each group the candidates are the
staged kernels and the fused LDS-tiled kernel with each tile shape of the
library's table that fits the LDS limit at the hierarchy's precision (for the
last group also the staged kernels with the update's next-state stores marked
non-temporal, which helps on some levels and hurts on others).  Each is
timed on the level's own patches (``hier_tune_time``: the first group, writing
only intermediate scratch, summed over the level's substeps;
``hier_tune_time_eu``: the last group on substep 0, writing only the level's
next-state buffer and EMF registers, which hold nothing between root steps);
the fastest is selected with ``hier_tune_set``.  All candidates give
bit-identical results.  Call it between root steps.

Choices are cached in a JSON file keyed by GPU architecture, precision and a
size class of the level (patch count and the median side of the patches'
primitive regions, each rounded to a power of two), so a later hierarchy of the
same shape class skips the search.  The cache lives at ``$AMRX_TUNE_CACHE`` if
set, else ``~/.cache/amrx/tune.json``.
"""
import json
import os

from .binding import (FP32_MIXED, TUNE_FLUX_SPLIT, TUNE_FUSED, TUNE_FUSED_EU, TUNE_TILE, TUNE_TILE_EU, TUNE_UPDATE_NT,
                      tile_table)

G = 4


def _pow2(x):
    p = 1
    while p < x:
        p <<= 1
    return p


def size_class(spec, level):
    """Patch count and median primitive-region side of `level`, each rounded up to a power of two."""
    sides = []
    count = 0
    for (lv, lo, hi) in spec.patches:
        if lv != level:
            continue
        count += 1
        grow = 0 if level == 0 else 2
        for a in range(3):
            sides.append(hi[a] - lo[a] + 2 * grow + 4)
    sides.sort()
    med = sides[len(sides) // 2] if sides else 0
    return f"n{_pow2(count)}-s{_pow2(med)}"


def arch_name(device=0):
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def cache_path():
    return os.environ.get("AMRX_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "amrx", "tune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a repeated search


STAGED = -1
STAGED_NT = -2   # edge/update group only: the staged kernels, the update storing non-temporally


def _apply(h, level, choice, group="a"):
    fused, tile = (TUNE_FUSED, TUNE_TILE) if group == "a" else (TUNE_FUSED_EU, TUNE_TILE_EU)
    if group != "a":
        h.tune_set(TUNE_UPDATE_NT, 1 if choice == STAGED_NT else 0, level)
    if choice in (STAGED, STAGED_NT):
        h.tune_set(fused, 0, level)
    else:
        h.tune_set(fused, 1, level)
        h.tune_set(tile, choice, level)


def _shape(table, choice):
    if choice == STAGED:
        return "staged"
    if choice == STAGED_NT:
        return "staged-nt"
    return "x".join(str(x) for x in table[choice][:3])


def autotune(h, reps=5, use_cache=True, path=None, groups=("a", "eu", "flux")):
    """Select staged or fused (and the tile) for every level of the bound hierarchy `h` and each group.

    Returns {level: (choice, shape, ms, source)} for the first three stages, and, when "eu" is in `groups`,
    the same for the edge/update stages under the key ("eu", level): choice -1 = staged, -2 = staged with the
    update storing the next state non-temporally (edge/update only), else the tile index; shape "staged",
    "staged-nt" or "TXxTYxTZ"; ms the measured time; source "search" or "cache".  In FP32_MIXED, "flux"
    also times the flux stage's two-launch and one-launch forms per level under ("flux", level), choice 1 or
    0; that choice depends on how many faces of the current state are low-beta, not on the level's shape,
    so it is never cached.
    """
    path = path or cache_path()
    cache = _load(path) if use_cache else {}
    table = tile_table(h.precision)
    candidates = {"a": [STAGED] + [t for t, (_, _, _, lds) in enumerate(table) if lds > 0],
                  "eu": [STAGED, STAGED_NT] + list(range(len(table)))}
    arch = arch_name()
    levels = 1 + max(p[0] for p in h.spec.patches)
    out = {}
    changed = False
    if "flux" in groups and h.precision == FP32_MIXED:
        for level in range(levels):
            times = {}
            for split in (1, 0):
                h.tune_time_flux(level, split, 1)  # warm-up
                times[split] = h.tune_time_flux(level, split, reps)
            best = min(times, key=times.get)
            h.tune_set(TUNE_FLUX_SPLIT, best, level)
            out[("flux", level)] = (best, "two launches" if best else "one launch", times[best], "search")
    for group in groups:
        if group == "flux":
            continue
        for level in range(levels):
            tag = "" if group == "a" else "|eu2"
            key = f"{arch}|p{h.precision}|l{min(level, 1)}|{size_class(h.spec, level)}{tag}"
            okey = level if group == "a" else ("eu", level)
            cands = candidates[group]
            hit = cache.get(key)
            if hit is not None and hit.get("choice") in cands and hit.get("shape") == _shape(table, hit["choice"]):
                _apply(h, level, hit["choice"], group)
                out[okey] = (hit["choice"], hit["shape"], hit.get("ms"), "cache")
                continue
            times = {}
            for t in cands:
                if group == "a":
                    nsub = 1 if level == 0 else 2
                    h.tune_time(level, 0, t, 1)  # warm-up
                    times[t] = sum(h.tune_time(level, s, t, reps) for s in range(nsub))
                else:
                    h.tune_time_eu(level, t, 1)  # warm-up
                    times[t] = h.tune_time_eu(level, t, reps)
            best = min(times, key=times.get)
            _apply(h, level, best, group)
            out[okey] = (best, _shape(table, best), times[best], "search")
            cache[key] = {"choice": best, "shape": _shape(table, best), "ms": times[best],
                          "candidates": {_shape(table, t): times[t] for t in times}}
            changed = True
    if use_cache and changed:
        _store(path, cache)
    return out
