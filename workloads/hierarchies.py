"""Seeded static patch hierarchies (ratio 2) used as workloads.

A hierarchy is a list of ``(level, lo, hi)`` boxes, ``lo``/``hi`` being
integer 3-vectors in the level's own index space (half-open [lo, hi)).  All
boxes obey the nesting rule the library enforces: on levels >= 1 both corners
are even, and the box lies inside one parent patch's interior shrunk by one
parent cell on every side; boxes of one level are disjoint.  The generators
are pure integer/geometry code and hold none of the solver's arithmetic.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class HierarchySpec:
    root_n: tuple
    patches: list = field(default_factory=list)  # (level, lo(3), hi(3))
    name: str = ""

    def levels(self):
        return 1 + max(p[0] for p in self.patches)

    def cells(self, level=None):
        tot = 0
        for lv, lo, hi in self.patches:
            if level is None or lv == level:
                tot += int(np.prod(np.asarray(hi) - np.asarray(lo)))
        return tot

    def zone_updates_per_root_step(self):
        """Interior cells times substeps (level l takes 2**l steps per root step)."""
        return sum(int(np.prod(np.asarray(hi) - np.asarray(lo))) * 2 ** lv for lv, lo, hi in self.patches)


def single_patch(n, name=""):
    n = tuple(int(x) for x in (n if hasattr(n, '__len__') else (n, n, n)))
    return HierarchySpec(root_n=n, patches=[(0, (0, 0, 0), n)], name=name or f"uniform {n[0]}^3")


def _box_dist2(lo, hi, c):
    """Squared distance from point c to box [lo, hi) (same units)."""
    d2 = 0.0
    for a in range(3):
        if c[a] < lo[a]:
            d2 += (lo[a] - c[a]) ** 2
        elif c[a] > hi[a]:
            d2 += (c[a] - hi[a]) ** 2
    return d2


def kd_ball_patches(rng, n_fine, centre, radius, count, lo_lim, hi_lim, smin=8, smax=64):
    """Exactly ``count`` disjoint boxes with sides in [smin, smax] (even), each meeting the ball.

    Seeded k-d bisection of the ball's bounding box (clipped to [lo_lim, hi_lim)):
    the largest ball-meeting leaf is cut along its longest axis at a random even
    position leaving >= smin on both sides, until ``count`` leaves meet the ball.
    """
    lo = [max(lo_lim, int(math.floor((centre[a] - radius) / 2)) * 2) for a in range(3)]
    hi = [min(hi_lim, int(math.ceil((centre[a] + radius) / 2)) * 2) for a in range(3)]
    r2 = radius * radius

    def meets(b):
        return _box_dist2(b[0], b[1], centre) < r2

    def ext(b):
        return [b[1][a] - b[0][a] for a in range(3)]

    def vol(b):
        e = ext(b)
        return e[0] * e[1] * e[2]

    # the leaves, the number of ball-meeting leaves and of those wider than smax, and a heap
    # of the ball-meeting leaves that can still be cut, largest volume first
    leaves = set()
    counts = [0, 0]
    heap = []

    def add(b):
        leaves.add(b)
        if meets(b):
            w = max(ext(b))
            counts[0] += 1
            counts[1] += w > smax
            if w >= 2 * smin:
                heapq.heappush(heap, (-vol(b), b))

    add((tuple(lo), tuple(hi)))
    while counts[0] < count or counts[1]:
        if not heap:
            raise ValueError("cannot reach the requested patch count")
        _, b = heapq.heappop(heap)
        e = ext(b)
        leaves.remove(b)
        counts[0] -= 1
        counts[1] -= max(e) > smax
        ax = e.index(max(e))  # first longest axis
        ncut = (e[ax] - 2 * smin) // 2 + 1
        cut = b[0][ax] + smin + 2 * int(rng.integers(0, ncut))
        l1 = list(b[1]); l1[ax] = cut
        h2 = list(b[0]); h2[ax] = cut
        add((b[0], tuple(l1)))
        add((tuple(h2), b[1]))
    hits = sorted([b for b in leaves if meets(b)])
    if len(hits) > count:
        # drop the leaves farthest from the centre (deterministic)
        hits.sort(key=lambda b: (_box_dist2(b[0], b[1], centre), b))
        hits = sorted(hits[:count])
    return hits


def two_level(root=128, count=512, seed=2, radius_frac=0.35):
    """Root patch plus exactly ``count`` level-1 patches packed in a seeded ball."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nf = 2 * root
    margin = radius_frac * nf + 2
    centre = [float(rng.uniform(margin, nf - margin)) for _ in range(3)]
    boxes = kd_ball_patches(rng, nf, centre, radius_frac * nf, count, 2, nf - 2)
    spec = HierarchySpec(root_n=(root,) * 3, name=f"two-level {root}^3 + {len(boxes)} patches")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    for b in boxes:
        spec.patches.append((1, b[0], b[1]))
    return spec


def _tile_axis(rng, a, b, wmin, wmax):
    """Split [a, b) (even, length >= wmin) into even widths in [wmin, wmax]."""
    L = b - a
    if L <= wmax:
        return [(a, b)]
    cuts = [a]
    x = a
    while b - x > wmax:
        hi = min(wmax, b - x - wmin)
        w = wmin + 2 * int(rng.integers(0, (hi - wmin) // 2 + 1))
        x += w
        cuts.append(x)
    cuts.append(b)
    return list(zip(cuts[:-1], cuts[1:]))


def deep_blast(levels=8, root=64, seed=3, r1=0.3, q=0.7, wmin=8, wmax=48):
    """Deep hierarchy refining around a seeded blast centre (ball radius r1*q**(l-1) on level l)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = [float(rng.uniform(0.3, 0.7)) for _ in range(3)]
    spec = HierarchySpec(root_n=(root,) * 3, name=f"deep {levels}-level {root}^3 blast")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    parents = [((0, 0, 0), (root,) * 3)]
    for lv in range(1, levels):
        n_l = root * 2 ** lv
        r = r1 * q ** (lv - 1) * n_l
        c = [x * n_l for x in centre]
        kids = []
        for plo, phi in parents:
            ilo = [2 * plo[a] + 2 for a in range(3)]
            ihi = [2 * phi[a] - 2 for a in range(3)]
            if any(ihi[a] - ilo[a] < wmin for a in range(3)):
                continue
            tiles = [_tile_axis(rng, ilo[a], ihi[a], wmin, wmax) for a in range(3)]
            for tz in tiles[2]:
                for ty in tiles[1]:
                    for tx in tiles[0]:
                        lo = (tx[0], ty[0], tz[0])
                        hi = (tx[1], ty[1], tz[1])
                        if _box_dist2(lo, hi, c) < r * r:
                            kids.append((lo, hi))
        if not kids:
            break
        for lo, hi in kids:
            spec.patches.append((lv, lo, hi))
        parents = kids
    return spec, centre


def small_two_level(root=16):
    """Tiny hierarchy for tests: root plus three level-1 patches (two of them adjacent)."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"small two-level {root}^3")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    spec.patches.append((1, (4, 6, 6), (12, 14, 14)))
    spec.patches.append((1, (12, 6, 8), (18, 12, 14)))
    spec.patches.append((1, (20, 18, 4), (28, 26, 10)))
    return spec


def block_two_level(root=16, k=3, side=8, start=2, wide=2):
    """Root plus a k x k x k block of adjacent level-1 patches of `side` fine cells (the last
    layer along each axis `wide` cells wider), so that the block's inner patch sides are
    covered by siblings and its outer sides are not."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"block two-level {root}^3, {k}^3 patches")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    edges = [start + side * i for i in range(k + 1)]
    edges[-1] += wide
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                lo = (edges[kx], edges[ky], edges[kz])
                hi = (edges[kx + 1], edges[ky + 1], edges[kz + 1])
                spec.patches.append((1, lo, hi))
    return spec


def small_three_level(root=16):
    """Tiny hierarchy for tests: three levels with adjacent siblings and a grandchild."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"small three-level {root}^3")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    spec.patches.append((1, (4, 4, 4), (16, 16, 14)))
    spec.patches.append((1, (16, 4, 6), (26, 14, 14)))
    spec.patches.append((2, (12, 12, 12), (24, 22, 20)))
    spec.patches.append((2, (24, 12, 14), (30, 20, 22)))
    spec.patches.append((2, (36, 12, 14), (46, 22, 24)))
    return spec


def minimal_patches(root=8):
    """Edge cases of patch size: an 8^3 root (ghost layers half its width), refined patches of the
    minimum width R = 2 (a 2^3 cube and a 2 x 8 x 2 slab), a corner-touching and a face-sharing
    sibling, and a 2^3 grandchild."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"minimal patches {root}^3")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    spec.patches.append((1, (2, 2, 2), (4, 4, 4)))
    spec.patches.append((1, (4, 4, 4), (12, 12, 12)))
    spec.patches.append((1, (12, 4, 4), (14, 12, 6)))
    spec.patches.append((2, (10, 10, 10), (12, 12, 12)))
    return spec


def small_three_level_td(root=16):
    """Tiny three-level hierarchy whose level-2 patches keep their prolongation stencils inside
    data that is valid at the parent's new time (the parent's interior, or parent ghost cells a
    sibling of the parent holds): two adjacent level-1 patches, one grandchild deep inside the
    first and one next to their shared side."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"small three-level {root}^3 (time-derivative ghosts)")
    spec.patches.append((0, (0, 0, 0), (root,) * 3))
    spec.patches.append((1, (4, 4, 4), (16, 16, 16)))
    spec.patches.append((1, (16, 4, 4), (28, 16, 16)))
    spec.patches.append((2, (14, 14, 14), (26, 26, 26)))
    spec.patches.append((2, (34, 14, 14), (42, 22, 22)))
    return spec


def root_tiled(root=16, split=2):
    """Root level made of split^3 patches (exercises same-level periodic ghost exchange)."""
    spec = HierarchySpec(root_n=(root,) * 3, name=f"root {root}^3 tiled {split}^3")
    w = root // split
    for k in range(split):
        for j in range(split):
            for i in range(split):
                spec.patches.append((0, (i * w, j * w, k * w), ((i + 1) * w, (j + 1) * w, (k + 1) * w)))
    return spec


def deep_blast_target(target_cells=40_000_000, levels=8, root=64, seed=3, q=0.7, iters=14):
    """``deep_blast`` with r1 chosen by a fixed bisection so the total cell count is near the target."""
    lo, hi = 0.05, 0.3
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        spec, centre = deep_blast(levels, root, seed, r1=mid, q=q)
        if best is None or abs(spec.cells() - target_cells) < abs(best[0].cells() - target_cells):
            best = (spec, centre, mid)
        if spec.cells() > target_cells:
            hi = mid
        else:
            lo = mid
    return best
