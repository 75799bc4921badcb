"""Regridding: refinement flags, clustering into patches, and the initialisation of the new
patches from the old ones and their parent; of the finest level alone, or of every level from a
given one upward, coarse to fine.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed here
  * Sec. 2.2 (grid life cycle): after a level's grids are created they decide
    which of their cells to refine and lay down child grids covering them;
    new grids are initialised from the preceding grids of their level where
    those overlap them, and by prolongation from the parent elsewhere (the
    Overlap and Prolongate steps).
  * Sec. 2: every child grid has exactly one parent; grids of a level do not
    overlap.

Readings where the paper is silent (it names no refinement criterion and no
clustering method):
  * flag: an interior cell of a level is flagged when the density jump to one
    of its face neighbours inside the same patch exceeds eps times the smaller
    of the two densities, |rho_n - rho_c| > eps * min(rho_n, rho_c),
    evaluated in the state's own precision (float32 for the FP32 modes);
  * buffer: the flags are then grown by one cell in all 26 directions, inside
    the patch;
  * cells within one parent cell of the parent's interior boundary are not
    refined (the nesting rule: a child lies inside its parent's interior
    shrunk by one parent cell);
  * clustering per parent (Berger-Rigoutsos signature splitting): shrink the
    box to its flags; accept it when flagged / volume >= efficiency or when
    no side is at least 2 * min_side long; otherwise cut at the zero of a
    signature (sum of flags over the other two axes) nearest the box middle,
    over all axes whose cut leaves both parts at least min_side long (ties:
    nearer the middle, then the lower axis, then the lower position); without
    such a zero, at the largest sign change of the signature's second
    difference (strength |D[i+1] - D[i]|, cut between i and i+1; same limits
    and ties); without that either, in the middle of the longest splittable
    axis (lower axis on ties);
  * new patch = the coarse box times R;
  * initialisation: cells (faces) of a new patch's interior (closure) copy the
    old same-level patch whose interior (closure) holds them (no periodic
    images: patches of refined levels lie inside the domain, their parents'
    interiors shrunk by one cell); the remaining
    parent cells under the new interior are prolongated as in ghost filling,
    from the parent's current state, with the outer fine faces that old
    patches hold kept and the divergence-free interior closure applied;
  * several levels (Sec. 2.2 applied level after level): the new level l is
    clustered over the flags of the new level l - 1 (already initialised), and
    initialised from the old level l and the new level l - 1; a level without
    flags ends the hierarchy there (the old finer levels are dropped).
"""
from __future__ import annotations

import numpy as np

from . import amr

R = amr.R
G = amr.G


# ---------------------------------------------------------------------------------------------
# flags
# ---------------------------------------------------------------------------------------------
def flag_cells(rho, eps, dtype=np.float64):
    """Flags of a patch interior from its interior density rho[z, y, x] (before the buffer)."""
    r = np.asarray(rho, dtype=dtype)
    e = dtype(eps)
    f = np.zeros(r.shape, dtype=bool)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        a, b = r[tuple(lo)], r[tuple(hi)]
        jump = np.abs(a - b) > e * np.minimum(a, b)
        f[tuple(lo)] |= jump
        f[tuple(hi)] |= jump
    return f


def buffer_flags(f):
    """Grow the flags by one cell in all 26 directions, inside the array."""
    g = f.copy()
    nz, ny, nx = f.shape
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                src = f[max(0, -dz):nz - max(0, dz), max(0, -dy):ny - max(0, dy), max(0, -dx):nx - max(0, dx)]
                g[max(0, dz):nz - max(0, -dz), max(0, dy):ny - max(0, -dy), max(0, dx):nx - max(0, -dx)] |= src
    return g


# ---------------------------------------------------------------------------------------------
# clustering
# ---------------------------------------------------------------------------------------------
def _bbox(f, lo, hi):
    sub = f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    if not sub.any():
        return None
    out_lo, out_hi = [], []
    for a in range(3):
        other = tuple(b for b in range(3) if b != a)
        # array axes are (z, y, x): array axis of coordinate a is 2 - a
        s = sub.any(axis=tuple(2 - b for b in other))
        idx = np.nonzero(s)[0]
        out_lo.append(lo[a] + int(idx[0]))
        out_hi.append(lo[a] + int(idx[-1]) + 1)
    return out_lo, out_hi


def _signature(f, lo, hi, a):
    sub = f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    other = tuple(2 - b for b in range(3) if b != a)
    return sub.sum(axis=other).astype(np.int64)


def _choose_cut(f, lo, hi, min_side):
    """(axis, cut) in absolute coordinates, or None."""
    n = [hi[a] - lo[a] for a in range(3)]
    best = None  # (key, axis, cut)
    # zeros of a signature
    for a in range(3):
        if n[a] < 2 * min_side:
            continue
        s = _signature(f, lo, hi, a)
        for i in range(min_side, n[a] - min_side + 1):
            # a zero at local index i (cut before it or after it keeps one side flag-free:
            # the box was shrunk to its flags, so a zero lies strictly inside)
            if i < n[a] and s[i] == 0:
                key = (abs(2 * i - n[a]), a, i)
                if best is None or key < best[0]:
                    best = (key, a, lo[a] + i)
    if best is not None:
        return best[1], best[2]
    # largest inflection of the signature's second difference
    for a in range(3):
        if n[a] < 2 * min_side:
            continue
        s = _signature(f, lo, hi, a)
        d = np.zeros(n[a], dtype=np.int64)
        d[1:-1] = s[2:] - 2 * s[1:-1] + s[:-2]
        for i in range(1, n[a] - 2):
            cut = i + 1                      # between local cells i and i + 1
            if cut < min_side or n[a] - cut < min_side:
                continue
            if d[i] * d[i + 1] < 0:
                key = (-int(abs(d[i + 1] - d[i])), abs(2 * cut - n[a]), a, cut)
                if best is None or key < best[0]:
                    best = (key, a, lo[a] + cut)
    if best is not None:
        return best[1], best[2]
    # middle of the longest splittable axis
    axes = [a for a in range(3) if n[a] >= 2 * min_side]
    if not axes:
        return None
    a = max(axes, key=lambda b: (n[b], -b))
    return a, lo[a] + n[a] // 2


def cluster(f, min_side=4, efficiency=0.7):
    """Boxes ((lo), (hi)) in (x, y, z) array coordinates covering every flag of f[z, y, x]."""
    out = []
    stack = [([0, 0, 0], [f.shape[2], f.shape[1], f.shape[0]])]
    while stack:
        lo, hi = stack.pop()
        bb = _bbox(f, lo, hi)
        if bb is None:
            continue
        lo, hi = bb
        vol = int(np.prod([hi[a] - lo[a] for a in range(3)]))
        nflag = int(f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].sum())
        if nflag >= efficiency * vol:
            out.append((tuple(lo), tuple(hi)))
            continue
        c = _choose_cut(f, lo, hi, min_side)
        if c is None:
            out.append((tuple(lo), tuple(hi)))
            continue
        a, cut = c
        lhi = list(hi)
        lhi[a] = cut
        rlo = list(lo)
        rlo[a] = cut
        # depth-first, low part first (the stack pops the last pushed)
        stack.append((rlo, hi))
        stack.append((lo, lhi))
    return out


# ---------------------------------------------------------------------------------------------
# the new finest level
# ---------------------------------------------------------------------------------------------
def child_boxes(h, level, eps, dtype=np.float64, min_side=4, efficiency=0.7):
    """Level-(level+1) boxes laid over the flagged cells of every level-`level` patch of oracle hierarchy h."""
    boxes = []
    for m in h.level_patches(level):
        n = m.n
        rho = m.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]]
        f = buffer_flags(flag_cells(rho, eps, dtype))
        # nesting: no child within one parent cell of the parent's interior boundary
        f[:1] = False
        f[-1:] = False
        f[:, :1] = False
        f[:, -1:] = False
        f[:, :, :1] = False
        f[:, :, -1:] = False
        for lo, hi in cluster(f, min_side, efficiency):
            glo = tuple(R * (int(m.lo[a]) + lo[a]) for a in range(3))
            ghi = tuple(R * (int(m.lo[a]) + hi[a]) for a in range(3))
            boxes.append((glo, ghi))
    return boxes


def init_from(new, old, level):
    """Fill the interiors (closures) of the level-`level` patches of oracle hierarchy `new` from the
    level-`level` patches of `old` where they overlap, and by prolongation from `new`'s parents (whose
    state must already be set) elsewhere.  Patches of other levels are not touched."""
    for p in new.level_patches(level):
        p.cells = np.full((5,) + p.shape, np.nan)
        p.faces = [np.full(p.shape, np.nan) for _ in range(3)]
        own_c = np.zeros(p.shape, dtype=bool)
        own_f = [np.zeros(p.shape, dtype=bool) for _ in range(3)]
        po = p.origin()
        for q in old.level_patches(level):
            qo = q.origin()
            # cells: the intersection of the two interiors
            lo = np.maximum(p.lo, q.lo)
            hi = np.minimum(p.hi, q.hi)
            if np.all(hi > lo):
                ps = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
                qs = tuple(slice(int(lo[a] - qo[a]), int(hi[a] - qo[a])) for a in (2, 1, 0))
                p.cells[(slice(None),) + ps] = q.cells[(slice(None),) + qs]
                own_c[ps] = True
            # faces normal to d: the intersection of the two closures (one more entry along d)
            for d in range(3):
                flo = np.maximum(p.lo, q.lo)
                fhi = np.minimum(p.hi, q.hi).copy()
                fhi[d] += 1
                if np.all(fhi > flo):
                    ps = tuple(slice(int(flo[a] - po[a]), int(fhi[a] - po[a])) for a in (2, 1, 0))
                    qs = tuple(slice(int(flo[a] - qo[a]), int(fhi[a] - qo[a])) for a in (2, 1, 0))
                    p.faces[d][ps] = q.faces[d][qs]
                    own_f[d][ps] = True
        _prolong_interior(new, p, own_c, own_f)


def _prolong_interior(h, p, own_c, own_f):
    """Prolongate the parent cells under p's interior whose fine cells no old patch holds."""
    m = p.parent
    uc = m.cells
    bc = m.faces
    M, outer_idx, inner_idx = amr.Hierarchy.interior_face_map()
    mo = m.origin()
    po = p.origin()
    nc = p.n // R
    for cz in range(int(nc[2])):
        for cy in range(int(nc[1])):
            for cx in range(int(nc[0])):
                fx, fy, fz = G + R * cx, G + R * cy, G + R * cz   # fine padded index of the first fine cell
                if own_c[fz, fy, fx]:
                    continue
                cg = (p.lo // R) + np.array([cx, cy, cz])
                X, Y, Z = (int(v) for v in (cg - mo))
                u0 = uc[:, Z, Y, X]
                slopes = []
                for d in range(3):
                    e = [0, 0, 0]
                    e[d] = 1
                    up = uc[:, Z + e[2], Y + e[1], X + e[0]]
                    dn = uc[:, Z - e[2], Y - e[1], X - e[0]]
                    slopes.append(amr.Hierarchy._minmod(up - u0, u0 - dn))
                for oz in (0, 1):
                    for oy in (0, 1):
                        for ox in (0, 1):
                            p.cells[:, fz + oz, fy + oy, fx + ox] = u0 + 0.25 * (
                                (2 * ox - 1) * slopes[0] + (2 * oy - 1) * slopes[1] + (2 * oz - 1) * slopes[2])
                outer = np.zeros(24)
                write = np.zeros(24, dtype=bool)
                for d in range(3):
                    a1, a2 = [a for a in range(3) if a != d]
                    for side in (0, 2):
                        cidx = [X, Y, Z]
                        cidx[d] += side // 2
                        bcf = bc[d][cidx[2], cidx[1], cidx[0]]
                        sl = []
                        for a in (a1, a2):
                            up = list(cidx)
                            up[a] += 1
                            dn = list(cidx)
                            dn[a] -= 1
                            sl.append(amr.Hierarchy._minmod(bc[d][up[2], up[1], up[0]] - bcf,
                                                            bcf - bc[d][dn[2], dn[1], dn[0]]))
                        for t2 in (0, 1):
                            for t1 in (0, 1):
                                fidx = [fx, fy, fz]
                                fidx[d] += side // 2 * R
                                fidx[a1] += t1
                                fidx[a2] += t2
                                k = outer_idx[(d, side, t2, t1)]
                                if own_f[d][fidx[2], fidx[1], fidx[0]]:
                                    outer[k] = p.faces[d][fidx[2], fidx[1], fidx[0]]
                                else:
                                    outer[k] = bcf + 0.25 * ((2 * t1 - 1) * sl[0] + (2 * t2 - 1) * sl[1])
                                    write[k] = True
                inner = M @ outer
                for (d, side, t2, t1), k in outer_idx.items():
                    if write[k]:
                        a1, a2 = [a for a in range(3) if a != d]
                        fidx = [fx, fy, fz]
                        fidx[d] += side // 2 * R
                        fidx[a1] += t1
                        fidx[a2] += t2
                        p.faces[d][fidx[2], fidx[1], fidx[0]] = outer[k]
                for (d, t2, t1), k in inner_idx.items():
                    a1, a2 = [a for a in range(3) if a != d]
                    fidx = [fx, fy, fz]
                    fidx[d] += 1
                    fidx[a1] += t1
                    fidx[a2] += t2
                    p.faces[d][fidx[2], fidx[1], fidx[0]] = inner[k]
                amr.Hierarchy.positivity_fallback(p, fx, fy, fz, u0, h.gamma, h.physics == "isothermal")


def regrid_levels(old, eps, dtype=np.float64, min_side=4, efficiency=0.7, from_level=1):
    """A new oracle hierarchy: the levels of `old` below `from_level` unchanged, every level from
    `from_level` up to old's finest laid over the flags of the new level below it and initialised
    from old's patches of its own level and from its new parents.  Stops at the first level whose
    parents hold no flag (ValueError when that is `from_level` itself)."""
    top = old.nlevels - 1
    if not 1 <= from_level <= top:
        raise ValueError("from_level must name a refined level")
    cur = old
    for level in range(from_level, top + 1):
        boxes = child_boxes(cur, level - 1, eps, dtype, min_side, efficiency)
        if not boxes:
            if level == from_level:
                raise ValueError("no cell below the first regridded level is flagged")
            break
        new = amr.Hierarchy(old.root_n, gamma=old.gamma, cfl=old.cfl, ghosts=old.ghosts, physics=old.physics,
                            cs=old.cs)
        keep = [p for p in cur.patches if p.level < level]
        for p in keep:
            new.add(p.level, tuple(int(v) for v in p.lo), tuple(int(v) for v in p.hi))
        for lo, hi in boxes:
            new.add(level, lo, hi)
        new.freeze()
        for q, p in zip(new.patches, keep):
            q.cells = p.cells.copy()
            q.faces = [f.copy() for f in p.faces]
        init_from(new, old, level)
        cur = new
    return cur


def evolve(h, steps, eps, every=1, from_level=None, dtype=np.float64, min_side=4, efficiency=0.7):
    """Root steps with regridding as part of the time stepping (Sec. 2.1, 2.2: grids are created
    anew from the flags of their parents and take the data of the preceding grids of their level
    where those overlap them, the rest by prolongation).  After every `every` root steps, when all
    levels have reached the same time, the levels from `from_level` (default: the finest) up are
    regridded coarse to fine; a regrid that finds no flag keeps the hierarchy.  Returns the final
    hierarchy and, per root step, (dt0, boxes of the regridded levels or None)."""
    if from_level is not None and not 1 <= from_level < h.nlevels:
        raise ValueError("from_level must name a refined level")
    log = []
    for k in range(steps):
        dt = h.root_step()
        boxes = None
        if (k + 1) % every == 0:
            lv = h.nlevels - 1 if from_level is None else from_level
            try:
                h = regrid_levels(h, eps, dtype, min_side, efficiency, from_level=lv)
                boxes = sorted((p.level, tuple(int(v) for v in p.lo), tuple(int(v) for v in p.hi))
                               for p in h.patches if p.level >= lv)
            except ValueError:
                pass
        log.append((dt, boxes))
    return h, log
