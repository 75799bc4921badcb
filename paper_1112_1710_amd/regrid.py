"""Regridding of a bound hierarchy, of its finest level or of every level from a given one
upward (Sec. 2.2: grids decide which cells to refine and lay down child grids over them; new
grids take the data of the preceding grids of their level where those overlap them and are
prolongated from the parent elsewhere).

Flags are computed on the GPU (``hier_flag``), grown by a one-cell buffer, kept off the parent's
boundary layer and clustered on the host (``hier_regrid_boxes``); the new hierarchy is built
and filled on the GPU (``hier_init_from``).  The topology of a hierarchy is fixed once it is
finalised, so a regrid returns a new hierarchy.
"""
from dataclasses import dataclass, field

from .binding import Hierarchy


@dataclass
class Spec:
    """Patch list of a hierarchy: root_n and [(level, lo, hi), ...] in level index space."""
    root_n: tuple
    patches: list = field(default_factory=list)
    name: str = ""

    def levels(self):
        return 1 + max(p[0] for p in self.patches)

    def cells(self, level=None):
        tot = 0
        for lv, lo, hi in self.patches:
            if level is None or lv == level:
                n = 1
                for a in range(3):
                    n *= hi[a] - lo[a]
                tot += n
        return tot

    def zone_updates_per_root_step(self):
        tot = 0
        for lv, lo, hi in self.patches:
            n = 1
            for a in range(3):
                n *= hi[a] - lo[a]
            tot += n * 2 ** lv
        return tot


def new_spec(h, eps, min_side=4, efficiency=0.7):
    """The patch list with the finest level of bound hierarchy h replaced by boxes over the
    flagged cells of the level below."""
    top = h.levels - 1
    if top < 1:
        raise ValueError("regridding needs a refined level")
    boxes = h.regrid_boxes(top - 1, eps, min_side, efficiency)
    if not boxes:
        raise ValueError("no cell of the level below the finest one is flagged")
    keep = [p for p in h.spec.patches if p[0] < top]
    return Spec(root_n=tuple(h.spec.root_n), patches=keep + [(top, lo, hi) for lo, hi in boxes],
                name=f"{getattr(h.spec, 'name', '')} (regridded)")


def regrid(h, eps, min_side=4, efficiency=0.7, **kwargs):
    """A new hierarchy whose finest level covers the flagged cells of the level below, filled from h."""
    spec = new_spec(h, eps, min_side, efficiency)
    kwargs.setdefault("physics", h.physics)
    kwargs.setdefault("cs", h.cs)
    h2 = Hierarchy(spec, h.precision, device=h.device, **kwargs)
    h2.init_from(h, h.levels - 1)
    return h2


def regrid_levels(h, eps, min_side=4, efficiency=0.7, from_level=1, **kwargs):
    """A new hierarchy with h's levels below `from_level` and every level from `from_level` up to h's
    finest regridded coarse to fine: level l is laid over the flags of the new level l - 1 and filled
    from h's level-l patches where they overlap and from the new level l - 1 elsewhere.  A level
    whose parents hold no flag ends the hierarchy (ValueError when that is `from_level`)."""
    top = h.levels - 1
    if not 1 <= from_level <= top:
        raise ValueError("from_level must name a refined level")
    kwargs.setdefault("physics", h.physics)
    kwargs.setdefault("cs", h.cs)
    cur = h
    for level in range(from_level, top + 1):
        boxes = cur.regrid_boxes(level - 1, eps, min_side, efficiency)
        if not boxes:
            if level == from_level:
                raise ValueError("no cell below the first regridded level is flagged")
            break
        keep = [p for p in cur.spec.patches if p[0] < level]
        spec = Spec(root_n=tuple(h.spec.root_n), patches=keep + [(level, lo, hi) for lo, hi in boxes],
                    name=f"{getattr(h.spec, 'name', '')} (regridded from level {from_level})")
        nxt = Hierarchy(spec, h.precision, device=h.device, **kwargs)
        nxt.init_from(h, level, below=cur)
        cur = nxt
    return cur


def evolve(h, steps, eps, every=1, from_level=None, mode=None, min_side=4, efficiency=0.7, **kwargs):
    """Root steps with regridding in the time stepping loop: after every `every` root steps (all
    levels then at one time) the levels from `from_level` (default: the finest) up are regridded
    coarse to fine (regrid_levels) and the run continues on the new hierarchy; a regrid that finds
    no flag keeps the hierarchy.  Returns the final hierarchy and, per root step, (dt0, boxes of the
    regridded levels or None)."""
    from .binding import GRAPH
    mode = GRAPH if mode is None else mode
    if from_level is not None and not 1 <= from_level < h.levels:
        raise ValueError("from_level must name a refined level")
    log = []
    for k in range(steps):
        dt = h.step(mode)
        boxes = None
        if (k + 1) % every == 0:
            lv = h.levels - 1 if from_level is None else from_level
            try:
                h = regrid_levels(h, eps, min_side, efficiency, from_level=lv, **kwargs)
                boxes = sorted((p[0], tuple(p[1]), tuple(p[2])) for p in h.spec.patches if p[0] >= lv)
            except ValueError:
                pass
        log.append((dt, boxes))
    return h, log
