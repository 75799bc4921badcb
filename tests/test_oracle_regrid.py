"""Pins of the oracle's regridding (refinement flags, clustering, initialisation of new patches).

Exact cases: a planar density jump flags exactly the two cell layers beside it and
the strict threshold decides ties; the buffer grows a flag into its 3x3x3
neighbourhood; separated blobs give one box each (signature holes); random flag sets
keep the clustering invariants (every flag covered, boxes disjoint and inside the
array, each box efficient or too small to split).  Initialisation: new patches equal
to the old ones are copied bit for bit; partially overlapping ones copy the overlap
bit for bit, their prolongated cells restrict back to the parent exactly, stay
divergence-free, and a uniform state stays uniform; the resulting hierarchies obey
the nesting rules.
"""
import numpy as np
import pytest

from oracle import amr, regrid
from workloads import hierarchies as H
from workloads.fields import G, SmoothField, Uniform


def test_flags_of_a_planar_jump_and_strict_threshold():
    rho = np.ones((6, 7, 16))
    rho[:, :, 8:] = 1.25
    f = regrid.flag_cells(rho, 0.2)
    want = np.zeros_like(f)
    want[:, :, 7:9] = True
    assert np.array_equal(f, want)
    assert not regrid.flag_cells(rho, 0.25).any()      # |1.25 - 1| = 0.25 is not > 0.25 * 1
    assert np.array_equal(regrid.flag_cells(rho, 0.2499), want)
    f32 = regrid.flag_cells(rho.astype(np.float32), 0.2, np.float32)
    assert np.array_equal(f32, want)
    assert not regrid.flag_cells(np.full((4, 4, 4), 2.0), 1e-12).any()


def test_buffer_grows_one_cell_in_all_directions():
    f = np.zeros((7, 8, 9), dtype=bool)
    f[3, 4, 5] = True
    f[0, 0, 0] = True
    g = regrid.buffer_flags(f)
    want = np.zeros_like(f)
    want[2:5, 3:6, 4:7] = True
    want[0:2, 0:2, 0:2] = True
    assert np.array_equal(g, want)


def _check_clusters(f, boxes, min_side, eff):
    cover = np.zeros(f.shape, dtype=np.int64)
    for lo, hi in boxes:
        assert all(0 <= lo[a] < hi[a] <= f.shape[2 - a] for a in range(3))
        cover[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
        sub = f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        n = [hi[a] - lo[a] for a in range(3)]
        assert sub.any()
        # accepted only when efficient or when no side can be cut into two parts of min_side
        assert sub.sum() >= eff * np.prod(n) or all(x < 2 * min_side for x in n)
        # shrunk to its flags: every face plane of the box holds a flag
        for a in range(3):
            ax = tuple(2 - b for b in range(3) if b != a)
            sig = sub.sum(axis=ax)
            assert sig[0] > 0 and sig[-1] > 0
    assert np.all(cover[f] == 1)            # every flag covered exactly once
    assert np.all(cover <= 1)               # boxes disjoint


def test_separated_blobs_give_one_box_each():
    f = np.zeros((16, 16, 24), dtype=bool)
    f[2:6, 3:7, 2:8] = True
    f[8:12, 9:13, 14:20] = True
    boxes = regrid.cluster(f, min_side=2, efficiency=0.9)
    assert sorted(boxes) == sorted([((2, 3, 2), (8, 7, 6)), ((14, 9, 8), (20, 13, 12))])
    _check_clusters(f, boxes, 2, 0.9)


def test_single_box_when_efficient():
    f = np.zeros((10, 10, 10), dtype=bool)
    f[2:8, 2:8, 2:8] = True
    f[2, 2, 2] = False
    assert regrid.cluster(f, min_side=2, efficiency=0.7) == [((2, 2, 2), (8, 8, 8))]


@pytest.mark.parametrize("seed", range(6))
def test_random_flags_keep_the_clustering_invariants(seed):
    rng = np.random.default_rng(seed)
    f = rng.random((14, 12, 18)) < 0.08
    f = regrid.buffer_flags(f) & (rng.random(f.shape) < 0.7)
    boxes = regrid.cluster(f, min_side=3, efficiency=0.7)
    assert len(boxes) > 1
    _check_clusters(f, boxes, 3, 0.7)


def _blast_hierarchy():
    spec = H.HierarchySpec(root_n=(16, 16, 16), patches=[(0, (0, 0, 0), (16, 16, 16)),
                                                        (1, (8, 8, 8), (20, 20, 18))])
    return spec


class _Step:
    """Density step at x = 0.5 (rho 1 | 1.6), uniform p, v = 0, uniform B: flags a plane of root cells."""

    def patch(self, level, root_n, lo, hi):
        return Uniform(1.0, (0.0, 0.0, 0.0), 1.0, (1.0, 0.5, 0.25)).patch(level, root_n, lo, hi)


def test_child_boxes_nest_and_cover_the_flags():
    spec = _blast_hierarchy()
    h = amr.build(spec, SmoothField(31))
    # make a sharp density feature on the root: a ball of rho 2
    m = h.patches[0]
    n = m.n
    z, y, x = np.meshgrid(*(np.arange(G, G + n[a]) for a in (2, 1, 0)), indexing="ij")
    ball = (x - G - 9.5) ** 2 + (y - G - 6.5) ** 2 + (z - G - 7.5) ** 2 < 9.0
    m.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]][ball] *= 2.0
    boxes = regrid.child_boxes(h, 0, 0.3)
    assert boxes
    # the boxes form a valid level 1 under the root
    nh = amr.Hierarchy(spec.root_n)
    nh.add(0, (0, 0, 0), (16, 16, 16))
    for lo, hi in boxes:
        nh.add(1, lo, hi)
    nh.freeze()
    # every flagged root cell (away from the root's boundary layer) lies under a box
    rho = m.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]]
    f = regrid.buffer_flags(regrid.flag_cells(rho, 0.3))
    f[:1] = f[-1:] = False
    f[:, :1] = f[:, -1:] = False
    f[:, :, :1] = f[:, :, -1:] = False
    cov = np.zeros(f.shape, dtype=bool)
    for lo, hi in boxes:
        cov[lo[2] // 2:hi[2] // 2, lo[1] // 2:hi[1] // 2, lo[0] // 2:hi[0] // 2] = True
    assert np.all(cov[f])


def _pair(old_boxes, new_boxes, field):
    root = (16, 16, 16)
    old = amr.Hierarchy(root)
    old.add(0, (0, 0, 0), root)
    for lo, hi in old_boxes:
        old.add(1, lo, hi)
    old.freeze()
    old.set_state(field)
    new = amr.Hierarchy(root)
    new.add(0, (0, 0, 0), root)
    for lo, hi in new_boxes:
        new.add(1, lo, hi)
    new.freeze()
    new.patches[0].cells = old.patches[0].cells.copy()
    new.patches[0].faces = [f.copy() for f in old.patches[0].faces]
    regrid.init_from(new, old, 1)
    return old, new


def test_identical_boxes_copy_bit_for_bit():
    boxes = [((4, 6, 6), (12, 14, 14)), ((12, 6, 8), (18, 12, 14))]
    old, new = _pair(boxes, boxes, SmoothField(32))
    for p, q in zip(old.patches[1:], new.patches[1:]):
        i = old._interior_mask(p)
        assert np.array_equal(p.cells[:, i], q.cells[:, i])
        for d in range(3):
            m = old._closure_mask(p, d)
            assert np.array_equal(p.faces[d][m], q.faces[d][m])


def test_partial_overlap_copies_then_prolongates_conservatively():
    old_boxes = [((4, 6, 6), (12, 14, 14))]
    new_boxes = [((8, 4, 8), (20, 12, 16))]
    old, new = _pair(old_boxes, new_boxes, SmoothField(33))
    p, q = new.patches[1], old.patches[1]
    root = new.patches[0]
    # the overlap [8, 12) x [6, 12) x [8, 14) copies the old patch bit for bit
    po, qo = p.origin(), q.origin()
    lo, hi = np.array([8, 6, 8]), np.array([12, 12, 14])
    ps = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
    qs = tuple(slice(int(lo[a] - qo[a]), int(hi[a] - qo[a])) for a in (2, 1, 0))
    assert np.array_equal(p.cells[(slice(None),) + ps], q.cells[(slice(None),) + qs])
    i = new._interior_mask(p)
    assert np.all(np.isfinite(p.cells[:, i]))
    for d in range(3):
        assert np.all(np.isfinite(p.faces[d][new._closure_mask(p, d)]))
    # divergence-free interior
    div = amr.mhd.divergence(p.faces, new.dxv(1))
    assert np.max(np.abs(div[i])) * new.dx(1) < 1e-13
    # prolongated coarse cells restrict back to the parent
    ro = root.origin()
    worst = 0.0
    for cz in range(p.n[2] // 2):
        for cy in range(p.n[1] // 2):
            for cx in range(p.n[0] // 2):
                g = p.lo // 2 + np.array([cx, cy, cz])
                if np.all(g * 2 >= lo) and np.all(g * 2 < hi):
                    continue
                fz, fy, fx = G + 2 * cz, G + 2 * cy, G + 2 * cx
                mean = p.cells[:, fz:fz + 2, fy:fy + 2, fx:fx + 2].mean(axis=(1, 2, 3))
                c = g - ro
                worst = max(worst, float(np.max(np.abs(mean - root.cells[:, c[2], c[1], c[0]]))))
    assert worst < 1e-14


def test_uniform_state_stays_uniform():
    fld = Uniform(1.3, (0.3, -0.2, 0.1), 0.9, (0.5, 0.7, -0.4))
    old, new = _pair([((4, 6, 6), (12, 14, 14))], [((6, 4, 8), (16, 12, 18))], fld)
    p = new.patches[1]
    i = new._interior_mask(p)
    ref = fld.patch(1, (16, 16, 16), tuple(p.lo), tuple(p.hi))
    assert np.max(np.abs(p.cells[:, i] - ref.cells[:, i])) < 1e-14
    for d in range(3):
        m = new._closure_mask(p, d)
        assert np.max(np.abs(p.faces[d][m] - ref.faces[d][m])) < 1e-14


# ---------------------------------------------------------------------------------------------
# regridding every level from a given one, coarse to fine
# ---------------------------------------------------------------------------------------------
def _bumped_three_level(seed=51, centre=(0.28, 0.27, 0.25), width=0.06):
    """The three-level test hierarchy with a density bump inside its old level-2 patches."""
    o = amr.build(H.small_three_level(), SmoothField(seed))
    for p in o.patches:
        n = o.nl(p.level)
        c = [(np.arange(p.lo[a] - G, p.hi[a] + G + 1) + 0.5) / n[a] for a in range(3)]
        z, y, x = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
        p.cells[0] *= 1.0 + 0.6 * np.exp(-r2 / width ** 2)
    return o


def _check_new_level(old, new, level, eps):
    """Nesting, flag coverage, copied overlaps, conservative prolongation and div B of new level `level`."""
    parents = new.level_patches(level - 1)
    kids = new.level_patches(level)
    for p in kids:
        m = p.parent
        assert m in parents
        # inside the parent's interior shrunk by one parent cell
        assert np.all(p.lo >= 2 * (m.lo + 1)) and np.all(p.hi <= 2 * (m.hi - 1))
    # every buffered flag of a parent (off its boundary layer) lies under a child
    for m in parents:
        n = m.n
        f = regrid.buffer_flags(regrid.flag_cells(m.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]], eps))
        f[:1] = f[-1:] = False
        f[:, :1] = f[:, -1:] = False
        f[:, :, :1] = f[:, :, -1:] = False
        cov = np.zeros(f.shape, dtype=bool)
        for p in kids:
            if p.parent is m:
                lo, hi = p.lo // 2 - m.lo, p.hi // 2 - m.lo
                cov[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
        assert np.all(cov[f])
    copied = prolonged = 0
    for p in kids:
        po = p.origin()
        under = np.zeros(p.shape, dtype=bool)
        for q in old.level_patches(level):
            lo, hi = np.maximum(p.lo, q.lo), np.minimum(p.hi, q.hi)
            if np.any(hi <= lo):
                continue
            qo = q.origin()
            ps = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
            qs = tuple(slice(int(lo[a] - qo[a]), int(hi[a] - qo[a])) for a in (2, 1, 0))
            assert np.array_equal(p.cells[(slice(None),) + ps], q.cells[(slice(None),) + qs])
            under[ps] = True
            copied += int(np.prod(hi - lo))
        # prolongated parent cells restrict back to the (new) parent
        m = p.parent
        mo = m.origin()
        for cz in range(p.n[2] // 2):
            for cy in range(p.n[1] // 2):
                for cx in range(p.n[0] // 2):
                    fz, fy, fx = G + 2 * cz, G + 2 * cy, G + 2 * cx
                    if under[fz, fy, fx]:
                        continue
                    g = p.lo // 2 + np.array([cx, cy, cz]) - mo
                    mean = p.cells[:, fz:fz + 2, fy:fy + 2, fx:fx + 2].mean(axis=(1, 2, 3))
                    ref = m.cells[:, g[2], g[1], g[0]]
                    assert np.max(np.abs(mean - ref)) <= 1e-14 * np.max(np.abs(ref))
                    prolonged += 8
        i = new._interior_mask(p)
        div = amr.mhd.divergence(p.faces, new.dxv(level))
        assert np.max(np.abs(div[i])) * new.dx(level) < 1e-13
    return copied, prolonged


def test_regrid_levels_lays_every_level_over_the_new_flags():
    old = _bumped_three_level()
    new = regrid.regrid_levels(old, 0.2, min_side=4)
    assert new.nlevels == 3
    # the root is untouched
    assert np.array_equal(new.patches[0].cells, old.patches[0].cells)
    assert all(np.array_equal(a, b) for a, b in zip(new.patches[0].faces, old.patches[0].faces))
    for level in (1, 2):
        copied, prolonged = _check_new_level(old, new, level, 0.2)
        assert copied > 0 and prolonged > 0, (level, copied, prolonged)


def test_regrid_levels_from_the_finest_keeps_the_coarser_levels():
    old = _bumped_three_level()
    new = regrid.regrid_levels(old, 0.2, min_side=4, from_level=2)
    for p, q in zip(new.patches, old.patches):
        if q.level == 2 or p.level == 2:
            break
        assert p.level == q.level and np.array_equal(p.lo, q.lo) and np.array_equal(p.hi, q.hi)
        assert np.array_equal(p.cells, q.cells)
    assert len(new.level_patches(1)) == len(old.level_patches(1))
    _check_new_level(old, new, 2, 0.2)


def test_regrid_levels_ends_at_a_level_without_flags():
    old = _bumped_three_level()
    new = regrid.regrid_levels(old, 0.25, min_side=4)
    assert new.nlevels == 2
    _check_new_level(old, new, 1, 0.25)
    flat = amr.build(H.small_three_level(), Uniform(1.0, (0.1, 0.0, 0.0), 1.0, (0.3, 0.2, 0.1)))
    with pytest.raises(ValueError):
        regrid.regrid_levels(flat, 0.01)


def test_evolve_regrids_in_the_time_stepping_loop_and_conserves():
    """Three root steps of the three-level hierarchy with levels 1 and 2 regridded after every root step
    (Sec. 2.1: new grids each step, filled from the preceding ones and the new parents): every regrid
    finds flags, the composite sums of mass, momentum and energy are conserved to round-off through
    the steps and the regrids (restricted coarse data under the old fine grids, copied overlaps and
    conservative prolongation), and div B stays zero on every level."""
    o = _bumped_three_level()
    c0 = o.conservation()
    scale = sum(abs(x) for x in c0[:5])
    h, log = regrid.evolve(o, 3, 0.05, every=1, from_level=1)
    assert all(boxes is not None for _, boxes in log)
    assert h is not o and h.nlevels == 3
    c1 = h.conservation()
    assert np.all(np.abs(c1[:5] - c0[:5]) <= 1e-13 * scale), (c1[:5] - c0[:5])
    assert h.max_divergence() < 1e-10
    # the regridded levels nest and are disjoint (the hierarchy was accepted by freeze())
    for p in h.patches:
        if p.level > 0:
            assert p.parent is not None and p.parent.level == p.level - 1
