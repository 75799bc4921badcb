"""Pins of the oracle's AMR layer against the paper and exact invariants.

Paper-fixed values: the extended-ghost update counts of the 2-D example in
Sec. 4 (160, 104, 416, 38 %), the serial level visit order 0,1,2,2,1,2,2
(Sec. 4), R^l substeps of level l per root step (Sec. 2.1), single parent and
no same-level overlap (Sec. 2).  Exact invariants: composite conservation of
mass, momentum and energy with refluxing, zero discrete divergence,
free-stream preservation across coarse/fine boundaries, restriction of a
prolongation, exactness of prolongation on linear fields, and
bit-identical results when stale ghost data are poisoned with NaN.
"""
import math
import os

import numpy as np
import pytest

from oracle import amr, mhd
from workloads import hierarchies as H
from workloads.fields import G, SmoothField, Uniform, _coords, _clean, PatchState


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """Key = value lines of a fixture under tests/golden (values as integer lists; '#' lines are comments)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = (t.strip() for t in line.split("=", 1))
                out[key] = [int(x) for x in val.split()]
    return out


def _boxcells(box):
    lo, hi = box
    return int(np.prod(np.asarray(hi) - np.asarray(lo)))


def test_extended_ghost_counts_of_the_paper_example():
    """The paper's 2-D example: 4x4 grid, R=2, n_ghost=4: 12x12 + 4x4 = 160 updates; four 2x2 pieces:
    4 x (10x10 + 2x2) = 416; 38 %.  The printed values come from tests/golden."""
    g = _golden("sec4_extended_ghost_example.txt")
    n, r, ng, k = g["grid"], g["ratio"][0], g["n_ghost"][0], g["pieces"][0]
    side = int(round(math.sqrt(k)))
    sub = tuple(x // side for x in n)
    whole = sum(_boxcells(amr.update_box((0, 0), tuple(n), 1, s, ratio=r, n_g=ng)) for s in range(r))
    piece = sum(_boxcells(amr.update_box((0, 0), sub, 1, s, ratio=r, n_g=ng)) for s in range(r))
    assert whole == g["updates_whole"][0]
    assert piece == g["updates_per_piece"][0]
    assert k * piece == g["updates_split_total"][0]
    assert round(100 * whole / (k * piece)) == g["efficiency_percent"][0]


def test_update_region_shrinks_by_stencil_depth():
    lo, hi = (4, 4, 4), (12, 12, 12)
    assert amr.update_box(lo, hi, 1, 0) == ((2, 2, 2), (14, 14, 14))
    assert amr.update_box(lo, hi, 1, 1) == (lo, hi)
    assert amr.update_box(lo, hi, 0, 0) == (lo, hi)


def test_nesting_rules():
    h = amr.Hierarchy((16, 16, 16))
    h.add(0, (0, 0, 0), (16, 16, 16))
    with pytest.raises(amr.NestingError):
        h.add(1, (3, 4, 4), (12, 12, 12))     # odd corner
    with pytest.raises(amr.NestingError):
        h.add(1, (0, 4, 4), (12, 12, 12))     # touches the parent boundary (no inset)
    with pytest.raises(amr.NestingError):
        h.add(2, (8, 8, 8), (16, 16, 16))     # no parent on level 1
    h.add(1, (4, 4, 4), (12, 12, 12))
    with pytest.raises(amr.NestingError):
        h.add(1, (10, 10, 10), (14, 14, 14))  # overlaps a sibling
    h.add(1, (12, 4, 4), (16, 12, 12))        # adjacent sibling is fine
    h.freeze()
    with pytest.raises(amr.NestingError):
        h.add(1, (20, 20, 20), (24, 24, 24))  # frozen
    h2 = amr.Hierarchy((16, 16, 16))
    h2.add(0, (0, 0, 0), (8, 16, 16))
    with pytest.raises(amr.NestingError):
        h2.freeze()                           # root not tiled


def test_visit_order_and_substep_counts():
    g = _golden("sec4_serial_visit_order.txt")
    spec = H.small_three_level()
    assert spec.levels() == g["levels"][0]
    h = amr.build(spec, SmoothField(7))
    h.root_step()
    assert h.log == g["order"]
    for lv in range(g["levels"][0]):
        assert h.log.count(lv) == g["ratio"][0] ** lv


@pytest.fixture(scope="module")
def three_level_run():
    h = amr.build(H.small_three_level(), SmoothField(1112))
    c0 = h.conservation()
    scale = []
    for q in range(5):
        scale.append(sum(float(np.sum(np.abs(p.cells[q][h.leaf_mask(p)]))) * h.dx(p.level) ** 3 for p in h.patches))
    for _ in range(2):
        h.root_step()
    return h, c0, scale


def test_composite_conservation(three_level_run):
    h, c0, scale = three_level_run
    c1 = h.conservation()
    for q in range(5):
        assert abs(c1[q] - c0[q]) <= 1e-14 * scale[q], (q, c1[q] - c0[q], scale[q])


def test_divergence_free_everywhere(three_level_run):
    h, _, _ = three_level_run
    assert h.max_divergence() < 1e-11


def test_same_level_sync_is_bit_zero(three_level_run):
    h, _, _ = three_level_run
    assert h.diag["sync_flux_max"] == 0.0
    assert h.diag["sync_face_max"] == 0.0


def test_free_stream_across_levels():
    fld = Uniform(1.3, (0.3, -0.2, 0.1), 0.9, (0.5, 0.7, -0.4))
    h = amr.build(H.small_three_level(), fld)
    ref = h.copy_state()
    h.root_step(0.003)
    for p, (c, f) in zip(h.patches, ref):
        i = h._interior_mask(p)
        assert np.max(np.abs(p.cells[:, i] - c[:, i])) < 1e-14
        for d in range(3):
            m = h._closure_mask(p, d)
            assert np.max(np.abs(p.faces[d][m] - f[d][m])) < 1e-14


def test_stale_ghosts_never_reach_the_interior():
    """Poisoning every value outside each substep's valid region leaves the results bit-identical."""
    spec = H.small_three_level()
    a = amr.build(spec, SmoothField(3))
    b = amr.build(spec, SmoothField(3))
    b.poison = True
    for _ in range(2):
        dt = a.root_step()
        b.root_step(dt)
    for p, q in zip(a.patches, b.patches):
        i = a._interior_mask(p)
        assert np.array_equal(p.cells[:, i], q.cells[:, i])
        for d in range(3):
            m = a._closure_mask(p, d)
            assert np.array_equal(p.faces[d][m], q.faces[d][m])


class _Linear:
    """Linear cells and the divergence-free linear field B = (1 + x + 2y, 0.5 - y + 3z, 2 - x + 0.25 y);
    the total energy 30 + x + y + z exceeds the kinetic plus magnetic energy everywhere on the test
    boxes, so every prolongated child is physical and the positivity fallback stays inactive."""

    def patch(self, level, root_n, lo, hi):
        h, c, l = _coords(level, root_n, lo, hi)
        # unreduced coordinates (no periodic wrap: the test stays away from the domain edge)
        c = [(np.arange(lo[a] - G, hi[a] + G + 1) + 0.5) * h[a] for a in range(3)]
        l = [np.arange(lo[a] - G, hi[a] + G + 1) * h[a] for a in range(3)]
        zz, yy, xx = np.meshgrid(c[2], c[1], c[0], indexing='ij')
        cells = np.stack([1 + 0.5 * xx - 0.25 * yy + 0.125 * zz, 0.1 * xx, -0.2 * yy, 0.3 * zz, 30 + xx + yy + zz])
        zl, yl, xl = np.meshgrid(l[2], l[1], l[0], indexing='ij')
        bx = 1 + xl + 2 * yy
        by = 0.5 - yl + 3 * zz
        bz = 2 - xx + 0.25 * yy
        # face averages of a linear function equal the value at the face centre
        bx = 1 + xl + 2 * yy
        by = 0.5 - yl + 3 * zz
        bz = 2 - xx + 0.25 * yy
        return _clean(PatchState(cells, [bx, by, bz + 0 * zl]))


def _prolong_setup(field):
    spec = H.HierarchySpec(root_n=(16, 16, 16), patches=[(0, (0, 0, 0), (16, 16, 16)), (1, (8, 8, 8), (16, 18, 20))])
    h = amr.build(spec, field)
    m, p = h.patches
    m.old_cells, m.old_faces = m.cells, m.faces
    truth = (p.cells.copy(), [f.copy() for f in p.faces])
    for a in (p.cells, *p.faces):
        a[...] = np.nan
    # keep the fine interior (own data) and let the ghost fill produce the ghost shell
    p.cells[:, G:-G - 1, G:-G - 1, G:-G - 1] = truth[0][:, G:-G - 1, G:-G - 1, G:-G - 1]
    for d in range(3):
        m_ = h._closure_mask(p, d)
        p.faces[d][m_] = truth[1][d][m_]
    h.ghost_fill(1, 0)
    return h, m, p, truth


def test_prolongation_exact_on_linear_fields():
    h, m, p, truth = _prolong_setup(_Linear())
    v = slice(0, -1)
    assert np.max(np.abs(p.cells[:, v, v, v] - truth[0][:, v, v, v])) < 1e-13
    assert np.max(np.abs(p.faces[0][v, v, :] - truth[1][0][v, v, :])) < 1e-13
    assert np.max(np.abs(p.faces[1][v, :, v] - truth[1][1][v, :, v])) < 1e-13
    assert np.max(np.abs(p.faces[2][:, v, v] - truth[1][2][:, v, v])) < 1e-13


def test_prolongation_is_conservative_and_divergence_free():
    h, m, p, truth = _prolong_setup(SmoothField(11))
    dxf = h.dx(1)
    div = mhd.divergence(p.faces, [dxf] * 3)[:-1, :-1, :-1]
    assert np.max(np.abs(div)) * dxf < 1e-13
    # restriction of the prolongated ghost shell gives back the coarse cells
    mo = m.origin()
    ncell = (p.n + 2 * G) // 2
    clo = (p.lo - G) // 2
    worst = 0.0
    for cz in range(ncell[2]):
        for cy in range(ncell[1]):
            for cx in range(ncell[0]):
                fz, fy, fx = 2 * cz, 2 * cy, 2 * cx
                if h.cell_src[p.id][fz, fy, fx] >= 0:
                    continue
                mean = p.cells[:, fz:fz + 2, fy:fy + 2, fx:fx + 2].mean(axis=(1, 2, 3))
                ci = clo + np.array([cx, cy, cz]) - mo
                worst = max(worst, float(np.max(np.abs(mean - m.cells[:, ci[2], ci[1], ci[0]]))))
                # area mean of the fine faces on the coarse x-face
                fm = p.faces[0][fz:fz + 2, fy:fy + 2, fx].mean()
                worst = max(worst, abs(fm - m.faces[0][ci[2], ci[1], ci[0]]))
    assert worst < 1e-14


def _shock_like_parent(o, rows):
    """Uniform state (rho 1, v 0, p 1, B (1, 0, 0)); along x on the given (y, z) rows of coarse cells
    0, 1, 2 the momentum rises 0, a, 2a with p = 0.01 in all three (each coarse cell physical)."""
    m = o.patches[0]
    gam = o.gamma
    for (y, z, a) in rows:
        for i, mx in enumerate((0.0, a, 2.0 * a)):
            X, Y, Z = G + i, G + y, G + z
            m.cells[1, Z, Y, X] = mx
            m.cells[4, Z, Y, X] = 0.5 * mx * mx + 0.5 + 0.01 / (gam - 1.0)
    m.old_cells, m.old_faces = m.cells.copy(), [f.copy() for f in m.faces]


def test_prolongation_positivity_fallback():
    """A coarse cell whose limited-linear children would carry more kinetic than total energy
    (momentum slope 3 at p = 0.01) hands its 8 children its own conserved values; a gentle
    slope (0.1) keeps the linear children; both keep the coarse mean exactly."""
    o = amr.build(H.small_two_level(), Uniform(1.0, (0, 0, 0), 1.0, (1, 0, 0)))
    _shock_like_parent(o, [(4, 4, 3.0), (4, 5, 0.1)])
    p = o.patches[1]                          # fine box (4,6,6)-(12,14,14): coarse x = 0, 1 are ghosts
    o._prolong(p)
    po = p.origin()

    def children(cx, cy, cz):
        f = 2 * np.array([cx, cy, cz]) - po
        return p.cells[:, f[2]:f[2] + 2, f[1]:f[1] + 2, f[0]:f[0] + 2]

    steep = children(1, 4, 4)
    u0 = o.patches[0].cells[:, G + 4, G + 4, G + 1]
    assert np.array_equal(steep, np.broadcast_to(u0[:, None, None, None], steep.shape))
    gentle = children(1, 4, 5)
    u1 = o.patches[0].cells[:, G + 5, G + 4, G + 1]
    assert np.ptp(gentle[1]) > 0.04                       # linear momentum children: 0.1 +- 0.025
    assert np.allclose(gentle.reshape(5, -1).mean(axis=1), u1, rtol=0, atol=1e-15)
    # without the fallback the steep cell's children would be unphysical
    bc = mhd.cell_centred_b(p.faces)
    f = 2 * np.array([1, 4, 4]) - po
    sl = (slice(f[2], f[2] + 2), slice(f[1], f[1] + 2), slice(f[0], f[0] + 2))
    slope = 3.0
    lin_mx = u0[1] + 0.25 * slope * np.array([-1.0, 1.0])
    lin_e = u0[4] + 0.25 * min(u0[4] - o.patches[0].cells[4, G + 4, G + 4, G + 0],
                              o.patches[0].cells[4, G + 4, G + 4, G + 2] - u0[4]) * np.array([-1.0, 1.0])
    p_lin = (o.gamma - 1) * (lin_e - 0.5 * lin_mx ** 2 - 0.5 * float(np.max(bc[0][sl] ** 2)))
    assert p_lin.min() < 0.0
    # the pressure of every prolongated ghost cell is positive
    w = mhd.prim_from_cons(p.cells, bc, o.gamma)
    ghost = o.cell_src[p.id] < 0
    ghost[:, :, -1] = ghost[:, -1, :] = ghost[-1, :, :] = False
    assert np.all(w[4][ghost] > 0.0)


def test_interior_face_map_zeroes_fine_divergence():
    M, outer_idx, inner_idx = amr.Hierarchy.interior_face_map()
    rng = np.random.default_rng(3)
    for _ in range(20):
        o = rng.standard_normal(24)
        # make the outer faces compatible (zero net flux out of the coarse cell)
        net = 0.0
        for (d, side, t2, t1), k in outer_idx.items():
            net += o[k] if side == 2 else -o[k]
        o[outer_idx[(0, 2, 0, 0)]] -= net
        inner = M @ o
        b = [np.zeros((2, 2, 3)), np.zeros((2, 3, 2)), np.zeros((3, 2, 2))]
        for (d, side, t2, t1), k in outer_idx.items():
            idx = [None, None, None]
            a1, a2 = [a for a in range(3) if a != d]
            idx[d], idx[a1], idx[a2] = side, t1, t2
            b[d][idx[2], idx[1], idx[0]] = o[k]
        for (d, t2, t1), k in inner_idx.items():
            idx = [None, None, None]
            a1, a2 = [a for a in range(3) if a != d]
            idx[d], idx[a1], idx[a2] = 1, t1, t2
            b[d][idx[2], idx[1], idx[0]] = inner[k]
        div = (b[0][:, :, 1:] - b[0][:, :, :-1]) + (b[1][:, 1:, :] - b[1][:, :-1, :]) + (b[2][1:] - b[2][:-1])
        assert np.max(np.abs(div)) < 1e-13


def test_ghost_sources_hold_the_periodic_image():
    h = amr.build(H.small_three_level())
    for p in h.patches:
        nl = h.nl(p.level)
        src = h.cell_src[p.id]
        for (z, y, x) in np.argwhere(src >= 0)[::7]:
            qid, lin = int(src[z, y, x] >> 32), int(src[z, y, x] & (2 ** 32 - 1))
            q = h.patches[qid]
            qz, rem = divmod(lin, q.shape[1] * q.shape[2])
            qy, qx = divmod(rem, q.shape[2])
            g = np.array([x, y, z]) + p.origin()
            gq = np.array([qx, qy, qz]) + q.origin()
            assert np.all((g - gq) % nl == 0)
            assert np.all(gq >= q.lo) and np.all(gq < q.hi)


def _image_axis(g, lo, hi, n, closure):
    """Per 1-D global index g: does some periodic image g + k n lie in [lo, hi) ([lo, hi] for a
    face's own axis)?  Tried for every shift k that can matter (|k| <= 2)."""
    ok = np.zeros(g.shape, dtype=bool)
    for k in range(-2, 3):
        x = g + k * n
        ok |= (x >= lo) & ((x <= hi) if closure else (x < hi))
    return ok


@pytest.mark.parametrize("name", ["small_two_level", "small_three_level", "root_tiled", "minimal_patches"])
def test_ghost_sources_brute_force_over_periodic_images(name):
    """Every padded cell and face of every patch, enumerated in global coordinates over all
    periodic shifts (independent of the map builder): the source is the patch itself if an
    image lies in its interior (closure, for faces), else the lowest-id same-level patch with
    such an image, else none; the stored entry must name that patch and an entry of it holding
    a periodic image of the same point.  Faces reach one entry further than cells on their own
    axis, so the last face plane of the padded box is included."""
    h = amr.build(getattr(H, name)())
    for p in h.patches:
        nl = h.nl(p.level)
        Z, Y, X = p.shape
        org = p.origin()
        coord = [np.arange((X, Y, Z)[a]) + org[a] for a in range(3)]
        same = [p] + [q for q in h.level_patches(p.level) if q is not p]
        for kind in range(4):                       # 0 = cells, 1 + d = faces normal to d
            d = kind - 1
            src = h.cell_src[p.id] if kind == 0 else h.face_src[p.id][d]
            valid = [coord[a] < p.hi[a] + G + (1 if a == d else 0) for a in range(3)]
            want = np.full(p.shape, -1, dtype=np.int64)
            for q in same:
                hit = [_image_axis(coord[a], q.lo[a], q.hi[a], nl[a], a == d) & valid[a] for a in range(3)]
                m = hit[2][:, None, None] & hit[1][None, :, None] & hit[0][None, None, :]
                want[m & (want < 0)] = q.id
            got_q = np.where(src >= 0, src >> 32, -1)
            assert np.array_equal(got_q, want), (name, p.id, kind)
            for (z, y, x) in np.argwhere(src >= 0):
                q = h.patches[int(src[z, y, x] >> 32)]
                lin = int(src[z, y, x] & (2 ** 32 - 1))
                qz, rem = divmod(lin, q.shape[1] * q.shape[2])
                qy, qx = divmod(rem, q.shape[2])
                gq = np.array([qx, qy, qz]) + q.origin()
                g = np.array([x, y, z]) + org
                assert np.all((g - gq) % nl == 0)
                for a in range(3):
                    assert q.lo[a] <= gq[a] and (gq[a] <= q.hi[a] if a == d else gq[a] < q.hi[a])


def test_ghost_sources_follow_neighbour_inheritance():
    """Sec. 3.1: a child's same-level neighbours are children of its parent or of the parent's neighbours."""
    h = amr.build(H.small_three_level())
    nbrs = {}
    for p in h.patches:
        src = h.cell_src[p.id]
        ids = set(int(v >> 32) for v in np.unique(src[src >= 0])) - {p.id}
        nbrs[p.id] = ids
    for p in h.patches:
        if p.level == 0:
            continue
        allowed = {p.parent.id} | nbrs[p.parent.id]
        for q in nbrs[p.id]:
            assert h.patches[q].parent.id in allowed


def test_cfl_brute_force():
    h = amr.build(H.small_two_level(), SmoothField(9))
    dt = h.cfl_dt()
    best = math.inf
    gam = h.gamma
    for lv in range(2):
        smax = 0.0
        dx = h.dx(lv)
        for p in h.level_patches(lv):
            for k in range(G, G + int(p.n[2])):
                for j in range(G, G + int(p.n[1])):
                    for i in range(G, G + int(p.n[0])):
                        rho = p.cells[0, k, j, i]
                        v = p.cells[1:4, k, j, i] / rho
                        b = [0.5 * (p.faces[0][k, j, i] + p.faces[0][k, j, i + 1]),
                             0.5 * (p.faces[1][k, j, i] + p.faces[1][k, j + 1, i]),
                             0.5 * (p.faces[2][k, j, i] + p.faces[2][k + 1, j, i])]
                        b2 = sum(x * x for x in b)
                        pr = (gam - 1) * (p.cells[4, k, j, i] - 0.5 * rho * float(v @ v) - 0.5 * b2)
                        s = 0.0
                        for d in range(3):
                            a2 = gam * pr / rho
                            cf = math.sqrt(0.5 * (a2 + b2 / rho + math.sqrt((a2 + b2 / rho) ** 2 - 4 * a2 * b[d] ** 2 / rho)))
                            s += (abs(v[d]) + cf) / dx
                        smax = max(smax, s)
        best = min(best, 2 ** lv * 0.4 / smax)
    assert abs(dt - best) <= 1e-13 * best


# ---------------------------------------------------------------------------------------------
# coarse-time-derivative ghosts (the other solution for isolated grids named in Sec. 2.3)
# ---------------------------------------------------------------------------------------------
def test_time_ghosts_update_only_interiors():
    """With time-derivative ghosts no patch updates ghost cells, at any substep."""
    for s in range(2):
        assert amr.update_box((4, 4, 4), (12, 10, 8), 1, s, ghosts="time") == ((4, 4, 4), (12, 10, 8))
    assert amr.update_box((4, 4, 4), (12, 10, 8), 1, 0) == ((2, 2, 2), (14, 12, 10))


def test_time_ghosts_nesting_rule():
    """A grandchild whose prolongation would read parent ghost cells that nothing refreshes at the
    parent's new time is rejected; one whose reads stay inside the parent or in ghost cells a
    sibling of the parent holds is accepted; extended ghosts accept both."""
    with pytest.raises(amr.NestingError):
        amr.build(H.small_three_level(), ghosts="time")
    amr.build(H.small_three_level(), ghosts="extended")
    amr.build(H.small_three_level_td(), ghosts="time")


def test_time_ghosts_free_stream():
    fld = Uniform(1.3, (0.3, -0.2, 0.1), 0.9, (0.5, 0.7, -0.4))
    h = amr.build(H.small_three_level_td(), fld, ghosts="time")
    ref = h.copy_state()
    h.root_step(0.003)
    for p, (c, f) in zip(h.patches, ref):
        i = h._interior_mask(p)
        assert np.max(np.abs(p.cells[:, i] - c[:, i])) < 1e-14
        for d in range(3):
            m = h._closure_mask(p, d)
            assert np.max(np.abs(p.faces[d][m] - f[d][m])) < 1e-14


def test_time_ghosts_conservation_divergence_and_sync():
    h = amr.build(H.small_three_level_td(), SmoothField(12), ghosts="time")
    s0 = h.conservation()
    scale = max(abs(s0[0]), abs(s0[4]))
    for _ in range(2):
        h.root_step()
    s1 = h.conservation()
    for q in range(5):
        assert abs(s1[q] - s0[q]) <= 1e-13 * scale, q
    assert h.max_divergence() < 1e-11
    assert h.diag["sync_flux_max"] == 0.0 and h.diag["sync_face_max"] == 0.0


def test_time_ghosts_stale_data_never_reach_the_interior():
    """Poisoning every value outside each substep's update region (the parent's advanced ghost layers
    included) leaves time-derivative-ghost results bit-identical."""
    spec = H.small_three_level_td()
    a = amr.build(spec, SmoothField(13), ghosts="time")
    b = amr.build(spec, SmoothField(13), ghosts="time")
    b.poison = True
    for _ in range(2):
        dt = a.root_step()
        b.root_step(dt)
    for p, q in zip(a.patches, b.patches):
        i = a._interior_mask(p)
        assert np.array_equal(p.cells[:, i], q.cells[:, i])
        for d in range(3):
            m = a._closure_mask(p, d)
            assert np.array_equal(p.faces[d][m], q.faces[d][m])


def test_time_ghosts_differ_from_extended_ghosts_at_truncation_level():
    """Both ghost treatments are consistent discretisations: one root step of a smooth flow differs
    between them, by far less than the flow's own change."""
    spec = H.small_two_level()
    a = amr.build(spec, SmoothField(14))
    b = amr.build(spec, SmoothField(14), ghosts="time")
    ref = a.copy_state()
    dt = a.root_step()
    b.root_step(dt)
    for c in range(5):
        diff = change = 0.0
        for p, q, (c0, _) in zip(a.patches, b.patches, ref):
            i = a._interior_mask(p)
            diff += float(np.sum(np.abs(p.cells[c][i] - q.cells[c][i])))
            change += float(np.sum(np.abs(p.cells[c][i] - c0[c][i])))
        assert 0.0 < diff < 0.1 * change, (c, diff, change)


def test_time_ghost_prolongation_is_linear_in_time():
    """For parent states linear in space at both ends of the step, the substep-1 ghosts equal the
    linear field of the time-interpolated parent state (the prolongation is exact on linear data)."""
    h, m, p, truth = _prolong_setup(_Linear())
    old_c, old_f = m.cells.copy(), [f.copy() for f in m.faces]
    # a second linear state: cells and the divergence-free field scaled, cells shifted
    new_c = 1.5 * old_c + 0.25
    new_f = [1.5 * f for f in old_f]
    m.old_cells, m.old_faces = old_c, old_f
    m.cells, m.faces = new_c, new_f
    want_c = 0.5 * (truth[0] + (1.5 * truth[0] + 0.25))
    want_f = [0.5 * (f + 1.5 * f) for f in truth[1]]
    # the fine patch's own faces (read where they bound a prolongated coarse cell) at the same time
    for d in range(3):
        own = h._closure_mask(p, d)
        p.faces[d][own] = want_f[d][own]
    h._prolong(p, 0.5)
    # compare where the prolongation writes: ghost entries without a same-level source (the
    # padding layer beyond the last cell excluded)
    v = (slice(0, -1),) * 3
    cm = np.zeros(p.shape, dtype=bool)
    cm[v] = h.cell_src[p.id][v] < 0
    assert cm.sum() > 0
    assert np.max(np.abs(p.cells[:, cm] - want_c[:, cm])) < 1e-12
    fv = [(slice(0, -1), slice(0, -1), slice(None)), (slice(0, -1), slice(None), slice(0, -1)),
          (slice(None), slice(0, -1), slice(0, -1))]
    for d in range(3):
        fm = np.zeros(p.shape, dtype=bool)
        fm[fv[d]] = h.face_src[p.id][d][fv[d]] < 0
        assert fm.sum() > 0
        assert np.max(np.abs(p.faces[d][fm] - want_f[d][fm])) < 1e-12, d
