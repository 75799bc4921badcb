"""Regridding on the GPU against the oracle: refinement flags bit for bit, the boxes laid over
them, the new levels' initial data (copied overlaps bit for bit, prolongated cells to the parity
tolerance) and a root step of the regridded hierarchy; the finest level alone and every level
coarse to fine."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr, regrid as oregrid  # noqa: E402
from paper_1112_1710_amd import BATCHED, FP32, FP32_MIXED, FP64, Hierarchy  # noqa: E402
from paper_1112_1710_amd.regrid import new_spec, regrid, regrid_levels  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import G, SmoothField  # noqa: E402

from ._common import FIELDS, rel_l1, upload_oracle_state  # noqa: E402

TOL = {FP64: 1e-12, FP32: 1e-5, FP32_MIXED: 1e-5}


def _say(*a):
    print(*a, flush=True)


def _bumped_oracle(spec, precision, seed=51, centre=(0.55, 0.45, 0.5), width=0.08):
    """Oracle hierarchy with a smooth field plus a sharp density bump (every level sampled at its cell
    centres), rounded to float32 for the FP32 runs."""
    o = amr.build(spec, SmoothField(seed))
    for p in o.patches:
        n = o.nl(p.level)
        c = [(np.arange(p.lo[a] - G, p.hi[a] + G + 1) + 0.5) / n[a] for a in range(3)]
        z, y, x = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
        p.cells[0] *= 1.0 + 0.6 * np.exp(-r2 / width ** 2)
        if precision != FP64:
            p.cells = p.cells.astype(np.float32).astype(np.float64)
            p.faces = [f.astype(np.float32).astype(np.float64) for f in p.faces]
    return o


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("name", ["small_two_level", "root_tiled"])
def test_flags_bit_exact(name, precision):
    spec = getattr(H, name)()
    _say("regrid flags", name, precision)
    o = _bumped_oracle(spec, precision)
    h = Hierarchy(spec, precision)
    upload_oracle_state(h, o)
    dtype = np.float64 if precision == FP64 else np.float32
    nflag = 0
    for level in range(spec.levels()):
        got = h.flags(level, 0.05)
        for pid, f in got.items():
            p = o.patches[pid]
            n = p.n
            want = oregrid.flag_cells(p.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]], 0.05, dtype)
            assert np.array_equal(f.astype(bool), want), pid
            nflag += int(want.sum())
    assert nflag > 0


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_regrid_matches_oracle(precision):
    """Regrid level 1 of a two-level hierarchy over the flagged root cells: same boxes as the oracle,
    the new level's data and one root step of the new hierarchy within the parity tolerance."""
    spec = H.small_two_level()
    _say("regrid", precision)
    o = _bumped_oracle(spec, precision)
    h = Hierarchy(spec, precision)
    upload_oracle_state(h, o)
    eps = 0.05
    spec2 = new_spec(h, eps, min_side=2, efficiency=0.7)
    want_boxes = oregrid.child_boxes(o, 0, eps, np.float64 if precision == FP64 else np.float32,
                                     min_side=2, efficiency=0.7)
    got_boxes = [(lo, hi) for lv, lo, hi in spec2.patches if lv == 1]
    assert got_boxes == want_boxes and len(got_boxes) > 0
    h2 = regrid(h, eps, min_side=2, efficiency=0.7)
    # oracle: the same new hierarchy, root copied, level 1 from the old level 1 and the root
    o2 = amr.Hierarchy(spec2.root_n)
    for lv, lo, hi in spec2.patches:
        o2.add(lv, lo, hi)
    o2.freeze()
    o2.patches[0].cells = o.patches[0].cells.copy()
    o2.patches[0].faces = [f.copy() for f in o.patches[0].faces]
    oregrid.init_from(o2, o, 1)
    err = rel_l1(h2, o2)
    assert np.all(err <= TOL[precision]), dict(zip(FIELDS, err))
    # overlapping old data arrives bit for bit
    for pid, p in enumerate(o2.patches):
        if p.level != 1:
            continue
        cells, faces = h2.download(pid)
        for q in o.patches:
            if q.level != 1:
                continue
            lo = np.maximum(p.lo, q.lo)
            hi = np.minimum(p.hi, q.hi)
            if np.any(hi <= lo):
                continue
            po = p.origin()
            sl = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
            assert np.array_equal(cells[(slice(None),) + sl], o2.patches[pid].cells[(slice(None),) + sl])
    # a root step of the regridded hierarchy
    dt = o2.cfl_dt()
    o2.root_step(dt)
    h2.step(BATCHED, dt)
    err = rel_l1(h2, o2)
    assert np.all(err <= TOL[precision]), dict(zip(FIELDS, err))
    d = h2.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


def test_regrid_full_size_two_level_fp32():
    """The benchmark's regrid (two-level 128^3 root + 512 patches, FP32, eps 0.02, default clustering) on a
    seeded state with a density bump: flags of the whole root bit for bit and the same boxes as the oracle;
    the root carried over bit for bit; the new level's data on a sample of new patches (no, partial and full
    overlap with the old level) against the oracle's initialisation of those patches."""
    from paper_1112_1710_amd.regrid import Spec
    spec = H.two_level()
    eps = 0.02
    _say("regrid full size")
    o = _bumped_oracle(spec, FP32, seed=61)
    h = Hierarchy(spec, FP32)
    upload_oracle_state(h, o)
    root = o.patches[0]
    n = root.n
    want_flags = oregrid.flag_cells(root.cells[0][G:G + n[2], G:G + n[1], G:G + n[0]], eps, np.float32)
    got_flags = h.flags(0, eps)[0].astype(bool)
    assert np.array_equal(got_flags, want_flags) and want_flags.sum() > 0
    want_boxes = oregrid.child_boxes(o, 0, eps, np.float32)
    h2 = regrid(h, eps)
    n0 = sum(1 for p in h2.spec.patches if p[0] == 0)
    got_boxes = [(tuple(lo), tuple(hi)) for lv, lo, hi in h2.spec.patches if lv == 1]
    assert got_boxes == [(tuple(lo), tuple(hi)) for lo, hi in want_boxes]
    _say("  flags", int(want_flags.sum()), "boxes", len(got_boxes))
    # the root is carried over unchanged
    c0, f0 = h.download(0)
    c1, f1 = h2.download(0)
    assert np.array_equal(c0, c1) and all(np.array_equal(a, b) for a, b in zip(f0, f1))
    # sample of new patches by overlap with the old level
    old1 = [q for q in o.patches if q.level == 1]

    def frac(b):
        lo, hi = np.array(b[0]), np.array(b[1])
        s = 0
        for q in old1:
            l, u = np.maximum(lo, q.lo), np.minimum(hi, q.hi)
            if np.all(u > l):
                s += int(np.prod(u - l))
        return s / int(np.prod(hi - lo))

    fr = [frac(b) for b in got_boxes]
    none = [i for i, f in enumerate(fr) if f == 0.0]
    part = [i for i, f in enumerate(fr) if 0.0 < f < 1.0]
    full = [i for i, f in enumerate(fr) if f == 1.0]
    assert none and part and full
    pick = sorted({none[0], none[-1], part[0], part[len(part) // 2], part[-1], full[0]})
    o2 = amr.Hierarchy(spec.root_n)
    for lv, lo, hi in spec.patches:
        if lv == 0:
            o2.add(lv, lo, hi)
    for i in pick:
        o2.add(1, got_boxes[i][0], got_boxes[i][1])
    o2.freeze()
    o2.patches[0].cells = root.cells.copy()
    o2.patches[0].faces = [f.copy() for f in root.faces]
    oregrid.init_from(o2, o, 1)
    num = np.zeros(8)
    den = np.zeros(8)
    for k, i in enumerate(pick):
        p = o2.patches[n0 + k]
        cells, faces = h2.download(n0 + i)
        m = o2._interior_mask(p)
        for c in range(5):
            num[c] += np.sum(np.abs(cells[c][m] - p.cells[c][m]))
            den[c] += np.sum(np.abs(p.cells[c][m]))
        for d in range(3):
            mk = o2._closure_mask(p, d)
            num[5 + d] += np.sum(np.abs(faces[d][mk] - p.faces[d][mk]))
            den[5 + d] += np.sum(np.abs(p.faces[d][mk]))
        # cells under old patches arrive bit for bit
        po = p.origin()
        for q in old1:
            lo, hi = np.maximum(p.lo, q.lo), np.minimum(p.hi, q.hi)
            if np.any(hi <= lo):
                continue
            sl = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
            assert np.array_equal(cells[(slice(None),) + sl], p.cells[(slice(None),) + sl]), (i, q.lo)
    err = num / np.maximum(den, 1e-300)
    assert np.all(err <= TOL[FP32]), dict(zip(FIELDS, err))


@pytest.mark.parametrize("precision", [FP64, FP32, FP32_MIXED])
@pytest.mark.parametrize("eps,levels", [(0.2, 3), (0.25, 2)])
def test_regrid_levels_matches_oracle(precision, eps, levels):
    """Regrid levels 1 and 2 of a three-level hierarchy coarse to fine (level 2 over the flags of the new
    level 1; at eps 0.25 the new level 1 holds no flag and the hierarchy ends there): the oracle's boxes
    on every level, its new state, old same-level data bit for bit, and one root step afterwards."""
    spec = H.small_three_level()
    _say("regrid levels", precision, eps)
    o = _bumped_oracle(spec, precision, centre=(0.28, 0.27, 0.25), width=0.06)
    h = Hierarchy(spec, precision)
    upload_oracle_state(h, o)
    dtype = np.float64 if precision == FP64 else np.float32
    want = oregrid.regrid_levels(o, eps, dtype, min_side=4)
    h2 = regrid_levels(h, eps, min_side=4)
    assert want.nlevels == levels and h2.levels == levels
    got = [(lv, tuple(int(v) for v in lo), tuple(int(v) for v in hi)) for lv, lo, hi in h2.spec.patches]
    exp = [(p.level, tuple(int(v) for v in p.lo), tuple(int(v) for v in p.hi)) for p in want.patches]
    assert got == exp
    err = rel_l1(h2, want)
    assert np.all(err <= TOL[precision]), dict(zip(FIELDS, err))
    copied = 0
    for pid, p in enumerate(want.patches):
        if p.level == 0:
            continue
        cells, _ = h2.download(pid)
        po = p.origin()
        for q in o.level_patches(p.level):
            lo, hi = np.maximum(p.lo, q.lo), np.minimum(p.hi, q.hi)
            if np.any(hi <= lo):
                continue
            sl = tuple(slice(int(lo[a] - po[a]), int(hi[a] - po[a])) for a in (2, 1, 0))
            assert np.array_equal(cells[(slice(None),) + sl], p.cells[(slice(None),) + sl]), (pid, q.lo)
            copied += 1
    assert copied > 0
    dt = want.cfl_dt()
    want.root_step(dt)
    h2.step(BATCHED, dt)
    err = rel_l1(h2, want)
    assert np.all(err <= TOL[precision]), dict(zip(FIELDS, err))
    d = h2.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


def test_evolve_with_regrids_in_the_loop_matches_oracle():
    """Regridding in the time stepping loop (FP64): three root steps of the three-level hierarchy, levels 1
    and 2 regridded after every step on both sides; the same boxes as the oracle at every regrid, the
    same dt0 and the state within the FP64 bar after every step."""
    from paper_1112_1710_amd.regrid import evolve
    from ._common import assert_parity
    spec = H.small_three_level()
    _say("evolve with regrids")
    o = _bumped_oracle(spec, FP64)
    # the same bump on the three-level hierarchy as the oracle pin uses
    h = Hierarchy(spec, FP64)
    upload_oracle_state(h, o)
    for k in range(3):
        o, olog = oregrid.evolve(o, 1, 0.05, every=1, from_level=1)
        h, hlog = evolve(h, 1, 0.05, every=1, from_level=1, mode=BATCHED)
        assert abs(hlog[0][0] - olog[0][0]) <= 1e-13 * olog[0][0]
        assert olog[0][1] is not None and hlog[0][1] == olog[0][1], k
        assert_parity(h, o, 1e-12, "evolve step %d" % k)
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
