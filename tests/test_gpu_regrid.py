"""Regridding on the GPU against the oracle: refinement flags bit for bit, the boxes laid over
them, the new finest level's initial data (copied overlaps bit for bit, prolongated cells to the
parity tolerance) and a root step of the regridded hierarchy."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr, regrid as oregrid  # noqa: E402
from paper_1112_1710_amd import BATCHED, FP32, FP64, Hierarchy  # noqa: E402
from paper_1112_1710_amd.regrid import new_spec, regrid  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import G, SmoothField  # noqa: E402

from ._common import FIELDS, rel_l1, upload_oracle_state  # noqa: E402

TOL = {FP64: 1e-12, FP32: 1e-5}


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
