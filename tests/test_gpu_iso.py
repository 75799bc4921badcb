"""The isothermal hydro workload on the GPU against the oracle's isothermal scheme: per-step parity
of root steps on the test hierarchies (FP64 1e-12, FP32 1e-5, relative L1 and element-wise), a plane
Riemann problem with bitwise identical transverse columns, schedule bit-identity and conservation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr  # noqa: E402
from paper_1112_1710_amd import BATCHED, FP32, FP32_MIXED, FP64, GRAPH, Hierarchy  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import G, Isothermal, PlaneRiemann, SmoothField  # noqa: E402

from ._common import assert_parity, upload_oracle_state  # noqa: E402

TOL = {FP64: 1e-12, FP32: 1e-5, FP32_MIXED: 1e-5}
CS = 0.7


def _say(*a):
    print(*a, flush=True)


def _pair(spec, field, precision):
    o = amr.build(spec, field, physics="isothermal", cs=CS)
    if precision != FP64:
        for p in o.patches:
            p.cells = p.cells.astype(np.float32).astype(np.float64)
    h = Hierarchy(spec, precision, physics="isothermal", cs=CS)
    upload_oracle_state(h, o)
    return h, o


@pytest.mark.parametrize("name", ["small_two_level", "small_three_level", "root_tiled", "minimal_patches"])
@pytest.mark.parametrize("precision", [FP64, FP32, FP32_MIXED])
def test_isothermal_root_step(name, precision):
    spec = getattr(H, name)()
    _say("isothermal", name, precision)
    h, o = _pair(spec, Isothermal(SmoothField(1115)), precision)
    dt_o = o.cfl_dt()
    dt_h = h.cfl_dt()
    assert abs(dt_h - dt_o) <= (1e-13 if precision == FP64 else 1e-6) * dt_o
    o.root_step(dt_o)
    h.step(BATCHED, dt_o)
    assert_parity(h, o, TOL[precision], "isothermal " + name, grouped=True)
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
    # energy and field slots stay zero on every interior (cells) and interior closure (faces)
    for pid, p in enumerate(o.patches):
        cells, faces = h.download(pid)
        assert np.all(cells[4][o._interior_mask(p)] == 0.0), pid
        for d in range(3):
            assert np.all(faces[d][o._closure_mask(p, d)] == 0.0), (pid, d)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_isothermal_plane_riemann(precision):
    """A shock and a rarefaction with a shear (transverse velocity jump) on a doubled periodic domain:
    per-step parity over three steps and bitwise identical transverse columns."""
    spec = H.single_patch(32)
    left = (2.5, 0.0, 0.4, 0.0, 2.5 * CS * CS, 0.0, 0.0, 0.0)
    right = (0.5, 0.0, -0.3, 0.1, 0.5 * CS * CS, 0.0, 0.0, 0.0)
    fld = Isothermal(PlaneRiemann(left, right, 5.0 / 3.0))
    _say("isothermal plane Riemann", precision)
    o = amr.build(spec, fld, physics="isothermal", cs=CS)
    h = Hierarchy(spec, precision, physics="isothermal", cs=CS)
    for step in range(3):
        if precision != FP64:
            for p in o.patches:
                p.cells = p.cells.astype(np.float32).astype(np.float64)
        upload_oracle_state(h, o)
        dt = o.cfl_dt()
        o.root_step(dt)
        h.step(BATCHED, dt)
        assert_parity(h, o, TOL[precision], "isothermal plane Riemann %d" % step, grouped=True)
        cells, _ = h.download(0)
        c = cells[:, G:G + 32, G:G + 32, G:G + 32]
        assert np.array_equal(c, np.broadcast_to(c[:, :1, :1, :], c.shape)), step


def test_isothermal_graph_equals_batched_and_conserves():
    spec = H.small_three_level()
    _say("isothermal schedules")
    fld = Isothermal(SmoothField(1116))
    a = Hierarchy(spec, FP64, physics="isothermal", cs=CS)
    b = Hierarchy(spec, FP64, physics="isothermal", cs=CS)
    a.set_field(fld)
    b.set_field(fld)
    s0, c0 = a.conservation()
    for _ in range(3):
        dt = a.step(BATCHED)
        assert b.step(GRAPH) == dt
    o = amr.build(spec)
    for pid, p in enumerate(o.patches):
        ca, _ = a.download(pid)
        cb, _ = b.download(pid)
        m = o._interior_mask(p)
        assert np.array_equal(ca[:, m], cb[:, m]), pid
    s1, c1 = a.conservation()
    tot0, tot1 = s0 + c0, s1 + c1
    scale = sum(abs(x) for x in tot0[:4])
    assert np.all(np.abs(tot1[:4] - tot0[:4]) <= 1e-14 * scale)
