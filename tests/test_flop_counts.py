"""The algorithmic flop counts the benchmark prices its ALU-bound kernel classes with, counted on the
oracle's formulas.

Every NumPy add, subtract, multiply, divide, square root, minimum and maximum counts once per array
element it produces; absolute values, negations, signs, comparisons and selects count nothing (on the
GPU they are instruction modifiers and selects).  The oracle evaluates every HLLD region's state and
flux and then selects one, so its Riemann-solver count is that of the whole formula set.  The stages
are composed from the oracle's own functions in the order its single-patch advance applies them, and
the composition is checked to add up to a count of that advance itself, so each stage's figure is the
method's arithmetic for one cell (or one face) computed once.
"""
import contextlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import mhd  # noqa: E402
from oracle.mhd import sh  # noqa: E402

COUNTED = {np.add, np.subtract, np.multiply, np.true_divide, np.divide, np.sqrt, np.minimum, np.maximum,
           np.power, np.square, np.reciprocal}


def _plain(x):
    if isinstance(x, _Ops):
        return x.view(np.ndarray)
    if isinstance(x, (list, tuple)):
        return type(x)(_plain(y) for y in x)
    if isinstance(x, dict):
        return {k: _plain(v) for k, v in x.items()}
    return x


def _wrap(x):
    if isinstance(x, np.ndarray) and not isinstance(x, _Ops):
        return x.view(_Ops)
    if isinstance(x, (list, tuple)):
        return type(x)(_wrap(y) for y in x)
    return x


class _Ops(np.ndarray):
    """Array that counts the elements produced by the arithmetic ufuncs applied to it."""
    n = 0

    def __array_ufunc__(self, ufunc, method, *inputs, **kw):
        if "out" in kw:
            kw["out"] = tuple(_plain(o) for o in kw["out"])
        res = getattr(ufunc, method)(*_plain(list(inputs)), **kw)
        if method == "__call__" and ufunc in COUNTED:
            _Ops.n += int(np.size(res[0] if isinstance(res, tuple) else res))
        return _wrap(res)

    def __array_function__(self, func, types, args, kwargs):
        if func is np.cross:  # the product's arithmetic, written out so that it is counted
            a, b = args[0], args[1]
            return _wrap(np.stack(_plain([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                                          a[0] * b[1] - a[1] * b[0]])))
        return _wrap(func(*_plain(list(args)), **_plain(kwargs)))


def _count(fn):
    _Ops.n = 0
    fn()
    return _Ops.n


@contextlib.contextmanager
def _counting_oracle():
    """The oracle's functions with their results wrapped, so that arithmetic on arrays they fill
    element by element (the physical flux, the Riemann fluxes) is counted too."""
    names = ("flux", "hlld", "mc_slope", "prim_from_cons", "cons_from_prim", "cell_centred_b", "edge_emf")
    saved = {n: getattr(mhd, n) for n in names}
    for n, fn in saved.items():
        setattr(mhd, n, lambda *a, _fn=fn, **k: _wrap(_fn(*a, **k)))
    try:
        yield
    finally:
        for n, fn in saved.items():
            setattr(mhd, n, fn)


def _patch(n=10, seed=3):
    """A padded periodic patch with a smooth positive state and a divergence-free-ish field."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    rho = 1.0 + 0.1 * rng.random(shape)
    m = 0.1 * rng.standard_normal((3,) + shape)
    faces = [np.full(shape, 1.0 if d == 0 else 0.0) + 0.05 * rng.standard_normal(shape) for d in range(3)]
    kin = 0.5 * np.sum(m ** 2, axis=0) / rho
    mag = 0.5 * sum((0.5 * (f + np.roll(f, -1, axis=2 - d))) ** 2 for d, f in enumerate(faces))
    e = 1.0 / (5.0 / 3.0 - 1.0) + kin + mag
    cells = np.concatenate([rho[None], m, e[None]])
    return cells, faces


def _stage_counts():
    """Per-element counts of the advance's stages, composed from the oracle's functions in its order."""
    cells, faces = _patch()
    nel = cells[0].size
    gamma, dt, dx = 5.0 / 3.0, 1e-3, np.full(3, 0.1)
    region = ((2, 2, 2), (cells.shape[3] - 2,) * 3)
    u, b = _wrap(cells), [_wrap(f) for f in faces]
    st = {}

    def primitives():
        st["bc"] = mhd.cell_centred_b(b)
        st["w"] = mhd.prim_from_cons(u, st["bc"], gamma)
        st["ec"] = -np.cross(st["w"][1:4], st["bc"], axis=0)

    def hancock():
        w = st["w"]
        st["slope"] = [mhd.mc_slope(w - sh(w, d, -1), sh(w, d, 1) - w) for d in range(3)]
        du = _wrap(np.zeros((8,) + u.shape[1:]))
        for d in range(3):
            fp = mhd.flux(w + 0.5 * st["slope"][d], d, gamma)
            fm = mhd.flux(w - 0.5 * st["slope"][d], d, gamma)
            du -= (0.5 * dt / dx[d]) * (fp - fm)
        st["du"] = du

    def half_step_faces():
        ec = st["ec"]
        ebar = []
        for e in range(3):
            a, c = (e + 1) % 3, (e + 2) % 3
            ebar.append(0.25 * (ec[e] + sh(ec[e], a, -1) + sh(ec[e], c, -1) + sh(sh(ec[e], a, -1), c, -1)))
        bh = []
        for d in range(3):
            a, c = (d + 1) % 3, (d + 2) % 3
            curl = (sh(ebar[c], a, 1) - ebar[c]) / dx[a] - (sh(ebar[a], c, 1) - ebar[a]) / dx[c]
            bh.append(b[d] - 0.5 * dt * curl)
        st["bh"] = bh

    def reference_emf():
        uh = _wrap(np.concatenate(_plain([u, st["bc"]]))) + st["du"]
        vh = uh[1:4] / uh[0]
        st["eref"] = -np.cross(vh, mhd.cell_centred_b(st["bh"]), axis=0)

    def face_fluxes():
        w, du, fl = st["w"], st["du"], []
        for d in range(3):
            up = mhd.cons_from_prim(w + 0.5 * st["slope"][d], gamma) + du
            um = mhd.cons_from_prim(w - 0.5 * st["slope"][d], gamma) + du
            wp = mhd.prim_from_cons(up[:5], up[5:], gamma)
            wm = mhd.prim_from_cons(um[:5], um[5:], gamma)
            fl.append(mhd.hlld(sh(wp, d, -1), wm, st["bh"][d], d, gamma))
        st["fl"] = fl

    def edges():
        fl = st["fl"]
        st["edges"] = [mhd.edge_emf(-fl[(e + 1) % 3][5 + (e + 2) % 3], fl[(e + 2) % 3][5 + (e + 1) % 3],
                                    st["eref"][e], fl[(e + 1) % 3][0], fl[(e + 2) % 3][0], (e + 1) % 3, (e + 2) % 3)
                       for e in range(3)]

    def update():
        fl, ed = st["fl"], st["edges"]
        div = _wrap(np.zeros_like(cells))
        for d in range(3):
            div += (sh(fl[d][:5], d, 1) - fl[d][:5]) / dx[d]
        sel = (slice(None),) + mhd._sel(region)
        st["u_new"] = u[sel] - dt * div[sel]
        for d in range(3):
            a, c = (d + 1) % 3, (d + 2) % 3
            curl = (sh(ed[c], a, 1) - ed[c]) / dx[a] - (sh(ed[a], c, 1) - ed[a]) / dx[c]
            fs = mhd._face_sel(region, d)
            st.setdefault("b_new", []).append(b[d][fs] - dt * curl[fs])

    with np.errstate(all="ignore"), _counting_oracle():
        stages = [("primitives", primitives), ("hancock", hancock), ("half_step_faces", half_step_faces),
                  ("reference_emf", reference_emf), ("face_fluxes", face_fluxes), ("edges", edges), ("update", update)]
        per = {name: _count(fn) / nel for name, fn in stages}
        whole = _count(lambda: mhd.advance(u, b, list(dx), dt, region, gamma)) / nel
    return per, whole


def test_stage_counts_add_up_to_the_oracle_advance():
    per, whole = _stage_counts()
    assert sum(per.values()) == whole, (per, whole)
    # the pointwise pieces the stages are made of
    assert per["primitives"] == 6 + 19 + 9    # cell-centred field, conserved -> primitive, cell EMF


def test_benchmark_flop_prices_equal_the_counted_stages():
    """bench.py's algorithmic flops: the fused first stages per cell of the grown-by-2 region
    (primitives and cell EMFs) and of the grown-by-1 region (half-step faces, Hancock increments,
    reference EMF); the flux stage per face (the two face states' conversions with the increment, and
    the Riemann solver).  The limited slopes belong to the Hancock stage and are priced once per cell
    and axis, although the flux kernel recomputes them at every face."""
    import bench
    per, _ = _stage_counts()
    assert bench.PRIMHALF_FLOPS["grown2"] == round(per["primitives"])
    assert bench.PRIMHALF_FLOPS["grown1"] == round(per["hancock"] + per["half_step_faces"] + per["reference_emf"])
    assert bench.ALU_BOUND["flux"] == round(per["face_fluxes"] / 3)
