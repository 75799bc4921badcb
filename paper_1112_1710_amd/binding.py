"""ctypes binding of libamrx (argument marshalling only; every step runs in the library)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrx.so")

FP64, FP32, FP32_MIXED = 0, 1, 2
PLAIN, BATCHED, GRAPH, PERSISTENT, CONCURRENT, LAYERED = 0, 1, 2, 3, 4, 5
G = 4

KERNEL_CLASSES = ("prim", "bhalf", "pred", "flux", "edge", "update", "copy", "prolong", "restrict",
                  "fluxcorr", "emfcorr", "sync", "cfl", "cons", "primhalf", "edgeupd")
(TUNE_FUSED, TUNE_TILE, TUNE_EXTEND_ALL, TUNE_PAIR, TUNE_FUSED_EU, TUNE_TILE_EU, TUNE_GHOSTS, TUNE_FLUX_SPLIT,
 TUNE_UPDATE_NT) = range(9)

_ERRORS = {-1: "EINVAL", -2: "ENEST", -3: "EOVERLAP", -4: "ENOMEM", -5: "EHIP", -6: "ESTATE", -7: "EPHYS"}


class AmrxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("root_n", C.c_int * 3), ("max_level", C.c_int), ("ratio", C.c_int), ("nghost", C.c_int),
                ("gamma", C.c_double), ("cfl", C.c_double), ("precision", C.c_int), ("stream", C.c_void_p)]


_lib = None

EXPORTS = {
    "hier_create": ([C.POINTER(Desc), C.POINTER(C.c_void_p)], C.c_int),
    "hier_destroy": ([C.c_void_p], C.c_int),
    "hier_last_error": ([C.c_void_p], C.c_char_p),
    "hier_set_isothermal": ([C.c_void_p, C.c_double], C.c_int),
    "patch_add": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "hier_finalize": ([C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)], C.c_int),
    "patch_layout": ([C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_int)], C.c_int),
    "patch_current": ([C.c_void_p, C.c_int, C.POINTER(C.c_int)], C.c_int),
    "hier_bind": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t], C.c_int),
    "level_ghost_fill": ([C.c_void_p, C.c_int, C.c_int], C.c_int),
    "advance_level": ([C.c_void_p, C.c_int, C.c_double, C.c_int], C.c_int),
    "restrict_level": ([C.c_void_p, C.c_int], C.c_int),
    "sync_level": ([C.c_void_p, C.c_int], C.c_int),
    "cfl_dt": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "hier_step": ([C.c_void_p, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "hier_steps": ([C.c_void_p, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)],
                   C.c_int),
    "hier_conservation": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "hier_diag": ([C.c_void_p, C.POINTER(C.c_double), C.c_int], C.c_int),
    "hier_timing_enable": ([C.c_void_p, C.c_int], C.c_int),
    "hier_timing_read": ([C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)], C.c_int),
    "hier_step_work": ([C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)], C.c_int),
    "hier_flag_bytes": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "hier_flag": ([C.c_void_p, C.c_int, C.c_double, C.c_void_p], C.c_int),
    "amrx_cluster": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int), C.c_int,
                      C.POINTER(C.c_int)], C.c_int),
    "hier_regrid_boxes": ([C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_int), C.c_int,
                           C.POINTER(C.c_int)], C.c_int),
    "hier_init_from_bytes": ([C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "hier_init_from": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t], C.c_int),
    "hier_init_from_levels_bytes": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "hier_init_from_levels": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t], C.c_int),
    "hier_init_from_levels_static": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "hier_debug_concurrent": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int)], C.c_int),
    "hier_debug_layers": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "hier_debug_schedule": ([C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "hier_debug_sources": ([C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_longlong)], C.c_int),
    "hier_debug_prolong_cells": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int], C.c_int),
    "hier_tune_set": ([C.c_void_p, C.c_int, C.c_int, C.c_int], C.c_int),
    "hier_tune_get": ([C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int)], C.c_int),
    "hier_tile_table": ([C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int], C.c_int),
    "hier_tune_time": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "hier_tune_time_eu": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "hier_tune_time_flux": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)], C.c_int),
    "hier_debug_tasks": ([C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int],
                         C.c_int),
    "hier_debug_update_box": ([C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
}


def tile_table(precision):
    """[(tx, ty, tz, lds_bytes)] of the fused first-three-stage kernel; lds_bytes 0 = not allowed."""
    lib = load_library()
    n = C.c_int()
    if lib.hier_tile_table(precision, C.byref(n), None, None, 0) != 0:
        raise AmrxError(-1, "hier_tile_table")
    shapes = (C.c_int * (3 * n.value))()
    lds = (C.c_int * n.value)()
    lib.hier_tile_table(precision, C.byref(n), shapes, lds, n.value)
    return [(shapes[3 * t], shapes[3 * t + 1], shapes[3 * t + 2], lds[t]) for t in range(n.value)]


def load_library(path=LIB_PATH):
    """Load libamrx.so (raises if it has not been built: no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libamrx.so not built at {path}; run __graft_entry__.build()")
    # torch carries its own HIP runtime; loading torch first makes the library's HIP dependency
    # resolve to that copy.  Loaded the other way round, the process maps two runtimes and the
    # library's one finds no device.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (args, res) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _i3(v):
    return (C.c_int * 3)(*[int(x) for x in v])


class Hierarchy:
    """A static patch hierarchy bound to device arenas allocated by PyTorch.

    ``spec`` is any object with ``root_n`` and ``patches`` = [(level, lo, hi), ...].
    With ``device=None`` only the host bookkeeping is built (no HIP call is made).
    ``extend_all=True`` extends the substep-0 update region of refined patches over every side
    (each grid treated as isolated) instead of only over sides lacking same-level cover.
    ``ghosts="time"`` selects coarse-time-derivative ghosts (interior-only updates; later-substep
    ghosts prolongated from the parent moved along its time derivative) instead of extended
    ghost regions.  ``physics="isothermal"`` selects the isothermal hydro workload with sound
    speed ``cs`` (hier_set_isothermal; its states keep E and the face fields at zero).
    """

    def __init__(self, spec, precision=FP64, gamma=5.0 / 3.0, cfl=0.4, device="cuda:0", stream=None,
                 extend_all=False, ghosts="extended", physics="mhd", cs=1.0):
        self.lib = load_library()
        self.precision = precision
        self.spec = spec
        d = Desc()
        d.root_n = _i3(spec.root_n)
        levels = 1 + max(p[0] for p in spec.patches)
        d.max_level = levels - 1
        d.ratio, d.nghost = 2, G
        d.gamma, d.cfl, d.precision = gamma, cfl, precision
        self._torch = None
        if device is not None:
            import torch
            self._torch = torch
            if stream is None:
                # a stream of its own (default priority): every library call and every
                # upload/download of this hierarchy is ordered on it; graph capture needs it
                stream = torch.cuda.Stream(device=torch.device(device))
            self.stream = stream
            d.stream = C.c_void_p(stream.cuda_stream)
        else:
            d.stream = None
        h = C.c_void_p()
        self._check(self.lib.hier_create(C.byref(d), C.byref(h)), None)
        self.h = h
        self.ids = []
        for lv, lo, hi in spec.patches:
            pid = C.c_int()
            self._check(self.lib.patch_add(self.h, int(lv), _i3(lo), _i3(hi), C.byref(pid)))
            self.ids.append(pid.value)
        if physics not in ("mhd", "isothermal"):
            raise ValueError("physics must be 'mhd' or 'isothermal'")
        self.physics, self.cs = physics, float(cs)
        if physics == "isothermal":
            self._check(self.lib.hier_set_isothermal(self.h, float(cs)))
        if extend_all:
            self._check(self.lib.hier_tune_set(self.h, 0, TUNE_EXTEND_ALL, 1))
        if ghosts not in ("extended", "time"):
            raise ValueError("ghosts must be 'extended' or 'time'")
        self.ghosts = ghosts
        if ghosts == "time":
            self._check(self.lib.hier_tune_set(self.h, 0, TUNE_GHOSTS, 1))
        sb, cb = C.c_size_t(), C.c_size_t()
        self._check(self.lib.hier_finalize(self.h, C.byref(sb), C.byref(cb)))
        self.state_bytes, self.scratch_bytes = sb.value, cb.value
        self.levels = levels
        self.device = device
        if device is not None:
            torch = self._torch
            self.state = torch.empty(self.state_bytes, dtype=torch.uint8, device=device)
            self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
            self._check(self.lib.hier_bind(self.h, C.c_void_p(self.state.data_ptr()), self.state_bytes,
                                           C.c_void_p(self.scratch.data_ptr()), self.scratch_bytes))
            self.real = self.state.view(torch.float64 if precision == FP64 else torch.float32)

    # ------------------------------------------------------------------ errors
    def _check(self, rc, h=0):
        if rc != 0:
            hh = self.h if h == 0 else h
            msg = self.lib.hier_last_error(hh).decode() if hh is not None else ""
            raise AmrxError(rc, msg)

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                self.lib.hier_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ------------------------------------------------------------------ layout
    def layout(self, pid, which):
        offs = (C.c_size_t * 8)()
        dims = (C.c_int * 3)()
        self._check(self.lib.patch_layout(self.h, pid, which, offs, dims))
        return list(offs), (dims[2], dims[1], dims[0])

    def current(self, pid):
        w = C.c_int()
        self._check(self.lib.patch_current(self.h, pid, C.byref(w)))
        return w.value

    def _views(self, pid, which=None):
        if which is None:
            which = self.current(pid)
        offs, shape = self.layout(pid, which)
        esize = 8 if self.precision == FP64 else 4
        vol = shape[0] * shape[1] * shape[2]
        out = []
        for m in range(8):
            o = offs[m] // esize
            out.append(self.real[o:o + vol].view(*shape))
        return out

    def upload(self, pid, cells, faces, which=None):
        """Copy float64 host arrays (5, Z, Y, X) and [bx, by, bz] into a patch buffer (default: current)."""
        torch = self._torch
        views = self._views(pid, which)
        dt = views[0].dtype
        with torch.cuda.stream(self.stream):
            for m in range(5):
                views[m].copy_(torch.from_numpy(np.ascontiguousarray(cells[m])).to(dt))
            for d in range(3):
                views[5 + d].copy_(torch.from_numpy(np.ascontiguousarray(faces[d])).to(dt))

    def download(self, pid, which=None):
        """(cells (5, Z, Y, X), [bx, by, bz]) of a patch as float64 NumPy arrays."""
        views = self._views(pid, which)
        with self._torch.cuda.stream(self.stream):
            arrs = [v.double().cpu().numpy() for v in views]
        return np.stack(arrs[:5]), arrs[5:]

    def download_box(self, pid, lo, hi, which=None):
        """Entries [lo, hi) (padded (x, y, z) indices, node box) of a patch buffer as float64 arrays."""
        views = self._views(pid, which)
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        with self._torch.cuda.stream(self.stream):
            arrs = [v[sl].double().cpu().numpy() for v in views]
        return np.stack(arrs[:5]), arrs[5:]

    def set_field(self, field):
        root = tuple(int(x) for x in self.spec.root_n)
        for pid, (lv, lo, hi) in zip(self.ids, self.spec.patches):
            st = field.patch(lv, root, tuple(lo), tuple(hi))
            self.upload(pid, st.cells, st.faces)
        self.synchronize()

    def synchronize(self):
        if self._torch is not None:
            self.stream.synchronize()

    # ------------------------------------------------------------------ operations
    def ghost_fill(self, level, substep):
        self._check(self.lib.level_ghost_fill(self.h, level, substep))

    def advance(self, level, dt, substep):
        self._check(self.lib.advance_level(self.h, level, float(dt), substep))

    def restrict(self, fine_level):
        self._check(self.lib.restrict_level(self.h, fine_level))

    def sync(self, level):
        self._check(self.lib.sync_level(self.h, level))

    def cfl_dt(self):
        v = C.c_double()
        self._check(self.lib.cfl_dt(self.h, C.byref(v)))
        return v.value

    def step(self, mode=BATCHED, dt=0.0):
        v = C.c_double(float(dt))
        self._check(self.lib.hier_step(self.h, mode, C.byref(v)))
        return v.value

    def steps(self, n, mode=BATCHED, dt=0.0):
        """`n` root steps with one synchronisation at the end (hier_steps): (time advanced, last dt)."""
        t = C.c_double()
        last = C.c_double()
        self._check(self.lib.hier_steps(self.h, mode, int(n), float(dt), C.byref(t), C.byref(last)))
        return t.value, last.value

    def conservation(self):
        s = (C.c_double * 8)()
        c = (C.c_double * 8)()
        self._check(self.lib.hier_conservation(self.h, s, c))
        return np.array(list(s)), np.array(list(c))

    def diag(self):
        out = (C.c_double * 3)()
        self._check(self.lib.hier_diag(self.h, out, 3))
        return {"sync_flux_max": out[0], "sync_face_max": out[1], "phys_flag": out[2]}

    # ------------------------------------------------------------------ measurement
    def timing(self, on):
        self._check(self.lib.hier_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        n = len(KERNEL_CLASSES)
        ms = (C.c_double * n)()
        cnt = (C.c_int * n)()
        self._check(self.lib.hier_timing_read(self.h, n, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def step_work(self):
        n = len(KERNEL_CLASSES)
        u = (C.c_double * n)()
        cnt = (C.c_int * n)()
        self._check(self.lib.hier_step_work(self.h, n, u, cnt))
        return {k: (u[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}

    # ------------------------------------------------------------------ tuning
    def tune_set(self, param, value, level=-1):
        """Set a tuning parameter for `level` (-1: every level)."""
        self._check(self.lib.hier_tune_set(self.h, level, param, int(value)))

    def tune_get(self, param, level=0):
        v = C.c_int()
        self._check(self.lib.hier_tune_get(self.h, level, param, C.byref(v)))
        return v.value

    def tune_time(self, level, substep, tile, reps=5):
        ms = C.c_double()
        self._check(self.lib.hier_tune_time(self.h, level, substep, tile, reps, C.byref(ms)))
        return ms.value

    def tune_time_eu(self, level, tile, reps=5):
        """Mean ms of the edge EMF and update stages of substep 0 (tile -1: staged, -2: staged with the
        non-temporal update); between steps only."""
        ms = C.c_double()
        self._check(self.lib.hier_tune_time_eu(self.h, level, tile, reps, C.byref(ms)))
        return ms.value

    def tune_time_flux(self, level, split, reps=5):
        """Mean ms of the flux stage of substep 0 in FP32_MIXED's two-launch (split 1) or one-launch (0)
        form; between steps only."""
        ms = C.c_double()
        self._check(self.lib.hier_tune_time_flux(self.h, level, int(split), reps, C.byref(ms)))
        return ms.value

    # ------------------------------------------------------------------ bookkeeping exports
    def update_box(self, pid, substep):
        """The update region ((lo), (hi)) in padded cell indices of a patch at `substep`."""
        lo, hi = (C.c_int * 3)(), (C.c_int * 3)()
        self._check(self.lib.hier_debug_update_box(self.h, pid, substep, lo, hi))
        return tuple(lo), tuple(hi)

    def debug_tasks(self, level, substep, stage):
        """Batched task list of an advance stage: (n, 9) int array of (patch, axis, lo[3], hi[3], first block)."""
        cnt = C.c_int(0)
        self._check(self.lib.hier_debug_tasks(self.h, level, substep, stage, C.byref(cnt), None, 0))
        out = (C.c_int * (9 * max(cnt.value, 1)))()
        self._check(self.lib.hier_debug_tasks(self.h, level, substep, stage, C.byref(cnt), out, cnt.value))
        return np.frombuffer(out, dtype=np.int32, count=9 * cnt.value).reshape(cnt.value, 9).copy()

    def debug_sources(self, pid, kind):
        offs, shape = self.layout(pid, 0)
        vol = shape[0] * shape[1] * shape[2]
        out = (C.c_longlong * vol)()
        self._check(self.lib.hier_debug_sources(self.h, pid, kind, out))
        return np.ctypeslib.as_array(out).reshape(shape).copy()

    def debug_schedule(self, fixed_dt=False, nworkgroups=1024):
        """Persistent schedule tables: nodes (N, 12), preds, items (M, 4), queues (Q, 2)."""
        sizes = (C.c_int * 4)()
        self._check(self.lib.hier_debug_schedule(self.h, int(fixed_dt), nworkgroups, sizes, None, None, None, None))
        nn, npr, ni, nq = (sizes[i] for i in range(4))
        nodes = (C.c_int * max(1, 12 * nn))()
        preds = (C.c_int * max(1, npr))()
        items = (C.c_int * max(1, 4 * ni))()
        queues = (C.c_int * max(1, 2 * nq))()
        self._check(self.lib.hier_debug_schedule(self.h, int(fixed_dt), nworkgroups, sizes, nodes, preds, items, queues))
        a = np.ctypeslib.as_array
        return (a(nodes)[:12 * nn].reshape(nn, 12).copy(), a(preds)[:npr].copy(),
                a(items)[:4 * ni].reshape(ni, 4).copy(), a(queues)[:2 * nq].reshape(nq, 2).copy())

    # ------------------------------------------------------------------ regridding
    def flag_array(self, level, eps):
        """Refinement flags of `level` (one byte per padded cell of every patch, see hier_flag) on the host."""
        torch = self._torch
        nb = C.c_size_t()
        self._check(self.lib.hier_flag_bytes(self.h, C.byref(nb)))
        with torch.cuda.stream(self.stream):
            buf = torch.zeros(max(1, nb.value), dtype=torch.uint8, device=self.device)
        self._check(self.lib.hier_flag(self.h, int(level), float(eps), C.c_void_p(buf.data_ptr())))
        self.synchronize()
        return buf.cpu().numpy()

    def flags(self, level, eps):
        """{patch id: interior flags [z, y, x] (uint8)} of the patches of `level`."""
        arr = self.flag_array(level, eps)
        esize = 8 if self.precision == FP64 else 4
        out = {}
        for pid, (lv, lo, hi) in enumerate(self.spec.patches):
            if lv != level:
                continue
            offs, shape = self.layout(pid, 0)
            base = offs[0] // esize // 16
            vol = shape[0] * shape[1] * shape[2]
            full = arr[base:base + vol].reshape(shape)
            n = [hi[a] - lo[a] for a in range(3)]
            out[pid] = full[G:G + n[2], G:G + n[1], G:G + n[0]].copy()
        return out

    def regrid_boxes(self, level, eps, min_side=4, efficiency=0.7):
        """Level-(level+1) boxes [((lo), (hi))] laid over the flagged cells of `level` (flags on the GPU,
        buffer, nesting and clustering on the host)."""
        return self.boxes_from_flags(level, self.flag_array(level, eps), min_side, efficiency)

    def boxes_from_flags(self, level, flag_array, min_side=4, efficiency=0.7):
        """Host part of regrid_boxes: buffer, nesting layer and clustering of a downloaded flag array."""
        arr = np.ascontiguousarray(flag_array, dtype=np.uint8)
        cap = 1 << 16
        boxes = (C.c_int * (6 * cap))()
        n = C.c_int()
        self._check(self.lib.hier_regrid_boxes(self.h, int(level), arr.ctypes.data_as(C.c_void_p), int(min_side),
                                               float(efficiency), boxes, cap, C.byref(n)))
        b = np.ctypeslib.as_array(boxes)[:6 * n.value].reshape(n.value, 6)
        return [(tuple(int(x) for x in r[:3]), tuple(int(x) for x in r[3:])) for r in b]

    def init_from_bytes(self, src, level, below=None):
        """Workspace bytes of init_from (pure host)."""
        nb = C.c_size_t()
        b = src if below is None else below
        self._check(self.lib.hier_init_from_levels_bytes(self.h, b.h, src.h, int(level), C.byref(nb)))
        return nb.value

    def init_from(self, src, level, below=None):
        """Fill this hierarchy, whose finest level is `level`: the lower levels from the identical patches
        of `below` (default: src), level `level` from src's overlapping patches of that level and by
        prolongation elsewhere (hier_init_from_levels)."""
        torch = self._torch
        b = src if below is None else below
        nb = self.init_from_bytes(src, level, below)
        with torch.cuda.stream(self.stream):
            work = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        addr = (work.data_ptr() + 255) & ~255
        src.synchronize()
        b.synchronize()
        self._check(self.lib.hier_init_from_levels(self.h, b.h, src.h, int(level), C.c_void_p(addr), nb))
        del work

    def init_from_static(self, src, level, below=None):
        """init_from without a workspace allocation: the library's static per-GPU workspace
        (hier_init_from_levels_static; AmrxError EINVAL when the transfer lists exceed it)."""
        b = src if below is None else below
        src.synchronize()
        b.synchronize()
        self._check(self.lib.hier_init_from_levels_static(self.h, b.h, src.h, int(level)))

    def debug_concurrent(self, fixed_dt=False):
        """Concurrent schedule capture plan: nodes (N, 12), preds, ops (K, 4: kind, stream, event,
        node), side streams, events."""
        sizes = (C.c_int * 5)()
        self._check(self.lib.hier_debug_concurrent(self.h, int(fixed_dt), sizes, None, None, None))
        nn, npr, nop = sizes[0], sizes[1], sizes[2]
        nodes = (C.c_int * max(1, 12 * nn))()
        preds = (C.c_int * max(1, npr))()
        ops = (C.c_int * max(1, 4 * nop))()
        self._check(self.lib.hier_debug_concurrent(self.h, int(fixed_dt), sizes, nodes, preds, ops))
        a = np.ctypeslib.as_array
        return (a(nodes)[:12 * nn].reshape(nn, 12).copy(), a(preds)[:npr].copy(),
                a(ops)[:4 * nop].reshape(nop, 4).copy(), sizes[3], sizes[4])

    def debug_layers(self, fixed_dt=False):
        """Layered schedule: the first item of each layer (layers + 1) and the items (M, 4) in launch order."""
        sizes = (C.c_int * 2)()
        self._check(self.lib.hier_debug_layers(self.h, int(fixed_dt), sizes, None, None))
        nl, ni = sizes[0], sizes[1]
        first = (C.c_int * (nl + 1))()
        items = (C.c_int * max(1, 4 * ni))()
        self._check(self.lib.hier_debug_layers(self.h, int(fixed_dt), sizes, first, items))
        a = np.ctypeslib.as_array
        return a(first)[:nl + 1].copy(), a(items)[:4 * ni].reshape(ni, 4).copy()

    def debug_prolong_cells(self, pid):
        cnt = C.c_int()
        self._check(self.lib.hier_debug_prolong_cells(self.h, pid, C.byref(cnt), None, 0))
        n = cnt.value
        buf = (C.c_int * max(1, 3 * n))()
        self._check(self.lib.hier_debug_prolong_cells(self.h, pid, C.byref(cnt), buf, n))
        return np.ctypeslib.as_array(buf)[:3 * n].reshape(n, 3).copy()


def cluster_flags(flags, min_side=4, efficiency=0.7):
    """Berger-Rigoutsos boxes [((lo x, y, z), (hi x, y, z))] of a flag array f[z, y, x] (amrx_cluster)."""
    lib = load_library()
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    nz, ny, nx = f.shape
    cap = max(16, f.size)
    boxes = (C.c_int * (6 * cap))()
    n = C.c_int()
    rc = lib.amrx_cluster(f.ctypes.data_as(C.c_void_p), nx, ny, nz, int(min_side), float(efficiency), boxes, cap,
                          C.byref(n))
    if rc != 0:
        raise AmrxError(rc, "amrx_cluster")
    b = np.ctypeslib.as_array(boxes)[:6 * n.value].reshape(n.value, 6)
    return [(tuple(int(x) for x in r[:3]), tuple(int(x) for x in r[3:])) for r in b]
