"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle cannot advance a whole 512-patch hierarchy or a 256^3 patch in a test,
so outputs are sampled: whole patches (ghost fill, prolongation, substep-0
advance) of the two-level workload and windows of the 256^3 advance are
recomputed by the oracle from the GPU's own input, and whole-hierarchy
properties (composite conservation, div B, bit-zero sync) are checked at full
size.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr, mhd  # noqa: E402
from paper_1112_1710_amd import BATCHED, FP32, FP64, GRAPH, Hierarchy  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import G, SmoothField  # noqa: E402


def _say(*a):
    print(*a, flush=True)


def _rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300))


def _fused_config(h):
    """Both fused kernels on every level, with the tiles the autotuner keeps for the benchmarked
    two-level workload's refined level (8x8x4 first stages, 32x4x4 edge/update)."""
    from paper_1112_1710_amd import binding
    shapes = [row[:3] for row in binding.tile_table(h.precision)]
    h.tune_set(binding.TUNE_FUSED, 1)
    h.tune_set(binding.TUNE_TILE, shapes.index((8, 8, 4)))
    h.tune_set(binding.TUNE_FUSED_EU, 1)
    h.tune_set(binding.TUNE_TILE_EU, shapes.index((32, 4, 4)))


@pytest.mark.parametrize("config", ["staged", "fused"])
@pytest.mark.parametrize("precision", [FP32, FP64])
def test_two_level_sampled_patches(precision, config):
    """Ghost fill + prolongation and the extended substep-0 advance of sampled level-1 patches, then
    their substep-1 ghost fill and advance."""
    spec = H.two_level()
    _say("two-level full size, sampled patches", precision, config)
    field = SmoothField(1112)
    h = Hierarchy(spec, precision)
    if config == "fused":
        _fused_config(h)
    h.set_field(field)
    o = amr.Hierarchy(spec.root_n)
    for lv, lo, hi in spec.patches:
        o.add(lv, lo, hi)
    o.freeze()
    rnd = (lambda a: a.astype(np.float32).astype(np.float64)) if precision == FP32 else (lambda a: a)
    root = o.patches[0]
    st = field.patch(0, spec.root_n, (0, 0, 0), spec.root_n)
    root.cells, root.faces = rnd(st.cells), [rnd(f) for f in st.faces]
    samples = [1, 77, 200, 311, 512]
    for pid in samples:
        p = o.patches[pid]
        st = field.patch(1, spec.root_n, tuple(p.lo), tuple(p.hi))
        p.cells, p.faces = rnd(st.cells), [rnd(f) for f in st.faces]
    # same-level sources of the sampled patches need their neighbours' interiors
    need = set()
    for pid in samples:
        src = o.cell_src[pid]
        need |= set(int(v >> 32) for v in np.unique(src[src >= 0]))
        for d in range(3):
            fs = o.face_src[pid][d]
            need |= set(int(v >> 32) for v in np.unique(fs[fs >= 0]))
    for pid in need - set(samples):
        p = o.patches[pid]
        st = field.patch(1, spec.root_n, tuple(p.lo), tuple(p.hi))
        p.cells, p.faces = rnd(st.cells), [rnd(f) for f in st.faces]
    dt = 2.0e-3
    # GPU: root ghost fill + advance (its pre-advance buffer feeds prolongation), level-1 ghost fill
    h.ghost_fill(0, 0)
    h.advance(0, dt, 0)
    h.ghost_fill(1, 0)
    h.synchronize()
    o.ghost_fill(0, 0)
    root.old_cells, root.old_faces = root.cells, root.faces
    tol_ghost = 1e-13 if precision == FP64 else 2e-6
    pre = {}
    for pid in samples:
        p = o.patches[pid]
        o._copy_from_sources(p)
        o._prolong(p)
        cells, faces = h.download(pid)
        # compare the region the substep-0 stencil reads: the update region grown by 2
        ulo, uhi = h.update_box(pid, 0)
        v = (slice(None), slice(ulo[2] - 2, uhi[2] + 2), slice(ulo[1] - 2, uhi[1] + 2), slice(ulo[0] - 2, uhi[0] + 2))
        assert _rel_l1(cells[v], p.cells[v]) <= tol_ghost, pid
        pre[pid] = (cells, faces)
    h.advance(1, dt / 2, 0)
    h.synchronize()
    tol = 1e-12 if precision == FP64 else 1e-5
    for pid in samples:
        p = o.patches[pid]
        cells, faces = pre[pid]
        # the oracle advances the fully extended region; the library's region is that region
        # shrunk on sides whose ghost layers are covered by siblings (compared there)
        full = amr.update_box(p.interior_box()[0], p.interior_box()[1], 1, 0)
        ref = mhd.advance(cells, faces, [o.dx(1)] * 3, dt / 2, full, o.gamma)
        reg = h.update_box(pid, 0)
        assert all(full[0][a] <= reg[0][a] and reg[1][a] <= full[1][a] for a in range(3))
        got_c, got_f = h.download(pid)
        sel = (slice(None),) + mhd._sel(reg)
        for m in range(5):
            assert _rel_l1(got_c[m][sel[1:]], ref.cells[m][sel[1:]]) <= tol, (pid, m)
        for d in range(3):
            fsel = mhd._face_sel(reg, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= tol, (pid, d)
    # substep 1: the same-level fill of its two ghost layers, then the advance of the interiors,
    # recomputed by the oracle from the GPU's filled input
    h.ghost_fill(1, 1)
    h.synchronize()
    pre1 = {pid: h.download(pid) for pid in samples}
    h.advance(1, dt / 2, 1)
    h.synchronize()
    for pid in samples:
        p = o.patches[pid]
        cells, faces = pre1[pid]
        reg = h.update_box(pid, 1)
        assert reg == amr.update_box(p.interior_box()[0], p.interior_box()[1], 1, 1)
        ref = mhd.advance(cells, faces, [o.dx(1)] * 3, dt / 2, reg, o.gamma)
        got_c, got_f = h.download(pid)
        sel = mhd._sel(reg)
        for m in range(5):
            assert _rel_l1(got_c[m][sel], ref.cells[m][sel]) <= tol, ("substep 1", pid, m)
            scale = float(np.max(np.abs(ref.cells[m][sel]))) or 1.0
            assert float(np.max(np.abs(got_c[m][sel] - ref.cells[m][sel]))) <= 50 * tol * scale, ("substep 1", pid, m)
        for d in range(3):
            fsel = mhd._face_sel(reg, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= tol, ("substep 1", pid, d)


def test_two_level_full_root_steps_properties():
    """Two graph-replayed FP32 root steps of the full workload, autotuned as the benchmark runs it:
    conservation, div B, bit-zero sync."""
    from paper_1112_1710_amd.autotune import autotune
    spec = H.two_level()
    _say("two-level full size, properties")
    h = Hierarchy(spec, FP32)
    h.set_field(SmoothField(1112))
    autotune(h, reps=2, use_cache=False)
    s0, c0 = h.conservation()
    for _ in range(2):
        h.step(GRAPH)
    s1, c1 = h.conservation()
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
    tot0, tot1 = s0 + c0, s1 + c1
    # float32 state: conserved to float32 round-off of the totals
    # the momentum totals are near zero: measure them against the momentum magnitude scale (~0.1)
    for q in range(5):
        scale = max(abs(tot0[q]), 0.05)
        assert abs(tot1[q] - tot0[q]) <= 1e-5 * scale, (q, tot0[q], tot1[q])


def test_two_level_time_ghosts_root_steps_properties():
    """The full two-level workload with coarse-time-derivative ghosts (as `bench.py --ghosts time` runs it):
    two graph-replayed FP32 root steps keep mass and energy to float32 round-off of the totals, the
    shared-face synchronisation exact and the state physical."""
    spec = H.two_level()
    _say("two-level full size, time-derivative ghosts")
    h = Hierarchy(spec, FP32, ghosts="time")
    h.set_field(SmoothField(1112))
    s0, c0 = h.conservation()
    for _ in range(2):
        h.step(GRAPH)
    s1, c1 = h.conservation()
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
    tot0, tot1 = s0 + c0, s1 + c1
    for q in range(5):
        scale = max(abs(tot0[q]), 0.05)
        assert abs(tot1[q] - tot0[q]) <= 1e-5 * scale, (q, tot0[q], tot1[q])


def test_uniform_256_sampled_windows():
    """Windows of the 256^3 FP32 advance recomputed by the oracle from the GPU's ghost-filled input."""
    n = 256
    spec = H.single_patch(n)
    _say("uniform 256^3 sampled windows")
    h = Hierarchy(spec, FP32)
    h.set_field(SmoothField(1710))
    h.ghost_fill(0, 0)
    h.synchronize()
    rng = np.random.default_rng(0)
    w = 8
    centres = [np.array([G, G, G]), np.array([G + n - w, G + n - w, G + n - w])] + \
              [G + rng.integers(0, n - w, 3) for _ in range(6)]
    halo = 4
    pre = []
    for c in centres:
        lo = c - halo
        hi = c + w + halo + 1
        pre.append(h.download_box(0, lo, hi))
    dt = 1.0e-3
    h.advance(0, dt, 0)
    h.synchronize()
    for c, (cells, faces) in zip(centres, pre):
        lo = c - halo
        region = ((halo,) * 3, (halo + w,) * 3)
        ref = mhd.advance(cells, faces, [1.0 / n] * 3, dt, region, 5.0 / 3.0)
        got_c, got_f = h.download_box(0, lo, c + w + halo + 1)
        sel = mhd._sel(region)
        for m in range(5):
            assert _rel_l1(got_c[m][sel], ref.cells[m][sel]) <= 1e-5, (c, m)
        for d in range(3):
            fsel = mhd._face_sel(region, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= 1e-5, (c, d)


def _deep_samples(spec, centre):
    """Patch ids: two level-3 patches nearest the blast surface (|x - c| = 0.1) and the largest finest patch."""
    root = spec.root_n[0]
    pick3 = []
    finest = spec.levels() - 1
    best_f, best_v = None, -1
    for pid, (lv, lo, hi) in enumerate(spec.patches):
        n = root << lv
        if lv == 3:
            ctr = [(lo[a] + hi[a]) / 2 / n for a in range(3)]
            r = sum(((ctr[a] - centre[a] + 0.5) % 1.0 - 0.5) ** 2 for a in range(3)) ** 0.5
            pick3.append((abs(r - 0.1), pid))
        if lv == finest:
            v = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
            if v > best_v:
                best_f, best_v = pid, v
    pick3.sort()
    return [pick3[0][1], pick3[1][1], best_f]


@pytest.mark.parametrize("steps_before", [0, 2])
def test_deep_hierarchy_sampled_patches(steps_before):
    """Deep 8-level blast hierarchy (64^3 root, ~40M cells), autotuned, FP32, from the initial state and
    after two graph-replayed root steps (the blast's shock then crosses patch and level boundaries):
    the first-substep chain of a root step (ghost fill + advance of every level in turn), then the
    finest level's substep-1 fill and advance; the oracle advances the sampled patches from the GPU's
    own ghost-filled input."""
    from paper_1112_1710_amd.autotune import autotune
    from workloads.fields import Blast
    spec, centre, _ = H.deep_blast_target()
    _say("deep hierarchy, sampled patches", len(spec.patches), "patches,", steps_before, "root steps before")
    h = Hierarchy(spec, FP32)
    h.set_field(Blast(centre))
    autotune(h, reps=2, use_cache=False)
    if steps_before:
        h.steps(steps_before, GRAPH)
    samples = _deep_samples(spec, centre)
    by_level = {}
    for pid in samples:
        by_level.setdefault(spec.patches[pid][0], []).append(pid)
    o = amr.Hierarchy(spec.root_n)
    dt0 = h.cfl_dt()
    assert dt0 > 0
    pre = {}
    for lv in range(spec.levels()):
        h.ghost_fill(lv, 0)
        if lv in by_level:
            h.synchronize()
            for pid in by_level[lv]:
                pre[pid] = h.download(pid)
        h.advance(lv, dt0 / 2 ** lv, 0)
    h.synchronize()
    for pid in samples:
        lv, lo, hi = spec.patches[pid]
        cells, faces = pre[pid]
        n = [hi[a] - lo[a] for a in range(3)]
        reg = h.update_box(pid, 0)
        dx = o.dx(lv)
        ref = mhd.advance(cells, faces, [dx] * 3, dt0 / 2 ** lv, reg, 5.0 / 3.0)
        got_c, got_f = h.download(pid)
        sel = mhd._sel(reg)
        for m in range(5):
            assert _rel_l1(got_c[m][sel], ref.cells[m][sel]) <= 1e-5, (pid, lv, m)
        for d in range(3):
            fsel = mhd._face_sel(reg, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= 1e-5, (pid, lv, d)
    # the finest level's second substep
    top = spec.levels() - 1
    fine = by_level.get(top, [])
    assert fine
    h.ghost_fill(top, 1)
    h.synchronize()
    pre1 = {pid: h.download(pid) for pid in fine}
    h.advance(top, dt0 / 2 ** top, 1)
    h.synchronize()
    for pid in fine:
        cells, faces = pre1[pid]
        reg = h.update_box(pid, 1)
        ref = mhd.advance(cells, faces, [o.dx(top)] * 3, dt0 / 2 ** top, reg, 5.0 / 3.0)
        got_c, got_f = h.download(pid)
        sel = mhd._sel(reg)
        for m in range(5):
            assert _rel_l1(got_c[m][sel], ref.cells[m][sel]) <= 1e-5, ("substep 1", pid, m)
        for d in range(3):
            fsel = mhd._face_sel(reg, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= 1e-5, ("substep 1", pid, d)


def test_deep_hierarchy_root_step_properties():
    """One graph-replayed FP32 root step of the deep blast hierarchy: bit-zero sync, no unphysical state,
    composite conservation to float32 round-off."""
    from workloads.fields import Blast
    spec, centre, _ = H.deep_blast_target()
    _say("deep hierarchy, root-step properties")
    h = Hierarchy(spec, FP32)
    h.set_field(Blast(centre))
    s0, c0 = h.conservation()
    h.step(GRAPH)
    s1, c1 = h.conservation()
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
    tot0, tot1 = s0 + c0, s1 + c1
    for q in range(5):
        scale = max(abs(tot0[q]), 0.05 * abs(tot0[4]))
        assert abs(tot1[q] - tot0[q]) <= 1e-5 * scale, (q, tot0[q], tot1[q])


@pytest.mark.parametrize("precision,steps", [(FP32, 20), (FP64, 3)])
def test_deep_hierarchy_consecutive_root_steps(precision, steps):
    """The deep 8-level blast runs consecutive root steps (graph-replayed) with no unphysical state:
    the blast's outgoing shock crosses coarse/fine boundaries, where prolongation needs the positivity
    fallback; composite mass and energy stay conserved to the state's round-off."""
    from workloads.fields import Blast
    spec, centre, _ = H.deep_blast_target()
    _say("deep hierarchy, consecutive root steps", precision, steps)
    h = Hierarchy(spec, precision)
    h.set_field(Blast(centre))
    s0, c0 = h.conservation()
    t = 0.0
    for k in range(steps):
        t += h.step(GRAPH)
        if k % 5 == 4:
            _say("  root step", k + 1, "t", t)
    s1, c1 = h.conservation()
    d = h.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0
    tot0, tot1 = s0 + c0, s1 + c1
    tol = 1e-5 if precision == FP32 else 1e-12
    for q in (0, 4):
        assert abs(tot1[q] - tot0[q]) <= tol * abs(tot0[q]), (q, tot0[q], tot1[q])


def test_uniform_512_sampled_windows_far_corner():
    """A 512^3 patch (521^3 padded entries: 64-bit intermediate offsets beyond 2^32 bytes), FP32: windows of
    one advance, including the far corner, recomputed by the oracle from the GPU's ghost-filled input."""
    from workloads.fields import LinearWave
    n = 512
    spec = H.single_patch(n)
    _say("uniform 512^3 sampled windows")
    k = np.array([1, 2, 3])
    rng = np.random.default_rng(5)
    vec = rng.standard_normal(8)
    vec[5:8] -= k * (vec[5:8] @ k) / (k @ k)
    gam = 5.0 / 3.0
    rho, v, p, b = 1.0, np.array([0.1, 0.05, 0.0]), 1.0, np.array([1.0, 0.5, 0.2])
    u0 = np.concatenate([[rho], rho * v, [p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * b @ b], b])
    h = Hierarchy(spec, FP32)
    h.set_field(LinearWave(u0, vec, 0.05, k))
    h.ghost_fill(0, 0)
    h.synchronize()
    w, halo = 8, 4
    centres = [np.array([G, G, G]), np.array([G + n - w] * 3), np.array([G + n - w, G, G + n - w]),
               G + rng.integers(0, n - w, 3)]
    pre = [h.download_box(0, c - halo, c + w + halo + 1) for c in centres]
    dt = 2.0e-4
    h.advance(0, dt, 0)
    h.synchronize()
    for c, (cells, faces) in zip(centres, pre):
        region = ((halo,) * 3, (halo + w,) * 3)
        ref = mhd.advance(cells, faces, [1.0 / n] * 3, dt, region, gam)
        got_c, got_f = h.download_box(0, c - halo, c + w + halo + 1)
        sel = mhd._sel(region)
        for m in range(5):
            assert _rel_l1(got_c[m][sel], ref.cells[m][sel]) <= 1e-5, (c, m)
        for d in range(3):
            fsel = mhd._face_sel(region, d)
            assert _rel_l1(got_f[d][fsel], ref.faces[d][fsel]) <= 1e-5, (c, d)


def test_two_level_low_beta_flux_forms_bit_identical():
    """FP32 with targeted FP64 on the full two-level hierarchy at beta 1e-3, where every face is
    low-beta: the float flux pass lists four waves per block, far more than the low-beta kernel's grid
    of at most 1024 workgroups covers in one sweep, so its walk over the list strides many times.  The
    two-launch form and the one-launch form give the same states and dts bit for bit, batched and
    graph-replayed, and the whole-hierarchy checks stay clean."""
    from paper_1112_1710_amd import FP32_MIXED, binding
    from workloads.fields import low_beta
    spec = H.two_level()
    field = low_beta(5)
    _say("two-level low beta, flux forms")
    a = Hierarchy(spec, FP32_MIXED)
    b = Hierarchy(spec, FP32_MIXED)
    b.tune_set(binding.TUNE_FLUX_SPLIT, 0)
    assert a.tune_get(binding.TUNE_FLUX_SPLIT, level=0) == 1
    n_root = a.debug_tasks(0, 0, 3)
    assert int(n_root[-1, 8]) + 1 > 1024           # more than one sweep of the list walk
    a.set_field(field)
    b.set_field(field)
    for mode in (BATCHED, GRAPH, GRAPH):
        assert a.step(mode) == b.step(mode)
    o = amr.build(spec)
    for pid, p in enumerate(o.patches):
        ca, fa = a.download(pid)
        cb, fb = b.download(pid)
        m = o._interior_mask(p)
        assert np.array_equal(ca[:, m], cb[:, m]), pid
        for d in range(3):
            mk = o._closure_mask(p, d)
            assert np.array_equal(fa[d][mk], fb[d][mk]), (pid, d)
    da = a.diag()
    assert da["phys_flag"] == 0.0 and da["sync_flux_max"] == 0.0
