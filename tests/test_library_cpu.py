"""Host-side checks of libamrx (no GPU): exported symbols, error codes, bookkeeping vs the oracle.

The ghost-source maps and the prolongation cell lists the library builds (in
C++) must equal the oracle's brute-force maps bit for bit (Sec. 2: data
shared with same-level neighbours; Sec. 2.2: prolongation from the parent).
"""
import ctypes
import functools
import os
import re

import numpy as np
import pytest

from oracle import amr
from workloads import hierarchies as H

binding = pytest.importorskip("paper_1112_1710_amd.binding")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return binding.load_library()
    except ImportError as e:  # not built
        pytest.skip(str(e))


@functools.lru_cache(maxsize=None)
def _schedule_hier(name):
    """Host-only hierarchy shared by the schedule-table tests (their calls are pure host reads;
    the tests that tune set every switch they depend on)."""
    return binding.Hierarchy(getattr(H, name)(), device=None)


def test_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "amrx.h")).read()
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", hdr, flags=re.M)
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n


def test_error_codes_on_bad_input():
    _lib()
    spec = H.HierarchySpec(root_n=(16, 16, 16), patches=[(0, (0, 0, 0), (16, 16, 16))])
    h = binding.Hierarchy(spec, device=None)
    lib = h.lib
    i3 = binding._i3
    pid = ctypes.c_int()
    # frozen hierarchy: patch_add after finalize
    assert lib.patch_add(h.h, 1, i3((4, 4, 4)), i3((8, 8, 8)), ctypes.byref(pid)) == -6
    d = binding.Desc()
    d.root_n = i3((16, 16, 16))
    d.max_level, d.ratio, d.nghost, d.gamma, d.cfl, d.precision = 2, 2, 4, 5 / 3, 0.4, 0
    hh = ctypes.c_void_p()
    assert lib.hier_create(ctypes.byref(d), ctypes.byref(hh)) == 0
    assert lib.patch_add(hh, 0, i3((0, 0, 0)), i3((16, 16, 16)), ctypes.byref(pid)) == 0
    assert lib.patch_add(hh, 1, i3((3, 4, 4)), i3((8, 8, 8)), ctypes.byref(pid)) == -2      # odd corner
    assert lib.patch_add(hh, 1, i3((0, 4, 4)), i3((8, 8, 8)), ctypes.byref(pid)) == -2      # no inset
    assert lib.patch_add(hh, 2, i3((8, 8, 8)), i3((12, 12, 12)), ctypes.byref(pid)) == -2   # no parent
    assert lib.patch_add(hh, 1, i3((4, 4, 4)), i3((12, 12, 12)), ctypes.byref(pid)) == 0
    assert lib.patch_add(hh, 1, i3((10, 10, 10)), i3((14, 14, 14)), ctypes.byref(pid)) == -3  # overlap
    assert lib.patch_add(hh, 3, i3((4, 4, 4)), i3((8, 8, 8)), ctypes.byref(pid)) == -1      # level > max
    assert lib.hier_bind(hh, None, 0, None, 0) == -1
    assert lib.hier_steps(h.h, binding.BATCHED, 1, 0.0, None, None) == -6  # not bound
    lib.hier_destroy(hh)
    d.ratio = 3
    assert lib.hier_create(ctypes.byref(d), ctypes.byref(hh)) == -1
    d.ratio, d.root_n = 2, i3((16, 8, 16))
    assert lib.hier_create(ctypes.byref(d), ctypes.byref(hh)) == -1


def test_root_must_be_tiled():
    _lib()
    spec = H.HierarchySpec(root_n=(16, 16, 16), patches=[(0, (0, 0, 0), (8, 16, 16))])
    with pytest.raises(binding.AmrxError):
        binding.Hierarchy(spec, device=None)


@pytest.mark.parametrize("name", ["small_two_level", "small_three_level", "root_tiled", "minimal_patches"])
def test_ghost_sources_match_oracle_bit_exact(name):
    _lib()
    spec = getattr(H, name)()
    h = binding.Hierarchy(spec, device=None)
    o = amr.build(spec)
    for pid, p in enumerate(o.patches):
        assert np.array_equal(h.debug_sources(pid, 0), o.cell_src[pid])
        for d in range(3):
            assert np.array_equal(h.debug_sources(pid, 1 + d), o.face_src[pid][d])


@pytest.mark.parametrize("name", ["small_two_level", "small_three_level", "minimal_patches"])
def test_prolongation_cells_match_oracle(name):
    _lib()
    spec = getattr(H, name)()
    h = binding.Hierarchy(spec, device=None)
    o = amr.build(spec)
    for pid, p in enumerate(o.patches):
        if p.level == 0:
            continue
        n = (p.n + 8) // 2
        ref = [((p.lo - 4) // 2 + np.array([cx, cy, cz]))
               for cz in range(n[2]) for cy in range(n[1]) for cx in range(n[0])
               if o.cell_src[pid][2 * cz, 2 * cy, 2 * cx] < 0]
        assert np.array_equal(h.debug_prolong_cells(pid), np.array(ref).reshape(-1, 3))


def test_two_level_workload_bookkeeping():
    """The 512-patch two-level workload builds; its level-1 ghost maps agree with the oracle on a sample."""
    _lib()
    spec = H.two_level()
    h = binding.Hierarchy(spec, device=None)
    o = amr.build(spec)
    for pid in (1, 100, 257, 512):
        assert np.array_equal(h.debug_sources(pid, 0), o.cell_src[pid])
        for d in range(3):
            assert np.array_equal(h.debug_sources(pid, 1 + d), o.face_src[pid][d])


def test_large_patch_sources_match_oracle_bit_exact():
    """Patches above 2^20 padded entries build their source maps plane slab by plane slab in
    parallel; with neighbours on every side (a 256^3 root tiled by eight 128^3 patches) the maps of
    cells and of z-faces still equal the oracle's brute-force maps bit for bit."""
    _lib()
    spec = H.root_tiled(256, 2)
    h = binding.Hierarchy(spec, device=None)
    o = amr.build(spec)
    pid = 3
    assert np.array_equal(h.debug_sources(pid, 0), o.cell_src[pid])
    assert np.array_equal(h.debug_sources(pid, 3), o.face_src[pid][2])


@pytest.mark.parametrize("name", ["small_three_level", "root_tiled", "two_level"])
@pytest.mark.parametrize("fixed_dt", [False, True])
def test_persistent_schedule_claims_complete(name, fixed_dt):
    """Simulate the fine-first claim protocol on the schedule tables the library builds.

    Virtual workgroups take the first ready item of the finest queue that has one
    and finish running items in random order; every item must be taken and every
    node completed (no dependency can block progress).  Predecessors always
    precede their node (acyclic) and each level's substeps appear 2^l times.
    """
    import random
    _lib()
    spec = getattr(H, name)()
    h = _schedule_hier(name)
    nodes, preds, items, queues = h.debug_schedule(fixed_dt, 1024)
    nn = len(nodes)
    nblk = nodes[:, 8]
    for v in range(nn):
        pf, npr = nodes[v, 10], nodes[v, 11]
        assert np.all(preds[pf:pf + npr] < v)
    update_op = 9
    for lv in range(spec.levels()):
        assert int(np.sum((nodes[:, 0] == update_op) & (nodes[:, 1] == lv))) == 2 ** lv
    done = np.zeros(nn, dtype=np.int64)
    heads = np.zeros(len(queues), dtype=np.int64)
    rng = random.Random(1)
    running = []

    def ready(v):
        pf, npr = nodes[v, 10], nodes[v, 11]
        return all(done[p] >= nblk[p] for p in preds[pf:pf + npr])

    while True:
        while len(running) < 48:
            got = None
            for q in range(len(queues) - 1, -1, -1):
                f, L = queues[q]
                if heads[q] < L and ready(items[f + heads[q], 0]):
                    got = f + heads[q]
                    heads[q] += 1
                    break
            if got is None:
                break
            running.append(got)
        if not running:
            break
        it = running.pop(rng.randrange(len(running)))
        done[items[it, 0]] += items[it, 2] - items[it, 1]
    assert all(heads[q] >= queues[q][1] for q in range(len(queues)))
    assert np.array_equal(done, nblk)


def _simulate_resident_claims(nodes, preds, items, queues, grid, resident, seed=2, max_idle_rounds=200):
    """Discrete-time model of the persistent kernel's loop: `grid` workgroups of which at most `resident`
    run at once (a workgroup not yet resident starts only when a resident one exits); a resident
    workgroup claims the first ready item of the finest queue that has one, runs it for a random number
    of ticks and adds its block count to its node's completion counter, polls while items are pending
    but none is ready, and exits when no queue holds an item.  Returns (completed counts, number of
    ticks in which every resident workgroup polled while nothing ran, i.e. a stall)."""
    import random
    rng = random.Random(seed)
    nn = len(nodes)
    nblk = nodes[:, 8]
    done = np.zeros(nn, dtype=np.int64)
    heads = np.zeros(len(queues), dtype=np.int64)
    started, exited = 0, 0
    active = {}          # workgroup -> (item, remaining ticks) or None while polling
    stall_ticks = 0

    def ready(v):
        pf, npr = nodes[v, 10], nodes[v, 11]
        return all(done[p] >= nblk[p] for p in preds[pf:pf + npr])

    def claim():
        pending = False
        for q in range(len(queues) - 1, -1, -1):
            f, L = queues[q]
            if heads[q] < L:
                pending = True
                if ready(items[f + heads[q], 0]):
                    heads[q] += 1
                    return f + heads[q] - 1, True
        return None, pending

    while exited < grid:
        while len(active) < resident and started < grid:
            active[started] = None
            started += 1
        running = False
        for wg in list(active):
            st = active[wg]
            if st is not None:
                it, left = st
                if left > 1:
                    active[wg] = (it, left - 1)
                    running = True
                    continue
                done[items[it, 0]] += items[it, 2] - items[it, 1]
                active[wg] = None
            got, pending = claim()
            if got is not None:
                active[wg] = (got, rng.randint(1, 4))
                running = True
            elif not pending:
                del active[wg]
                exited += 1
        if not running and active:
            stall_ticks += 1
            if stall_ticks > max_idle_rounds:
                break
        else:
            stall_ticks = 0
    return done, stall_ticks


@pytest.mark.parametrize("name", ["small_three_level", "two_level"])
@pytest.mark.parametrize("resident", [8, 96])
def test_persistent_schedule_residency_model(name, resident):
    """The persistent kernel's claim loop with a grid larger than the co-resident workgroups (the launch
    uses 4 workgroups per CU, 1024 on the MI355X): every node completes exactly its block count and no
    tick passes with all resident workgroups polling and nothing running; the same model reports a
    stall when one item is missing from the tables (a node whose completion count stays short)."""
    _lib()
    spec = getattr(H, name)()
    h = _schedule_hier(name)
    nodes, preds, items, queues = h.debug_schedule(False, 1024)
    for v in range(len(nodes)):                       # items of every node cover its blocks exactly once
        cover = np.zeros(nodes[v, 8], dtype=np.int64)
        for it in items[items[:, 0] == v]:
            cover[it[1]:it[2]] += 1
        assert np.all(cover == 1), v
    done, stall = _simulate_resident_claims(nodes, preds, items, queues, grid=1024, resident=resident)
    assert stall == 0 and np.array_equal(done, nodes[:, 8])
    # control: drop one item of a node that has successors; its completion count stays short
    succ = set(int(p) for p in preds)
    victim = next(i for i in range(len(items)) if int(items[i, 0]) in succ)
    q = next(k for k, (f, L) in enumerate(queues) if f <= victim < f + L)
    items2 = np.delete(items, victim, axis=0)
    queues2 = queues.copy()
    queues2[q, 1] -= 1
    queues2[q + 1:, 0] -= 1
    done2, stall2 = _simulate_resident_claims(nodes, preds, items2, queues2, grid=1024, resident=resident)
    assert stall2 > 0 and not np.array_equal(done2, nodes[:, 8])


@pytest.mark.parametrize("name", ["small_three_level", "root_tiled", "two_level"])
@pytest.mark.parametrize("fixed_dt", [False, True])
def test_layered_schedule_plan(name, fixed_dt):
    """The layered schedule covers every block of every node of the dependency graph exactly once,
    puts every node after all its predecessors' layers (so a layer's launches are independent),
    and orders a layer's items finest level first, program order within a level."""
    _lib()
    spec = getattr(H, name)()
    h = _schedule_hier(name)
    nodes, preds, _, _ = h.debug_schedule(fixed_dt, 1)
    first, items = h.debug_layers(fixed_dt)
    nn = len(nodes)
    layer_of_item = np.repeat(np.arange(len(first) - 1), np.diff(first))
    node_layer = np.full(nn, -1)
    covered = [[] for _ in range(nn)]
    for it, L in zip(items, layer_of_item):
        v = it[0]
        assert node_layer[v] in (-1, L)
        node_layer[v] = L
        covered[v].append((it[1], it[2]))
    for v in range(nn):
        spans = sorted(covered[v])
        want = nodes[v, 8]
        if want == 0:
            continue
        assert spans[0][0] == 0 and spans[-1][1] == want, v
        assert all(a[1] == b[0] for a, b in zip(spans, spans[1:])), v
        pf, npr = nodes[v, 10], nodes[v, 11]
        for p in preds[pf:pf + npr]:
            if nodes[p, 8] > 0:
                assert node_layer[p] < node_layer[v], (p, v)
    for L in range(len(first) - 1):
        lv = [nodes[items[i, 0], 1] for i in range(first[L], first[L + 1])]
        assert lv == sorted(lv, reverse=True), L
    assert len(first) - 1 <= nn
    if spec.levels() > 1:
        assert len(first) - 1 < nn  # launches of different levels share layers


def _simulate_capture(ops, nn, nstreams, nevents):
    """Stream-capture semantics over a capture plan: a stream joins the capture by waiting for an
    event recorded in it, a launch depends on everything its stream has seen so far, a record
    snapshots that set.  Returns each launch's direct dependencies, the ancestor bitmasks, the
    capturing stream's final set and each side stream's final set (bit nn = the slot clear)."""
    CLEAR = nn
    frontier = {-1: 0}
    events = {}
    deps = {}
    for kind, st, ev, v in ops:
        assert -1 <= st < nstreams
        if kind == 0:  # record
            assert st in frontier, "record on a stream outside the capture"
            assert 0 <= ev < nevents and ev not in events, ev
            events[ev] = frontier[st]
        elif kind == 1:  # wait
            assert ev in events, "wait for an event not recorded in this capture"
            frontier[st] = frontier.get(st, 0) | events[ev]
        elif kind == 2:  # launch
            assert st in frontier, "launch on a stream outside the capture"
            assert 0 <= v < nn and v not in deps, v
            deps[v] = frontier[st]
            frontier[st] = 1 << v
        else:  # slot clear
            assert kind == 3 and st == -1 and CLEAR not in deps
            deps[CLEAR] = frontier[st]
            frontier[st] = 1 << CLEAR
    anc = {}
    for v in sorted(deps, key=lambda x: -1 if x == CLEAR else x):
        m = deps[v]
        a = m
        for u in range(nn + 1):
            if m >> u & 1:
                a |= anc[u]
        anc[v] = a
    return deps, anc, frontier


@pytest.mark.parametrize("name", ["small_three_level", "root_tiled", "two_level"])
@pytest.mark.parametrize("fixed_dt", [False, True])
@pytest.mark.parametrize("fused", [(0, 0), (1, 0), (1, 1)])
def test_concurrent_capture_plan(name, fixed_dt, fused):
    """The concurrent schedule's capture plan (switched off after its first capture crashed on the
    GPU): every operation names a stream, event and node inside the pools the library creates for
    it, every side stream enters the capture through the fork before its first launch and is joined
    back before the capture ends, every event is recorded before it is waited for, every node is
    launched exactly once after all its predecessors (and after the slot clear when dt comes from
    the CFL condition), and launches of different levels are left free to overlap."""
    _lib()
    spec = getattr(H, name)()
    h = _schedule_hier(name)
    h.tune_set(binding.TUNE_FUSED, fused[0])
    h.tune_set(binding.TUNE_FUSED_EU, fused[1])
    nodes, preds, ops, nstreams, nevents = h.debug_concurrent(fixed_dt)
    nn = len(nodes)
    assert nstreams == max(1, min(spec.levels(), 4)) and nevents == nn + nstreams + 1
    sched_nodes, sched_preds, _, _ = h.debug_schedule(fixed_dt, 1)
    if fused == (0, 0):  # without fused tiles the plan runs the persistent schedule's graph
        assert np.array_equal(nodes, sched_nodes) and np.array_equal(preds, sched_preds)
    fused_ops = {14, 15}  # fused first stages, fused edge EMF + update
    assert bool(np.isin(nodes[:, 0], list(fused_ops)).any()) == (fused != (0, 0))
    deps, anc, frontier = _simulate_capture([tuple(int(x) for x in o) for o in ops], nn, nstreams, nevents)
    assert sorted(v for v in deps if v < nn) == list(range(nn))
    assert (nn in deps) == (not fixed_dt)
    for v in range(nn):
        pf, npr = nodes[v, 10], nodes[v, 11]
        for p in preds[pf:pf + npr]:
            assert p < v and anc[v] >> int(p) & 1, (p, v)
        if not fixed_dt:
            assert anc[v] >> nn & 1, v
    final = frontier[-1]
    for u in range(nn + 1):
        if final >> u & 1:
            final |= anc[u]
    for st in range(nstreams):
        assert st in frontier and frontier[st] & ~final == 0, st
    if spec.levels() > 1:
        free = any(not (anc[v] >> u & 1) and not (anc[u] >> v & 1)
                   for v in range(nn) for u in range(v) if nodes[u, 1] != nodes[v, 1])
        assert free


def test_padded_volume_limit():
    """Patches whose ghost-padded volume reaches 2^31 entries are rejected (kernels index them with 32 bits)."""
    lib = _lib()
    i3 = binding._i3
    d = binding.Desc()
    d.root_n = i3((1400, 1400, 1400))
    d.max_level, d.ratio, d.nghost, d.gamma, d.cfl, d.precision = 0, 2, 4, 5 / 3, 0.4, 1
    hh = ctypes.c_void_p()
    pid = ctypes.c_int()
    assert lib.hier_create(ctypes.byref(d), ctypes.byref(hh)) == 0
    assert lib.patch_add(hh, 0, i3((0, 0, 0)), i3((1400, 1400, 1400)), ctypes.byref(pid)) == -1
    assert lib.patch_add(hh, 0, i3((0, 0, 0)), i3((1200, 1200, 1200)), ctypes.byref(pid)) == 0  # 1209^3 < 2^31
    lib.hier_destroy(hh)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_tile_table_and_tuning_switches(prec):
    _lib()
    table = binding.tile_table(prec)
    word = 8 if prec == 0 else 4
    assert len(table) >= 2
    for tx, ty, tz, lds in table:
        need = (11 * (tx + 2) * (ty + 2) * (tz + 2) + 3 * (tx + 1) * (ty + 1) * (tz + 1)) * word
        assert lds == (need if need <= 65536 else 0)
    assert table[0][3] > 0  # the default tile is allowed at every precision
    spec = H.small_three_level()
    h = binding.Hierarchy(spec, precision=prec, device=None)
    assert all(h.tune_get(binding.TUNE_FUSED, level=lv) == 0 for lv in range(3))  # staged by default
    staged = h.step_work()
    h.tune_set(binding.TUNE_FUSED, 1)
    assert all(h.tune_get(binding.TUNE_FUSED, level=lv) == 1 for lv in range(3))
    fused = h.step_work()
    h.tune_set(binding.TUNE_FUSED, 0, level=1)
    mixed = h.step_work()
    assert 0 < mixed["prim"][0] < staged["prim"][0] and 0 < mixed["primhalf"][0] < fused["primhalf"][0]
    h.tune_set(binding.TUNE_FUSED, 1)
    for k in ("prim", "bhalf", "pred"):
        assert fused[k] == (0.0, 0) and staged[k][0] > 0
    assert staged["primhalf"] == (0.0, 0)
    assert fused["primhalf"][0] == 16 * staged["prim"][0] + 14 * staged["pred"][0]
    assert fused["primhalf"][1] == staged["prim"][1]
    for k in ("flux", "edge", "update", "copy"):
        assert fused[k] == staged[k]
    for lvl in range(3):
        for t, (_, _, _, lds) in enumerate(table):
            if lds:
                h.tune_set(binding.TUNE_TILE, t, level=lvl)
                assert h.tune_get(binding.TUNE_TILE, level=lvl) == t
            else:
                with pytest.raises(binding.AmrxError):
                    h.tune_set(binding.TUNE_TILE, t, level=lvl)
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_TILE, len(table), level=0)
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_FUSED, 2)
    with pytest.raises(binding.AmrxError):
        h.tune_set(9, 0)
    # non-temporal stores of the staged update: off by default, selectable per level
    assert all(h.tune_get(binding.TUNE_UPDATE_NT, level=lv) == 0 for lv in range(3))
    h.tune_set(binding.TUNE_UPDATE_NT, 1, level=1)
    assert [h.tune_get(binding.TUNE_UPDATE_NT, level=lv) for lv in range(3)] == [0, 1, 0]
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_UPDATE_NT, 2)
    h.tune_set(binding.TUNE_UPDATE_NT, 0)
    # FP32_MIXED flux stage: two launches by default, one launch selectable per level
    assert all(h.tune_get(binding.TUNE_FLUX_SPLIT, level=lv) == 1 for lv in range(3))
    h.tune_set(binding.TUNE_FLUX_SPLIT, 0, level=2)
    assert [h.tune_get(binding.TUNE_FLUX_SPLIT, level=lv) for lv in range(3)] == [1, 1, 0]
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_FLUX_SPLIT, 2)
    h.tune_set(binding.TUNE_FLUX_SPLIT, 1)
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_TILE, 0, level=16)
    # fused edge EMF + update stages: every tile allowed (LDS 3 (tx+1)(ty+1)(tz+1) reals)
    h.tune_set(binding.TUNE_FUSED, 0)
    assert all(h.tune_get(binding.TUNE_FUSED_EU, level=lv) == 0 for lv in range(3))
    assert staged["edgeupd"] == (0.0, 0)
    h.tune_set(binding.TUNE_FUSED_EU, 1)
    feu = h.step_work()
    assert feu["edge"] == (0.0, 0) and feu["update"] == (0.0, 0)
    assert feu["edgeupd"][0] == 31 * staged["update"][0] + 3 * staged["edge"][0]
    assert feu["edgeupd"][1] == staged["update"][1]
    for k in ("prim", "bhalf", "pred", "flux", "copy"):
        assert feu[k] == staged[k]
    for t in range(len(table)):
        h.tune_set(binding.TUNE_TILE_EU, t, level=1)
        assert h.tune_get(binding.TUNE_TILE_EU, level=1) == t
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_TILE_EU, len(table))
    with pytest.raises(binding.AmrxError):
        h.tune_set(binding.TUNE_FUSED_EU, 2)


def test_autotune_size_classes():
    from paper_1112_1710_amd import autotune
    spec = H.two_level()
    assert autotune.size_class(spec, 0) == "n1-s256"          # one 128^3 root patch: side 132
    assert autotune.size_class(spec, 1).startswith("n512-s")


def _covered_sides(o, pid, depth=2, G=4):
    """Per side (2*axis + high): every ghost entry of the side's extended layers has a same-level source."""
    p = o.patches[pid]
    n = [p.hi[a] - p.lo[a] for a in range(3)]
    maps = [o.cell_src[pid]] + [o.face_src[pid][d] for d in range(3)]
    out = []
    for side in range(6):
        d, high = divmod(side, 2)
        ok = True
        for kind, arr in enumerate(maps):
            sl = []
            for a in range(3):
                plus = 1 if (kind >= 1 and a == kind - 1) else 0
                lo, hi = G - depth, G + n[a] + depth + plus
                if a == d:
                    lo, hi = (G + n[a] + plus, hi) if high else (lo, G)
                sl.append(slice(lo, hi))
            ok = ok and bool(np.all(arr[sl[2], sl[1], sl[0]] >= 0))
        out.append(ok)
    return out


@pytest.mark.parametrize("name", ["block_two_level", "small_three_level", "two_level"])
def test_update_regions_follow_sibling_cover(name):
    """The substep-0 update region of a refined patch skips exactly the sides whose extended ghost
    layers are all covered by same-level sources (checked against the oracle's source maps)."""
    _lib()
    spec = getattr(H, name)()
    h = binding.Hierarchy(spec, device=None)
    full = binding.Hierarchy(spec, device=None, extend_all=True)
    o = amr.build(spec)
    pids = [pid for pid, (lv, _, _) in enumerate(spec.patches) if lv > 0]
    if len(pids) > 60:
        pids = pids[::9]
    for pid in pids:
        lv, lo, hi = spec.patches[pid]
        n = [hi[a] - lo[a] for a in range(3)]
        cov = _covered_sides(o, pid)
        blo, bhi = h.update_box(pid, 0)
        for a in range(3):
            assert blo[a] == (4 if cov[2 * a] else 2), (pid, a)
            assert bhi[a] == 4 + n[a] + (0 if cov[2 * a + 1] else 2), (pid, a)
        assert full.update_box(pid, 0) == ((2, 2, 2), tuple(6 + x for x in n))
        assert h.update_box(pid, 1) == ((4, 4, 4), tuple(4 + x for x in n))
    if name == "block_two_level":
        assert h.update_box(14, 0) == ((4, 4, 4), (12, 12, 12))  # the centre patch: covered on all sides


class _FakeTuned:
    """Stands in for a bound hierarchy: records tuning calls, times candidates from a table."""

    def __init__(self, spec, precision, times):
        self.spec, self.precision, self.times, self.calls = spec, precision, times, []

    def tune_set(self, param, value, level=-1):
        self.calls.append((param, value, level))

    def tune_time(self, level, substep, tile, reps=5):
        return self.times[(level, tile)]

    def tune_time_eu(self, level, tile, reps=5):
        return self.times[("eu", level, tile)]


def test_autotune_search_and_cache(tmp_path, monkeypatch):
    """The autotuner keeps the fastest candidate per level (staged = -1, for edge/update also staged with
    the non-temporal update = -2, or a tile), caches it, and a second run applies the cached choice
    without timing."""
    _lib()
    from paper_1112_1710_amd import autotune as at
    monkeypatch.setattr(at, "arch_name", lambda device=0: "gfx950")
    spec = H.small_two_level()
    table = binding.tile_table(1)
    allowed = [t for t, row in enumerate(table) if row[3] > 0]
    times = {(lv, t): 1.0 + 0.01 * (t + 1) for lv in range(2) for t in [-1] + allowed}
    times[(0, -1)] = 0.5           # level 0: staged fastest
    times[(1, allowed[2])] = 0.1   # level 1: one tile fastest
    for lv in range(2):
        for t in [-2, -1] + list(range(len(table))):
            times[("eu", lv, t)] = 1.0 + 0.01 * (t + 3)
    times[("eu", 0, len(table) - 1)] = 0.2  # edge/update: a tile on level 0, staged on level 1
    times[("eu", 1, -1)] = 0.3
    fake = _FakeTuned(spec, 1, times)
    path = str(tmp_path / "tune.json")
    out = at.autotune(fake, reps=1, path=path)
    assert out[0][0] == -1 and out[0][1] == "staged" and out[0][3] == "search"
    assert out[1][0] == allowed[2] and out[1][3] == "search"
    assert (binding.TUNE_FUSED, 0, 0) in fake.calls
    assert (binding.TUNE_FUSED, 1, 1) in fake.calls and (binding.TUNE_TILE, allowed[2], 1) in fake.calls
    assert out[("eu", 0)][0] == len(table) - 1 and out[("eu", 1)][1] == "staged"
    assert (binding.TUNE_FUSED_EU, 1, 0) in fake.calls and (binding.TUNE_TILE_EU, len(table) - 1, 0) in fake.calls
    assert (binding.TUNE_FUSED_EU, 0, 1) in fake.calls
    assert (binding.TUNE_UPDATE_NT, 0, 0) in fake.calls and (binding.TUNE_UPDATE_NT, 0, 1) in fake.calls
    # the non-temporal staged update wins where it is fastest
    times_nt = dict(times)
    times_nt[("eu", 1, -2)] = 0.25
    fake_nt = _FakeTuned(spec, 1, times_nt)
    out_nt = at.autotune(fake_nt, reps=1, use_cache=False)
    assert out_nt[("eu", 1)][:2] == (-2, "staged-nt")
    assert (binding.TUNE_UPDATE_NT, 1, 1) in fake_nt.calls and (binding.TUNE_FUSED_EU, 0, 1) in fake_nt.calls

    def no_timing(*a, **k):
        raise AssertionError("timed although cached")
    fake2 = _FakeTuned(spec, 1, times)
    fake2.tune_time = no_timing
    fake2.tune_time_eu = no_timing
    out2 = at.autotune(fake2, reps=1, path=path)
    assert all(v[3] == "cache" for v in out2.values())
    assert [v[0] for v in out2.values()] == [v[0] for v in out.values()]


@pytest.mark.parametrize("name", ["small_two_level", "small_three_level", "small_three_level_td", "root_tiled",
                                  "block_two_level", "two_level", "minimal_patches"])
def test_time_ghost_nesting_rule_matches_oracle(name):
    """Coarse-time-derivative ghosts: the library accepts exactly the hierarchies the oracle accepts, and
    refined patches then update their interiors only, at both substeps."""
    _lib()
    spec = getattr(H, name)()
    try:
        amr.build(spec, ghosts="time")
        want = True
    except amr.NestingError:
        want = False
    if not want:
        with pytest.raises(binding.AmrxError) as ei:
            binding.Hierarchy(spec, device=None, ghosts="time")
        assert ei.value.code == -2  # ENEST
        return
    h = binding.Hierarchy(spec, device=None, ghosts="time")
    assert h.tune_get(binding.TUNE_GHOSTS) == 1
    for pid, (lv, lo, hi) in enumerate(spec.patches):
        n = tuple(hi[a] - lo[a] for a in range(3))
        for s in (0, 1):
            if lv == 0 and s == 1:
                continue
            assert h.update_box(pid, s) == ((4, 4, 4), tuple(4 + x for x in n)), (pid, s)


def test_time_ghost_switch_and_step_work():
    _lib()
    spec = H.small_three_level_td()
    ext = binding.Hierarchy(spec, device=None)
    td = binding.Hierarchy(spec, device=None, ghosts="time")
    assert ext.tune_get(binding.TUNE_GHOSTS) == 0
    with pytest.raises(binding.AmrxError) as ei:
        td.tune_set(binding.TUNE_GHOSTS, 0)  # only before finalize
    assert ei.value.code == -6
    we, wt = ext.step_work(), td.step_work()
    # interior-only updates: less work in every advance stage
    for k in ("prim", "bhalf", "pred", "flux", "edge", "update"):
        assert wt[k][0] < we[k][0] and wt[k][1] == we[k][1], k
    # substep 1 of each refined level adds a prolongation and a ghost copy of its parent level
    # (level 1: once per root step, level 2: twice)
    assert wt["prolong"][1] == we["prolong"][1] + 3
    assert wt["copy"][1] == we["copy"][1] + 3
    assert wt["prolong"][0] == 2 * we["prolong"][0]


@pytest.mark.parametrize("seed", range(8))
def test_clustering_matches_oracle(seed):
    """The library's Berger-Rigoutsos clustering returns the oracle's boxes, in the same order."""
    _lib()
    from oracle import regrid as oregrid
    rng = np.random.default_rng(100 + seed)
    shape = tuple(int(x) for x in rng.integers(6, 20, 3))
    f = rng.random(shape) < rng.uniform(0.02, 0.2)
    if seed % 2:
        f = oregrid.buffer_flags(f) & (rng.random(shape) < 0.8)
    for min_side, eff in ((2, 0.7), (3, 0.85), (4, 0.5)):
        want = oregrid.cluster(f, min_side, eff)
        got = binding.cluster_flags(f, min_side, eff)
        assert got == want, (min_side, eff)


def test_regrid_boxes_match_oracle():
    """From the same raw flags the library's buffer, nesting layer and clustering per parent give the
    oracle's level-1 boxes (host logic; the flags here come from the oracle's criterion)."""
    _lib()
    from oracle import regrid as oregrid
    from workloads.fields import SmoothField
    spec = H.root_tiled()
    o = amr.build(spec, SmoothField(41))
    h = binding.Hierarchy(spec, device=None)
    nb = ctypes.c_size_t()
    assert h.lib.hier_flag_bytes(h.h, ctypes.byref(nb)) == 0
    arr = np.zeros(nb.value, dtype=np.uint8)
    for pid, p in enumerate(o.patches):
        n = p.n
        rho = p.cells[0][4:4 + n[2], 4:4 + n[1], 4:4 + n[0]]
        raw = oregrid.flag_cells(rho, 0.02)
        offs, shape = h.layout(pid, 0)
        base = offs[0] // 8 // 16
        full = np.zeros(shape, dtype=np.uint8)
        full[4:4 + n[2], 4:4 + n[1], 4:4 + n[0]] = raw
        arr[base:base + full.size] = full.ravel()
    cap = 4096
    boxes = (ctypes.c_int * (6 * cap))()
    cnt = ctypes.c_int()
    assert h.lib.hier_regrid_boxes(h.h, 0, arr.ctypes.data_as(ctypes.c_void_p), 2, 0.7, boxes, cap,
                                   ctypes.byref(cnt)) == 0
    got = [(tuple(boxes[6 * i:6 * i + 3]), tuple(boxes[6 * i + 3:6 * i + 6])) for i in range(cnt.value)]
    want = oregrid.child_boxes(o, 0, 0.02, min_side=2, efficiency=0.7)
    assert cnt.value > 0 and got == want


def test_init_from_levels_checks_its_sources():
    """The two-source transfer (coarser levels from one hierarchy, the new finest level from another) is
    planned on the host: it needs the destination's lower levels in `below`, the new level as the
    destination's finest one and one precision; the one-source form is its special case."""
    _lib()
    from paper_1112_1710_amd import FP32, FP64, AmrxError
    old = binding.Hierarchy(H.small_three_level(), FP64, device=None)
    b1 = [(1, (4, 4, 4), (20, 20, 20))]
    b2 = [(2, (12, 12, 12), (24, 24, 24))]
    root = [p for p in H.small_three_level().patches if p[0] == 0]
    cur = binding.Hierarchy(H.HierarchySpec(root_n=(16, 16, 16), patches=root + b1), FP64, device=None)
    dst = binding.Hierarchy(H.HierarchySpec(root_n=(16, 16, 16), patches=root + b1 + b2), FP64, device=None)
    assert dst.init_from_bytes(old, 2, below=cur) > 0
    assert cur.init_from_bytes(old, 1) > 0          # one source: the root is shared
    for args in ((old, 2, old), (old, 1, cur)):
        with pytest.raises(AmrxError) as ei:
            dst.init_from_bytes(args[0], args[1], below=args[2])
        assert ei.value.code == -1
    cur32 = binding.Hierarchy(H.HierarchySpec(root_n=(16, 16, 16), patches=root + b1), FP32, device=None)
    with pytest.raises(AmrxError) as ei:
        dst.init_from_bytes(old, 2, below=cur32)
    assert ei.value.code == -1


def test_library_binds_to_the_hip_runtime_torch_loads():
    """Loading the library maps exactly one HIP runtime into the process (torch's): a second copy,
    mapped when the library is loaded before torch, finds no device."""
    import subprocess
    import sys
    _lib()
    code = ("from paper_1112_1710_amd import binding; binding.load_library(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_isothermal_switch_rejects_bad_sound_speed():
    _lib()
    with pytest.raises(binding.AmrxError) as ei:
        binding.Hierarchy(H.small_two_level(), device=None, physics="isothermal", cs=0.0)
    assert ei.value.code == -1
    h = binding.Hierarchy(H.small_two_level(), device=None, physics="isothermal", cs=0.7)
    assert h.physics == "isothermal" and h.cs == 0.7


def _stage_region(stage, axis, lo, hi):
    """Entries a stage visits for an update box [lo, hi): flux faces normal to `axis` and the face
    layers around them, edge EMFs along `axis`."""
    rlo, rhi = list(lo), list(hi)
    for a in range(3):
        if stage == 3:
            rlo[a], rhi[a] = (lo[a], hi[a] + 1) if a == axis else (lo[a] - 1, hi[a] + 1)
        else:
            rlo[a], rhi[a] = (lo[a], hi[a]) if a == axis else (lo[a], hi[a] + 1)
    return rlo, rhi


_TASK_SPECS = {"uniform256": lambda: H.single_patch((256, 256, 256)), "two_level": H.two_level,
               "small_three_level": H.small_three_level}


@pytest.mark.parametrize("name", sorted(_TASK_SPECS))
def test_flux_and_edge_tasks_are_axis_interleaved_slabs(name):
    """The flux and edge stages' task lists: per patch, each axis's region covered exactly once by
    slabs of whole z planes (at most 32768 entries a slab unless a single plane is larger), the
    axes of a slab adjacent, and the first blocks of the tasks consecutive in whole blocks."""
    spec = _TASK_SPECS[name]()
    h = binding.Hierarchy(spec, device=None)
    for level in range(spec.levels()):
        for substep in range(1 if level == 0 else 2):
            for stage in (3, 4):
                t = h.debug_tasks(level, substep, stage)
                assert len(t)
                blk = 0
                for row in t:
                    assert row[8] == blk
                    blk += -(-int(np.prod(row[5:8] - row[2:5])) // 256)
                by_patch = {}
                for row in t:
                    by_patch.setdefault(int(row[0]), []).append(row)
                for pid, rows in by_patch.items():
                    lo, hi = h.update_box(pid, substep)
                    for axis in range(3):
                        rlo, rhi = _stage_region(stage, axis, lo, hi)
                        mine = [r for r in rows if r[1] == axis]
                        assert all(list(r[2:4]) == rlo[:2] and list(r[5:7]) == rhi[:2] for r in mine)
                        z = sorted((int(r[4]), int(r[7])) for r in mine)
                        assert z[0][0] == rlo[2] and z[-1][1] == rhi[2]
                        assert all(a[1] == b[0] for a, b in zip(z, z[1:]))       # contiguous, disjoint
                        plane = (rhi[0] - rlo[0]) * (rhi[1] - rlo[1])
                        assert all(b - a == 1 or (b - a) * plane <= 32768 for a, b in z)
                    # slab by slab, the axes of a slab adjacent and in order: (slab, axis) increases
                    zmin = min(int(r[4]) for r in rows)
                    dz = max(int(r[7]) - int(r[4]) for r in rows)
                    keys = [((int(r[4]) - zmin) // dz, int(r[1])) for r in rows]
                    assert all(a < b for a, b in zip(keys, keys[1:])), keys
                    if name == "uniform256" and level == 0:
                        assert len(rows) > 3                                       # large planes: one per slab
