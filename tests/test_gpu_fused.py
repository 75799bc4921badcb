"""The LDS-tiled kernels that fuse the first three advance stages and the
last two (edge EMFs and update), and their autotuner.

The fused kernels perform the staged kernels' operations in the same order,
so whole root steps must agree with the staged schedule bit for bit, for
every tile shape (ragged tiles included: the regions of these hierarchies are
not multiples of any tile) and every precision; the EMF registers the fused
edge/update kernel writes feed the restriction's corrections, so root steps
of multi-level hierarchies check them too.  Parity with the oracle is
checked with both fusions on.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr  # noqa: E402
from paper_1112_1710_amd import BATCHED, FP32, FP32_MIXED, FP64, GRAPH, PLAIN, Hierarchy  # noqa: E402
from paper_1112_1710_amd import binding  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import SmoothField  # noqa: E402


def _say(*a):
    print(*a, flush=True)


def _same_interiors(spec, a, b):
    o = amr.build(spec)
    for pid, p in enumerate(o.patches):
        ca, fa = a.download(pid)
        cb, fb = b.download(pid)
        m = o._interior_mask(p)
        assert np.array_equal(ca[:, m], cb[:, m]), pid
        for d in range(3):
            mk = o._closure_mask(p, d)
            assert np.array_equal(fa[d][mk], fb[d][mk]), (pid, d)


def _allowed(prec):
    return [t for t, row in enumerate(binding.tile_table(prec)) if row[3] > 0]


def _cases():
    try:
        return [(prec, t) for prec in (FP64, FP32, FP32_MIXED) for t in _allowed(prec)]
    except ImportError:  # library not built: nothing to parametrize (the CPU suite only collects)
        return []


CASES = _cases()


def _cases_eu():
    try:
        n = len(binding.tile_table(FP64))
    except ImportError:
        return []
    return [(prec, t) for prec in (FP64, FP32, FP32_MIXED) for t in range(n)]


CASES_EU = _cases_eu()


@pytest.mark.parametrize("prec,tile", CASES_EU)
def test_fused_edge_update_matches_staged_bit_for_bit(prec, tile):
    spec = H.small_three_level()
    _say("fused edge/update vs staged", prec, tile, binding.tile_table(prec)[tile][:3])
    field = SmoothField(29)
    a = Hierarchy(spec, prec)
    b = Hierarchy(spec, prec)
    a.tune_set(binding.TUNE_FUSED, 0)
    b.tune_set(binding.TUNE_FUSED, 0)
    b.tune_set(binding.TUNE_FUSED_EU, 1)
    b.tune_set(binding.TUNE_TILE_EU, tile)
    a.set_field(field)
    b.set_field(field)
    for _ in range(2):
        dt = a.step(BATCHED)
        assert b.step(BATCHED) == dt
    _same_interiors(spec, a, b)
    d = b.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


@pytest.mark.parametrize("prec,tile", CASES)
def test_fused_matches_staged_bit_for_bit(prec, tile):
    spec = H.small_three_level()
    _say("fused vs staged", prec, tile, binding.tile_table(prec)[tile][:3])
    field = SmoothField(21)
    a = Hierarchy(spec, prec)
    b = Hierarchy(spec, prec)
    a.tune_set(binding.TUNE_FUSED, 0)
    b.tune_set(binding.TUNE_FUSED, 1)
    for lvl in range(spec.levels()):
        b.tune_set(binding.TUNE_TILE, tile, level=lvl)
    a.set_field(field)
    b.set_field(field)
    for _ in range(2):
        dt = a.step(BATCHED)
        dtb = b.step(BATCHED)
        assert dt == dtb
    _same_interiors(spec, a, b)
    assert b.diag()["phys_flag"] == 0


@pytest.mark.parametrize("name", ["root_tiled", "single32", "small_three_level", "minimal_patches"])
def test_fused_plain_and_graph_schedules(name):
    spec = H.single_patch(32) if name == "single32" else getattr(H, name)()
    _say("fused plain/graph", name)
    field = SmoothField(22)
    ref = Hierarchy(spec, FP32)
    ref.tune_set(binding.TUNE_FUSED, 0)
    pl = Hierarchy(spec, FP32)
    gr = Hierarchy(spec, FP32)
    for h in (pl, gr):
        h.tune_set(binding.TUNE_FUSED, 1)
        h.tune_set(binding.TUNE_TILE, 7)  # 24x8x2: ragged in x on these patches
        h.tune_set(binding.TUNE_FUSED_EU, 1)
        h.tune_set(binding.TUNE_TILE_EU, 3)  # 32x4x2
    for h in (ref, pl, gr):
        h.set_field(field)
    for _ in range(3):
        dt = ref.step(BATCHED)
        assert pl.step(PLAIN) == dt
        assert gr.step(GRAPH) == dt
    _same_interiors(spec, ref, pl)
    _same_interiors(spec, ref, gr)


def test_autotune_selects_allowed_tiles_and_keeps_results(tmp_path):
    from paper_1112_1710_amd.autotune import autotune
    spec = H.small_three_level()
    _say("autotune")
    field = SmoothField(23)
    a = Hierarchy(spec, FP32)
    b = Hierarchy(spec, FP32)
    a.tune_set(binding.TUNE_FUSED, 0)
    a.set_field(field)
    b.set_field(field)
    cache = str(tmp_path / "tune.json")
    chosen = autotune(b, reps=2, path=cache)
    allowed = _allowed(FP32)
    levels = list(range(spec.levels()))
    assert sorted(k for k in chosen if isinstance(k, int)) == levels
    assert sorted(k[1] for k in chosen if not isinstance(k, int)) == levels
    for key, (t, shape, ms, src) in chosen.items():
        assert src == "search" and ms > 0
        if isinstance(key, int):
            assert t == -1 or t in allowed
            assert b.tune_get(binding.TUNE_FUSED, level=key) == (0 if t == -1 else 1)
            if t >= 0:
                assert b.tune_get(binding.TUNE_TILE, level=key) == t
        else:
            assert b.tune_get(binding.TUNE_FUSED_EU, level=key[1]) == (0 if t < 0 else 1)
            assert b.tune_get(binding.TUNE_UPDATE_NT, level=key[1]) == (1 if t == -2 else 0)
            if t >= 0:
                assert b.tune_get(binding.TUNE_TILE_EU, level=key[1]) == t
    again = autotune(b, reps=2, path=cache)
    assert all(v[3] == "cache" and v[0] == chosen[k][0] for k, v in again.items())
    # timing runs touch only intermediates: the state still gives the staged result
    for _ in range(2):
        assert a.step(BATCHED) == b.step(GRAPH)
    _same_interiors(spec, a, b)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_fused_path_matches_oracle(prec):
    """One root step with every level running both fused kernels against the oracle (per-field relative L1,
    as the parity tests)."""
    from ._common import FIELDS, oracle_from, rel_l1, upload_oracle_state
    spec = H.small_three_level()
    _say("fused vs oracle", prec)
    o = oracle_from(spec, SmoothField(24), round32=prec != FP64)
    h = Hierarchy(spec, prec)
    h.tune_set(binding.TUNE_FUSED, 1)
    h.tune_set(binding.TUNE_FUSED_EU, 1)
    upload_oracle_state(h, o)
    dt = o.cfl_dt()
    o.root_step(dt)
    h.step(BATCHED, dt)
    err = rel_l1(h, o)
    assert np.all(err <= (1e-12 if prec == FP64 else 1e-5)), dict(zip(FIELDS, err))


@pytest.mark.skip(reason="concurrent schedule switched off: its first GPU capture ended the test process with a "
                         "segmentation fault and the cause is not yet shown")
@pytest.mark.parametrize("name,fused", [("small_three_level", False), ("small_three_level", True),
                                        ("root_tiled", False), ("two_level", False), ("two_level", True)])
@pytest.mark.parametrize("fixed_dt", [False, True])
def test_concurrent_schedule_is_bit_identical_to_batched(name, fused, fixed_dt):
    """Replays of the per-level-branch graph equal the batched schedule bit for bit over several root steps."""
    from paper_1112_1710_amd import CONCURRENT
    spec = getattr(H, name)()
    _say("concurrent schedule", name, fused, fixed_dt)
    field = SmoothField(25)
    prec = FP32 if name == "two_level" else FP64
    a = Hierarchy(spec, prec)
    b = Hierarchy(spec, prec)
    if fused:
        b.tune_set(binding.TUNE_FUSED, 1)
    a.set_field(field)
    b.set_field(field)
    for _ in range(3):
        dt = a.step(BATCHED, 1e-3 if fixed_dt else 0.0)
        assert b.step(CONCURRENT, 1e-3 if fixed_dt else 0.0) == dt
    _same_interiors(spec, a, b)
    d = b.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


def test_disabled_schedules_report_einval():
    """The switched-off schedules are refused before any launch."""
    from paper_1112_1710_amd import CONCURRENT, PERSISTENT, AmrxError
    spec = H.small_three_level()
    h = Hierarchy(spec, FP64)
    h.set_field(SmoothField(26))
    for mode in (PERSISTENT, CONCURRENT):
        with pytest.raises(AmrxError) as ei:
            h.step(mode)
        assert ei.value.code == -1
    h.step(BATCHED)


@pytest.mark.parametrize("name,prec", [("block_two_level", FP64), ("two_level", FP32)])
def test_sibling_covered_sides_skip_extended_update(name, prec):
    """Refined patches advance their extended ghost layers only on sides not covered by siblings;
    the interiors equal, bit for bit, those of the run that treats every patch as isolated."""
    spec = getattr(H, name)()
    _say("per-side extended regions", name)
    field = SmoothField(27)
    a = Hierarchy(spec, prec, extend_all=True)
    b = Hierarchy(spec, prec)
    shrunk = sum(1 for pid, (lv, _, _) in enumerate(spec.patches) if lv > 0 and a.update_box(pid, 0) != b.update_box(pid, 0))
    assert shrunk > 0
    a.set_field(field)
    b.set_field(field)
    for k in range(3):
        dt = a.step(BATCHED)
        assert b.step(GRAPH if k else BATCHED) == dt
    _same_interiors(spec, a, b)
    d = b.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


@pytest.mark.parametrize("name,prec", [("small_three_level", FP64), ("block_two_level", FP64), ("two_level", FP32)])
def test_paired_levels_bit_identical(name, prec):
    """A level's advance sharing launches with the finer level's first substep gives the sequential
    schedule's results bit for bit (batched and graph-captured)."""
    spec = getattr(H, name)()
    _say("paired levels", name)
    field = SmoothField(28)
    a = Hierarchy(spec, prec)
    b = Hierarchy(spec, prec)
    g = Hierarchy(spec, prec)
    for x in (b, g):
        x.tune_set(binding.TUNE_PAIR, 1)
        assert x.tune_get(binding.TUNE_PAIR) == 1
    for x in (a, b, g):
        x.set_field(field)
    for _ in range(3):
        dt = a.step(BATCHED)
        assert b.step(BATCHED) == dt
        assert g.step(GRAPH) == dt
    _same_interiors(spec, a, b)
    _same_interiors(spec, a, g)
    d = g.diag()
    assert d["sync_flux_max"] == 0.0 and d["sync_face_max"] == 0.0 and d["phys_flag"] == 0.0


@pytest.mark.parametrize("prec", [FP64, FP32, FP32_MIXED])
def test_non_temporal_update_is_bit_identical(prec):
    """The staged update with its next-state stores marked non-temporal (on every level, then on one level)
    gives the same states and dts as ordinary stores, batched and graph-replayed."""
    spec = H.small_three_level()
    _say("non-temporal update", prec)
    field = SmoothField(26)
    a = Hierarchy(spec, prec)
    b = Hierarchy(spec, prec)
    b.tune_set(binding.TUNE_UPDATE_NT, 1)
    a.set_field(field)
    b.set_field(field)
    for mode in (BATCHED, GRAPH, GRAPH):
        assert a.step(mode) == b.step(mode)
    b.tune_set(binding.TUNE_UPDATE_NT, 0, level=1)
    for mode in (PLAIN, GRAPH):
        assert a.step(mode) == b.step(mode)
    _same_interiors(spec, a, b)
    assert b.tune_time_eu(1, -2, 1) > 0
