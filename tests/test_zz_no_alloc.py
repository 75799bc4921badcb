"""The regrid transfer that allocates nothing (hier_init_from_levels_static) against the same transfer with a
caller workspace (hier_init_from_levels): bit-identical new hierarchies on two calls in a row, the second
with smaller transfer lists than the first (the static workspace keeps the last call's contents), and a
clear error when the lists exceed the static workspace."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import amr  # noqa: E402
from paper_1112_1710_amd import FP32, FP64, AmrxError, Hierarchy  # noqa: E402
from workloads import hierarchies as H  # noqa: E402
from workloads.fields import SmoothField  # noqa: E402


def _say(*a):
    print(*a, flush=True)


def _same_interiors(spec, a, b):
    o = amr.build(spec)  # index masks only
    for pid, p in enumerate(o.patches):
        ca, fa = a.download(pid)
        cb, fb = b.download(pid)
        m = o._interior_mask(p)
        assert np.array_equal(ca[:, m], cb[:, m]), pid
        for d in range(3):
            mk = o._closure_mask(p, d)
            assert np.array_equal(fa[d][mk], fb[d][mk]), (pid, d)


def _spec(boxes):
    spec = H.HierarchySpec(root_n=(16, 16, 16))
    spec.patches.append((0, (0, 0, 0), (16, 16, 16)))
    for lo, hi in boxes:
        spec.patches.append((1, lo, hi))
    return spec


# new level-1 layouts over the small two-level hierarchy's root: partial overlaps with the old level-1
# patches, a patch with no overlap (prolongated throughout), then a single small patch
BIG = [((2, 4, 4), (14, 16, 16)), ((16, 16, 2), (30, 28, 12)), ((4, 20, 20), (10, 26, 28))]
SMALL = [((6, 6, 6), (10, 10, 10))]


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_static_transfer_equals_workspace_transfer(precision):
    old = Hierarchy(H.small_two_level(), precision)
    old.set_field(SmoothField(71))
    for k, boxes in enumerate((BIG, SMALL)):
        spec = _spec(boxes)
        _say("no-alloc transfer", precision, "call", k, len(boxes), "patches")
        ref = Hierarchy(spec, precision)
        ref.init_from(old, 1)
        got = Hierarchy(spec, precision)
        got.init_from_static(old, 1)
        got.synchronize()
        _same_interiors(spec, ref, got)
        assert ref.init_from_bytes(old, 1) <= 32 << 20


def test_static_transfer_refuses_lists_beyond_its_size():
    src = Hierarchy(H.single_patch(128), FP32)
    src.set_field(SmoothField(72))
    spec = H.HierarchySpec(root_n=(128, 128, 128))
    spec.patches.append((0, (0, 0, 0), (128, 128, 128)))
    spec.patches.append((1, (2, 2, 2), (254, 254, 254)))
    dst = Hierarchy(spec, FP32)
    assert dst.init_from_bytes(src, 1) > 32 << 20
    _say("no-alloc transfer beyond the static workspace")
    with pytest.raises(AmrxError) as ei:
        dst.init_from_static(src, 1)
    assert ei.value.code == -1 and "static workspace" in str(ei.value)
