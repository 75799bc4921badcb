"""Helpers shared by the test modules: run the oracle and the HIP path on the same seeded inputs."""
import numpy as np

from oracle import amr
from workloads.fields import G

FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")


def oracle_from(spec, field, round32=False, gamma=5.0 / 3.0, ghosts="extended"):
    o = amr.build(spec, field, gamma=gamma, ghosts=ghosts)
    if round32:
        for p in o.patches:
            p.cells = p.cells.astype(np.float32).astype(np.float64)
            p.faces = [f.astype(np.float32).astype(np.float64) for f in p.faces]
    return o


def upload_oracle_state(h, o):
    for pid, p in enumerate(o.patches):
        h.upload(pid, p.cells, p.faces)
    h.synchronize()


def rel_l1(h, o):
    """Per-field relative L1 difference over all patch interiors (cells) and interior closures (faces)."""
    num = np.zeros(8)
    den = np.zeros(8)
    for pid, p in enumerate(o.patches):
        cells, faces = h.download(pid)
        n = p.n
        sl = (slice(G, G + n[2]), slice(G, G + n[1]), slice(G, G + n[0]))
        for m in range(5):
            num[m] += np.sum(np.abs(cells[m][sl] - p.cells[m][sl]))
            den[m] += np.sum(np.abs(p.cells[m][sl]))
        for d in range(3):
            hi = [G + int(x) for x in n]
            hi[d] += 1
            fs = (slice(G, hi[2]), slice(G, hi[1]), slice(G, hi[0]))
            num[5 + d] += np.sum(np.abs(faces[d][fs] - p.faces[d][fs]))
            den[5 + d] += np.sum(np.abs(p.faces[d][fs]))
    return num / np.maximum(den, 1e-300)


def max_abs_interior(h, o):
    worst = 0.0
    for pid, p in enumerate(o.patches):
        cells, faces = h.download(pid)
        m = o._interior_mask(p)
        worst = max(worst, float(np.max(np.abs(cells[:, m] - p.cells[:, m]))))
        for d in range(3):
            mk = o._closure_mask(p, d)
            worst = max(worst, float(np.max(np.abs(faces[d][mk] - p.faces[d][mk]))))
    return worst


def max_rel(h, o):
    """Per-field element-wise error: max |q_gpu - q_ref| over all patch interiors (cells) and
    interior closures (faces), divided by max |q_ref| of that field; a momentum or field
    component is measured against the largest magnitude of its vector's components, so a
    component that is exactly zero in the reference (e.g. m_z of a plane-parallel state) is
    still judged on the vector's scale.  Unlike rel_l1 this sees a localized error, such as one
    at a coarse/fine corner, whatever the patch sizes."""
    err = np.zeros(8)
    ref = np.zeros(8)
    for pid, p in enumerate(o.patches):
        cells, faces = h.download(pid)
        m = o._interior_mask(p)
        for q in range(5):
            err[q] = max(err[q], float(np.max(np.abs(cells[q][m] - p.cells[q][m]))))
            ref[q] = max(ref[q], float(np.max(np.abs(p.cells[q][m]))))
        for d in range(3):
            mk = o._closure_mask(p, d)
            err[5 + d] = max(err[5 + d], float(np.max(np.abs(faces[d][mk] - p.faces[d][mk]))))
            ref[5 + d] = max(ref[5 + d], float(np.max(np.abs(p.faces[d][mk]))))
    den = ref.copy()
    for group in ((1, 2, 3), (5, 6, 7)):
        top = max(ref[q] for q in group)
        for q in group:
            den[q] = top
    return err / np.maximum(den, 1e-300)


def grouped_rel_l1(h, o):
    """rel_l1 with each momentum and field component measured against the L1 norm of its whole
    vector when that is larger (a component that starts at zero, e.g. b_z of a field lying in the
    x-y plane, is only round-off or a small dynamical by-product and has no scale of its own)."""
    num = np.zeros(8)
    ref = np.zeros(8)
    for pid, p in enumerate(o.patches):
        cells, faces = h.download(pid)
        m = o._interior_mask(p)
        for q in range(5):
            num[q] += np.sum(np.abs(cells[q][m] - p.cells[q][m]))
            ref[q] += np.sum(np.abs(p.cells[q][m]))
        for d in range(3):
            mk = o._closure_mask(p, d)
            num[5 + d] += np.sum(np.abs(faces[d][mk] - p.faces[d][mk]))
            ref[5 + d] += np.sum(np.abs(p.faces[d][mk]))
    den = ref.copy()
    for group in ((1, 2, 3), (5, 6, 7)):
        total = sum(ref[q] for q in group)
        for q in group:
            den[q] = max(den[q], total)
    return num / np.maximum(den, 1e-300)


def assert_parity(h, o, tol, what="", grouped=False, elem_tol=None):
    """Both bars of a per-step comparison: relative L1 per field (grouped_rel_l1 when ``grouped``)
    and the element-wise bound, each <= tol (1e-12 FP64, 1e-5 FP32) unless ``elem_tol`` sets the
    element-wise bar apart."""
    l1 = grouped_rel_l1(h, o) if grouped else rel_l1(h, o)
    mx = max_rel(h, o)
    elem_tol = tol if elem_tol is None else elem_tol
    print("parity", what, "rel-L1 max %.2e, element-wise max %.2e" % (float(np.max(l1)), float(np.max(mx))),
          flush=True)
    assert np.all(l1 <= tol), ("rel-L1", what, dict(zip(FIELDS, l1)))
    assert np.all(mx <= elem_tol), ("element-wise", what, dict(zip(FIELDS, mx)))
    return l1, mx
