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
