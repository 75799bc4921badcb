"""The patch hierarchy and the recursive level driver of the AMR method.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed here
  * Sec. 2: grids of level l have cell width dx_{l-1} = R dx_l, are nested in
    a single parent of level l-1, and exchange data with parent, children and
    same-level neighbours.
  * Sec. 2.2 (grid life cycle and the recursive AMR(l) routine): each level
    step is Advance; Prolongate the pre-advance data to the children;
    recurse; Restrict the children's data and fluxes onto the parent;
    Synchronise fluxes with same-level neighbours and update ghosts.  The
    parent takes one step of dt_l while its children take R steps of
    dt_l / R.  The Overlap step is the identity on the static hierarchies
    used here.
  * Sec. 2.3 (isolated grids): extended ghost cells R * n_ghost wide let a
    refined grid take its R substeps without new ghost data from the parent,
    updating a region that shrinks by n_ghost per substep.  The same section
    names the other solution: advance the parent first and update the ghost
    cells of later substeps with the coarse grid's time derivative
    (``ghosts="time"`` here; readings below).
  * Sec. 4: the serial level visit order 0, 1, 2, 2, 1, 2, 2 for three levels.

Readings where the paper is silent (the solver is not described at all):
  * R = 2, ghost width G = R * n_g = 4 with n_g = 2 the stencil depth;
  * nesting: level >= 1 boxes have even corners and lie inside ONE parent's
    interior shrunk by one parent cell (so prolongation never needs parent
    ghost data deeper than 2 cells, which the parent's own extended ghost
    update keeps valid);
  * level 0 takes one step per root step; its update region is its interior;
  * same-level ghost cells/faces copy the interior (closure, for faces) of
    the same-level patch holding their periodic image; the patch's own
    closure faces are its own; among several candidates the lowest patch id
    wins.  Ghost data with no same-level source is prolongated from the
    parent's pre-advance data at substep 0 and otherwise keeps the value the
    patch advanced itself;
  * prolongation: conservative minmod-limited linear cells; divergence-free
    faces (Balsara-type: fine faces on coarse faces are b_c plus limited
    transverse slopes unless the coarse face already holds same-level fine
    data; the 12 faces inside a coarse cell start from the mean of the two
    aligned outer faces and receive the least-norm correction that zeroes
    the divergence of all 8 fine cells); positivity fallback: when one of
    the 8 fine cells of a coarse cell would get rho <= 0 or p <= 0 (its own
    conserved values, with the cell-centred field of its prolongated faces;
    limiting rho, m and E separately does not bound the kinetic energy by
    the total energy across a strong shock), all 8 take the coarse cell's
    conserved values instead (first-order, still conservative; the faces
    keep their divergence-free values);
  * restriction: volume mean of cells, area mean of faces on the closure of
    each child box;
  * flux correction: at coarse faces with exactly one covered side the coarse
    flux is replaced by the time- and area-averaged fine flux; at coarse edges
    with covered and uncovered neighbours the coarse EMF is replaced by the
    time- and length-averaged fine EMF and the uncovered faces around the
    edge receive the corresponding Stokes correction (the fine data of the
    first covered neighbour cell in a fixed order are used);
  * synchronisation: fluxes through faces shared by same-level patches are
    compared; the average replaces both and the adjacent cells are corrected
    (the comparison is expected to find exact equality);
  * time step: dt_l,max = C / max (sum_d (|v_d| + c_f,d) / dx_l) over the
    level's interior cells, dt_0 = min_l R^l dt_l,max, dt_l = dt_0 / R^l.
  * coarse-time-derivative ghosts (``ghosts="time"``): refined patches update
    only their interiors at every substep; at substep s >= 1 the ghost data
    without a same-level source is prolongated (as above) from the parent
    state advanced by s dt_{l+1} along the coarse time derivative,
    U^n + (s / R) (U^{n+1} - U^n), taken from the parent's pre-advance and
    advanced arrays before restriction; the parent level's ghost layers of
    depth n_g are first refreshed from their same-level sources at the new
    time.  Every parent entry this prolongation reads must then be valid:
    interior (closure, for faces) or a ghost entry within n_g layers that has
    a same-level source; the hierarchy is rejected otherwise.
"""
from __future__ import annotations

import math

import numpy as np

from . import hydro, mhd

R = 2
G = 4


def _box_inter(alo, ahi, blo, bhi):
    lo = np.maximum(alo, blo)
    hi = np.minimum(ahi, bhi)
    if np.any(hi <= lo):
        return None
    return lo, hi


class NestingError(ValueError):
    pass


class _LazyMaps:
    """Dictionary-like access to per-patch source maps that are built on first use."""

    def __init__(self, h, kind):
        self.h, self.kind = h, kind

    def __getitem__(self, pid):
        m = self.h._maps_of(int(pid))
        return m[0] if self.kind == 0 else m[1]


def update_box(lo, hi, level, substep, ratio=R, n_g=mhd.N_G, ghosts="extended"):
    """Cell box a patch updates at a substep (Sec. 2.3 extended ghost cells).

    Level 0 updates its interior; a refined patch at substep s in 0..R-1
    updates its interior grown by (R - 1 - s) * n_g cells, so an isolated grid
    whose ghost region is R * n_g wide can take all R substeps.  With
    coarse-time-derivative ghosts every patch updates its interior.
    """
    g = 0 if (level == 0 or ghosts == "time") else (ratio - 1 - substep) * n_g
    return tuple(x - g for x in lo), tuple(x + g for x in hi)


class Patch:
    def __init__(self, pid, level, lo, hi):
        self.id = pid
        self.level = level
        self.lo = np.asarray(lo, dtype=np.int64)
        self.hi = np.asarray(hi, dtype=np.int64)
        self.n = self.hi - self.lo
        self.shape = tuple(int(x) + 2 * G + 1 for x in self.n[::-1])   # (Z, Y, X) node padded
        self.cells = None
        self.faces = None
        self.old_cells = None
        self.old_faces = None
        self.parent = None
        self.children = []
        self.facc = None     # per axis (5, ...) accumulated F*dt over the parent step
        self.eacc = None     # per edge axis, accumulated E*dt
        self.last = None     # StepResult of the latest substep
        self.last_dt = None

    def origin(self):
        """Global index of padded array index 0."""
        return self.lo - G

    def interior_box(self):
        return (tuple(int(G) for _ in range(3)), tuple(int(G + x) for x in self.n))

    def pidx(self, g):
        """Padded (x, y, z) index of a global (x, y, z) index."""
        return np.asarray(g) - self.origin()


class Hierarchy:
    def __init__(self, root_n, gamma=5.0 / 3.0, cfl=0.4, ghosts="extended", physics="mhd", cs=1.0):
        if ghosts not in ("extended", "time"):
            raise ValueError("ghosts must be 'extended' or 'time'")
        if physics not in ("mhd", "isothermal"):
            raise ValueError("physics must be 'mhd' or 'isothermal'")
        self.physics = physics
        self.cs = float(cs)
        self.ghosts = ghosts
        self.root_n = np.asarray(root_n, dtype=np.int64)
        self.gamma = gamma
        self.cfl = cfl
        self.patches = []
        self.frozen = False
        self.poison = False
        self.log = []
        self.diag = {"sync_flux_max": 0.0, "sync_face_max": 0.0}

    # ------------------------------------------------------------------ topology
    def nl(self, level):
        return self.root_n * R ** level

    def dx(self, level):
        """Cell width of a level (refined hierarchies require cubic cells)."""
        return 1.0 / float(self.root_n[0] * R ** level)

    def dxv(self, level):
        return [1.0 / float(self.root_n[a] * R ** level) for a in range(3)]

    def level_patches(self, level):
        return [p for p in self.patches if p.level == level]

    @property
    def nlevels(self):
        return 1 + max(p.level for p in self.patches)

    def add(self, level, lo, hi):
        if self.frozen:
            raise NestingError("hierarchy frozen")
        lo = np.asarray(lo, dtype=np.int64)
        hi = np.asarray(hi, dtype=np.int64)
        if np.any(hi <= lo) or level < 0:
            raise NestingError("empty box or negative level")
        if level == 0:
            if np.any(lo < 0) or np.any(hi > self.root_n):
                raise NestingError("root box outside the domain")
        else:
            if not (self.root_n[0] == self.root_n[1] == self.root_n[2]):
                raise NestingError("refinement requires a cubic root grid")
            if np.any(lo % R) or np.any(hi % R):
                raise NestingError("box corners must be multiples of R")
            parents = [q for q in self.level_patches(level - 1)
                       if np.all(R * (q.lo + 1) <= lo) and np.all(hi <= R * (q.hi - 1))]
            if len(parents) != 1:
                raise NestingError("box must lie inside exactly one parent interior shrunk by one parent cell")
        for q in self.level_patches(level):
            if _box_inter(lo, hi, q.lo, q.hi) is not None:
                raise NestingError("overlaps a same-level patch")
        p = Patch(len(self.patches), level, lo, hi)
        if level > 0:
            p.parent = parents[0]
            parents[0].children.append(p)
        self.patches.append(p)
        return p.id

    def freeze(self):
        vol = sum(int(np.prod(p.n)) for p in self.level_patches(0))
        if vol != int(np.prod(self.root_n)):
            raise NestingError("level-0 patches must tile the root grid")
        self.frozen = True
        self._build_maps()
        if self.ghosts == "time":
            self._check_time_ghosts()

    def _check_time_ghosts(self):
        """Every parent entry a substep >= 1 prolongation reads must be valid at the parent's new time."""
        ng = mhd.N_G
        for m in self.patches:
            if not m.children:
                continue
            nb = m.n + 2 * G
            gidx = [np.arange(int(nb[a]) + 1) for a in range(3)]
            # ghost depth of each padded entry along each axis (0 inside the interior / closure)

            def depth(a, closure):
                i = gidx[a]
                hi = G + int(m.n[a]) + (1 if closure else 0)
                return np.maximum(np.maximum(G - i, i - (hi - 1)), 0)
            csrc = self.cell_src[m.id]
            dz, dy, dx_ = (depth(2, False)[:, None, None], depth(1, False)[None, :, None], depth(0, False)[None, None, :])
            cdep = np.maximum(np.maximum(dz, dy), dx_)
            cell_ok = (cdep == 0) | ((cdep <= ng) & (csrc >= 0))
            face_ok = []
            for d in range(3):
                dd = [depth(a, a == d) for a in range(3)]
                fdep = np.maximum(np.maximum(dd[2][:, None, None], dd[1][None, :, None]), dd[0][None, None, :])
                face_ok.append((fdep == 0) | ((fdep <= ng) & (self.face_src[m.id][d] >= 0)))
            mo = m.origin()
            for p in m.children:
                csrc_p = self.cell_src[p.id]
                clo = (p.lo - G) // R
                ncell = (p.n + 2 * G) // R
                for cz in range(ncell[2]):
                    for cy in range(ncell[1]):
                        for cx in range(ncell[0]):
                            if csrc_p[R * cz, R * cy, R * cx] >= 0:
                                continue
                            ci = clo + np.array([cx, cy, cz]) - mo
                            X, Y, Z = (int(v) for v in ci)
                            reads = [(Z, Y, X)]
                            for d in range(3):
                                e = [0, 0, 0]
                                e[d] = 1
                                reads += [(Z + e[2], Y + e[1], X + e[0]), (Z - e[2], Y - e[1], X - e[0])]
                            if not all(cell_ok[r] for r in reads):
                                raise NestingError("time-derivative ghosts: patch %d reads parent cells "
                                                   "without new-time data" % p.id)
                            for d in range(3):
                                a1, a2 = [a for a in range(3) if a != d]
                                for side in (0, 1):
                                    f = [X, Y, Z]
                                    f[d] += side
                                    fr = [tuple(f)]
                                    for a in (a1, a2):
                                        for sgn in (1, -1):
                                            g = list(f)
                                            g[a] += sgn
                                            fr.append(tuple(g))
                                    if not all(face_ok[d][z, y, x] for (x, y, z) in fr):
                                        raise NestingError("time-derivative ghosts: patch %d reads parent faces "
                                                           "without new-time data" % p.id)

    # ------------------------------------------------------------------ ghost maps (brute force)
    def _images(self, p, q):
        """Periodic shifts s with q's box + s meeting p's padded box (faces reach one entry further)."""
        nl = self.nl(p.level)
        out = []
        for sz in (-1, 0, 1):
            for sy in (-1, 0, 1):
                for sx in (-1, 0, 1):
                    s = np.array([sx, sy, sz]) * nl
                    if _box_inter(p.lo - G, p.hi + G + 1, q.lo + s, q.hi + s + 1) is not None:
                        out.append(s)
        return out

    def _candidates(self, p):
        """p itself, then the same-level patches (id order) whose periodic images can meet p's padded box."""
        same = self.level_patches(p.level)
        los = np.array([q.lo for q in same])
        his = np.array([q.hi for q in same])
        nl = self.nl(p.level)
        near = np.zeros(len(same), dtype=bool)
        for sz in (-1, 0, 1):
            for sy in (-1, 0, 1):
                for sx in (-1, 0, 1):
                    s = np.array([sx, sy, sz]) * nl
                    lo = np.maximum(p.lo - G, los + s)
                    hi = np.minimum(p.hi + G + 1, his + s + 1)
                    near |= np.all(hi > lo, axis=1)
        return [p] + [q for q, ok in zip(same, near) if ok and q is not p]

    def _build_maps(self):
        """Source of every padded cell and face of every patch (same level only), built on first use.

        cell_src[p.id]: int64 array (Z, Y, X) over padded cells: q_id * 2**32 + linear
        padded index in q, or -1 when no same-level patch holds the cell.
        face_src[p.id][d]: same for the faces normal to axis d.
        """
        self.cell_src = _LazyMaps(self, 0)
        self.face_src = _LazyMaps(self, 1)
        self._maps = {}

    def _maps_of(self, pid):
        if pid in self._maps:
            return self._maps[pid]
        p = self.patches[pid]
        Z, Y, X = p.shape
        csrc = np.full((Z, Y, X), -1, dtype=np.int64)
        fsrc = [np.full((Z, Y, X), -1, dtype=np.int64) for _ in range(3)]
        gz, gy, gx = np.meshgrid(*(np.arange(p.shape[2 - a]) + p.origin()[a] for a in (2, 1, 0)), indexing='ij')
        g = [gx, gy, gz]
        valid_cell = (gx < p.hi[0] + G) & (gy < p.hi[1] + G) & (gz < p.hi[2] + G)
        for q in self._candidates(p):
            for s in self._images(p, q):
                qlo = q.lo + s
                qhi = q.hi + s
                inside = valid_cell.copy()
                for a in range(3):
                    inside &= (g[a] >= qlo[a]) & (g[a] < qhi[a])
                take = inside & (csrc < 0)
                if np.any(take):
                    qi = [g[a] - s[a] - q.origin()[a] for a in range(3)]
                    lin = (qi[2] * q.shape[1] + qi[1]) * q.shape[2] + qi[0]
                    csrc[take] = q.id * 2 ** 32 + lin[take]
                for d in range(3):
                    inside = np.ones_like(valid_cell)
                    for a in range(3):
                        top = p.hi[a] + G + (1 if a == d else 0)
                        inside &= g[a] < top
                        if a == d:
                            inside &= (g[a] >= qlo[a]) & (g[a] <= qhi[a])
                        else:
                            inside &= (g[a] >= qlo[a]) & (g[a] < qhi[a])
                    take = inside & (fsrc[d] < 0)
                    if np.any(take):
                        qi = [g[a] - s[a] - q.origin()[a] for a in range(3)]
                        lin = (qi[2] * q.shape[1] + qi[1]) * q.shape[2] + qi[0]
                        fsrc[d][take] = q.id * 2 ** 32 + lin[take]
        self._maps[pid] = (csrc, fsrc)
        return self._maps[pid]

    # ------------------------------------------------------------------ state
    def set_state(self, field):
        for p in self.patches:
            st = field.patch(p.level, tuple(int(x) for x in self.root_n), tuple(p.lo), tuple(p.hi))
            p.cells = st.cells.copy()
            p.faces = [f.copy() for f in st.faces]

    def copy_state(self):
        return [(p.cells.copy(), [f.copy() for f in p.faces]) for p in self.patches]

    def load_state(self, st):
        for p, (c, f) in zip(self.patches, st):
            p.cells = c.copy()
            p.faces = [x.copy() for x in f]

    # ------------------------------------------------------------------ ghost fill
    def _copy_from_sources(self, p):
        csrc = self.cell_src[p.id]
        own = p.id
        mask = csrc >= 0
        qids = csrc >> 32
        lins = csrc & (2 ** 32 - 1)
        for qid in np.unique(qids[mask]):
            q = self.patches[int(qid)]
            m = mask & (qids == qid)
            if qid == own:
                m &= ~self._interior_mask(p)
            src = q.cells.reshape(5, -1)[:, lins[m]]
            for c in range(5):
                p.cells[c][m] = src[c]
        for d in range(3):
            fs = self.face_src[p.id][d]
            mask = fs >= 0
            qids = fs >> 32
            lins = fs & (2 ** 32 - 1)
            for qid in np.unique(qids[mask]):
                q = self.patches[int(qid)]
                m = mask & (qids == qid)
                if qid == own:
                    m &= ~self._closure_mask(p, d)
                p.faces[d][m] = q.faces[d].reshape(-1)[lins[m]]

    def _interior_mask(self, p):
        m = np.zeros(p.shape, dtype=bool)
        m[G:G + p.n[2], G:G + p.n[1], G:G + p.n[0]] = True
        return m

    def _closure_mask(self, p, d):
        m = np.zeros(p.shape, dtype=bool)
        hi = [int(G + x) for x in p.n]
        hi[d] += 1
        m[G:hi[2], G:hi[1], G:hi[0]] = True
        return m

    def ghost_fill(self, level, substep):
        for p in self.level_patches(level):
            self._copy_from_sources(p)
        if level > 0 and substep == 0:
            for p in self.level_patches(level):
                self._prolong(p)
        elif level > 0 and self.ghosts == "time":
            # the parent level has advanced: refresh its ghost layers at the new time, then
            # prolongate from the parent state moved along the coarse time derivative
            for q in self.level_patches(level - 1):
                self._copy_from_sources(q)
            for p in self.level_patches(level):
                self._prolong(p, substep / R)

    # ------------------------------------------------------------------ prolongation
    @staticmethod
    def _minmod(a, b):
        return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)

    @staticmethod
    def positivity_fallback(p, fx, fy, fz, u0, gamma, isothermal=False):
        """After the limited-linear prolongation of one coarse cell into the fine cells
        [fx, fx+2) x [fy, fy+2) x [fz, fz+2) of p (and of its faces), give all 8 fine cells the
        coarse conserved values u0 if any of them has rho <= 0, p <= 0 or a non-finite value
        (isothermal gas: p = c_s^2 rho, so rho <= 0 or a non-finite value).  Returns True when it did."""
        sl = (slice(fz, fz + 2), slice(fy, fy + 2), slice(fx, fx + 2))
        u = p.cells[(slice(None),) + sl]
        if isothermal:
            if np.all(np.isfinite(u[:4])) and np.all(u[0] > 0.0):
                return False
            p.cells[(slice(None),) + sl] = u0[:, None, None, None]
            return True
        bc = mhd.cell_centred_b([f[fz:fz + 3, fy:fy + 3, fx:fx + 3] for f in p.faces])[:, :2, :2, :2]
        with np.errstate(all='ignore'):
            w = mhd.prim_from_cons(u, bc, gamma)
        if np.all(np.isfinite(w)) and np.all(w[0] > 0.0) and np.all(w[4] > 0.0):
            return False
        p.cells[(slice(None),) + sl] = u0[:, None, None, None]
        return True

    _interior_map = None

    @classmethod
    def interior_face_map(cls):
        """12 x 24 linear map from the outer fine faces of a coarse cell to its interior fine faces.

        Local fine face arrays of one coarse cell: bx[k][j][i], i in {0,1,2}
        (0 and 2 outer, 1 interior), j,k in {0,1}; by[k][j][i] with j in {0,1,2};
        bz[k][j][i] with k in {0,1,2}.  Outer order: axis, side, then the two
        remaining offsets in (z, y, x) order; interior order: axis, then offsets.
        The interior faces start from the mean of the two aligned outer faces
        and receive the minimum-norm correction that makes the divergence of
        all eight fine cells vanish (pseudo-inverse of the 8 x 12 system).
        """
        if cls._interior_map is not None:
            return cls._interior_map
        outer_idx, inner_idx = {}, {}
        for d in range(3):
            for side in (0, 2):
                for t2 in (0, 1):
                    for t1 in (0, 1):
                        outer_idx[(d, side, t2, t1)] = len(outer_idx)
        for d in range(3):
            for t2 in (0, 1):
                for t1 in (0, 1):
                    inner_idx[(d, t2, t1)] = len(inner_idx)

        def face_key(d, pos, t2, t1):
            return ('o', (d, pos, t2, t1)) if pos in (0, 2) else ('i', (d, t2, t1))

        def transverse(d, x, y, z):
            # (position along d, offsets of the other two axes as (t2, t1)) in (z, y, x) order
            if d == 0:
                return x, z, y
            if d == 1:
                return y, z, x
            return z, y, x

        A_in = np.zeros((8, 12))
        A_out = np.zeros((8, 24))
        row = 0
        for z in (0, 1):
            for y in (0, 1):
                for x in (0, 1):
                    cell = (x, y, z)
                    for d in range(3):
                        pos, t2, t1 = transverse(d, *cell)
                        for sgn, fp in ((-1.0, pos), (1.0, pos + 1)):
                            kind, key = face_key(d, fp, t2, t1)
                            if kind == 'o':
                                A_out[row, outer_idx[key]] += sgn
                            else:
                                A_in[row, inner_idx[key]] += sgn
                    row += 1
        guess = np.zeros((12, 24))
        for (d, t2, t1), i in inner_idx.items():
            guess[i, outer_idx[(d, 0, t2, t1)]] = 0.5
            guess[i, outer_idx[(d, 2, t2, t1)]] = 0.5
        pinv = np.linalg.pinv(A_in)
        # interior = guess o + pinv (-(A_out o + A_in guess o))
        M = guess - pinv @ (A_out + A_in @ guess)
        cls._interior_map = (M, outer_idx, inner_idx)
        return cls._interior_map

    def _prolong(self, p, w=0.0):
        """Fill p's ghost cells/faces that have no same-level source from the parent's pre-advance data,
        or (w > 0) from the parent state U^n + w (U^{n+1} - U^n)."""
        m = p.parent
        if w == 0.0:
            uc = m.old_cells
            bc = m.old_faces
        else:
            uc = m.old_cells + w * (m.cells - m.old_cells)
            bc = [o + w * (f - o) for o, f in zip(m.old_faces, m.faces)]
        csrc = self.cell_src[p.id]
        fsrc = self.face_src[p.id]
        M, outer_idx, inner_idx = self.interior_face_map()
        clo = (p.lo - G) // R           # coarse global index of the first coarse cell of the padded box
        ncell = (p.n + 2 * G) // R
        mo = m.origin()
        for cz in range(ncell[2]):
            for cy in range(ncell[1]):
                for cx in range(ncell[0]):
                    fx, fy, fz = R * cx, R * cy, R * cz      # fine padded index of the first fine cell
                    if csrc[fz, fy, fx] >= 0:
                        continue                          # covered by same-level data (all 8 fine cells)
                    cg = clo + np.array([cx, cy, cz])
                    ci = cg - mo                          # parent padded index
                    X, Y, Z = int(ci[0]), int(ci[1]), int(ci[2])
                    # cells: conservative limited-linear
                    u0 = uc[:, Z, Y, X]
                    slopes = []
                    for d in range(3):
                        e = [0, 0, 0]
                        e[d] = 1
                        up = uc[:, Z + e[2], Y + e[1], X + e[0]]
                        dn = uc[:, Z - e[2], Y - e[1], X - e[0]]
                        slopes.append(self._minmod(up - u0, u0 - dn))
                    for oz in (0, 1):
                        for oy in (0, 1):
                            for ox in (0, 1):
                                val = u0 + 0.25 * ((2 * ox - 1) * slopes[0] + (2 * oy - 1) * slopes[1]
                                                   + (2 * oz - 1) * slopes[2])
                                p.cells[:, fz + oz, fy + oy, fx + ox] = val
                    # faces: outer faces (from fine data where a same-level closure holds them)
                    outer = np.zeros(24)
                    write = np.zeros(24, dtype=bool)
                    for d in range(3):
                        a1, a2 = [a for a in range(3) if a != d]   # a1 < a2: offsets stored (t2=a2, t1=a1)
                        for side in (0, 2):
                            cidx = [X, Y, Z]
                            cidx[d] += side // 2
                            bcf = bc[d][cidx[2], cidx[1], cidx[0]]
                            sl = []
                            for a in (a1, a2):
                                up = list(cidx); up[a] += 1
                                dn = list(cidx); dn[a] -= 1
                                sl.append(self._minmod(bc[d][up[2], up[1], up[0]] - bcf, bcf - bc[d][dn[2], dn[1], dn[0]]))
                            for t2 in (0, 1):
                                for t1 in (0, 1):
                                    fidx = [fx, fy, fz]
                                    fidx[d] += side // 2 * R
                                    fidx[a1] += t1
                                    fidx[a2] += t2
                                    k = outer_idx[(d, side, t2, t1)]
                                    if fsrc[d][fidx[2], fidx[1], fidx[0]] >= 0:
                                        outer[k] = p.faces[d][fidx[2], fidx[1], fidx[0]]
                                    else:
                                        outer[k] = bcf + 0.25 * ((2 * t1 - 1) * sl[0] + (2 * t2 - 1) * sl[1])
                                        write[k] = True
                    inner = M @ outer
                    for (d, side, t2, t1), k in outer_idx.items():
                        if write[k]:
                            a1, a2 = [a for a in range(3) if a != d]
                            fidx = [fx, fy, fz]
                            fidx[d] += side // 2 * R
                            fidx[a1] += t1
                            fidx[a2] += t2
                            p.faces[d][fidx[2], fidx[1], fidx[0]] = outer[k]
                    for (d, t2, t1), k in inner_idx.items():
                        a1, a2 = [a for a in range(3) if a != d]
                        fidx = [fx, fy, fz]
                        fidx[d] += 1
                        fidx[a1] += t1
                        fidx[a2] += t2
                        # interior faces of an uncovered coarse cell never lie on a same-level closure
                        p.faces[d][fidx[2], fidx[1], fidx[0]] = inner[k]
                    self.positivity_fallback(p, fx, fy, fz, u0, self.gamma, self.physics == "isothermal")

    # ------------------------------------------------------------------ advance
    def region(self, p, substep):
        lo, hi = p.interior_box()
        return update_box(lo, hi, p.level, substep, ghosts=self.ghosts)

    def advance_level(self, level, dt, substep):
        self.log.append(level)
        dx = self.dxv(level)
        for p in self.level_patches(level):
            reg = self.region(p, substep)
            if self.physics == "isothermal":
                res = hydro.advance(p.cells, p.faces, dx, dt, reg, self.cs)
            else:
                res = mhd.advance(p.cells, p.faces, dx, dt, reg, self.gamma)
            p.old_cells, p.old_faces = p.cells, p.faces
            p.cells, p.faces = res.cells, res.faces
            if self.poison:
                self._poison_outside(p, reg)
            p.last = res
            p.last_dt = dt
            fdt = [f[:5] * dt for f in res.fluxes]
            edt = [e * dt for e in res.edges]
            if substep == 0 or p.facc is None:
                p.facc, p.eacc = fdt, edt
            else:
                p.facc = [a + b for a, b in zip(p.facc, fdt)]
                p.eacc = [a + b for a, b in zip(p.eacc, edt)]

    def _poison_outside(self, p, reg):
        keep = np.zeros(p.shape, dtype=bool)
        keep[mhd._sel(reg)] = True
        p.cells = np.where(keep[None], p.cells, np.nan)
        for d in range(3):
            kf = np.zeros(p.shape, dtype=bool)
            kf[mhd._face_sel(reg, d)] = True
            p.faces[d] = np.where(kf, p.faces[d], np.nan)

    # ------------------------------------------------------------------ coverage
    def coverage(self, m):
        """Child id covering each padded cell of parent m, -1 where uncovered."""
        cov = np.full(m.shape, -1, dtype=np.int64)
        mo = m.origin()
        for c in m.children:
            lo = c.lo // R - mo
            hi = c.hi // R - mo
            cov[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = c.id
        return cov

    # ------------------------------------------------------------------ restriction + corrections
    def restrict(self, fine_level):
        dxc = self.dx(fine_level - 1)
        for m in self.level_patches(fine_level - 1):
            if not m.children:
                continue
            cov = self.coverage(m)
            covered = cov >= 0
            mo = m.origin()
            # -- flux correction: dF at coverage-boundary faces (F*dt sums)
            dF = [np.zeros((5,) + m.shape) for _ in range(3)]
            for d in range(3):
                lo_cov = mhd.sh(cov, d, -1)       # cell on the low side of face (left face of each cell)
                hi_cov = cov
                bnd = (lo_cov >= 0) != (hi_cov >= 0)
                idx = np.argwhere(bnd)
                for (z, y, x) in idx:
                    cid = int(max(lo_cov[z, y, x], hi_cov[z, y, x]))
                    c = self.patches[cid]
                    # fine faces on this coarse face
                    cg = np.array([x, y, z]) + mo
                    f0 = R * cg - c.origin()
                    a1, a2 = [a for a in range(3) if a != d]
                    acc = np.zeros(5)
                    for t2 in (0, 1):
                        for t1 in (0, 1):
                            fi = f0.copy()
                            fi[a1] += t1
                            fi[a2] += t2
                            acc += c.facc[d][:, fi[2], fi[1], fi[0]]
                    dF[d][:, z, y, x] = 0.25 * acc - m.last.fluxes[d][:5, z, y, x] * m.last_dt
            corr = np.zeros((5,) + m.shape)
            for d in range(3):
                corr += (mhd.sh(dF[d], d, 1) - dF[d]) / dxc
            unc = ~covered
            m.cells = np.where(unc[None], m.cells - corr, m.cells)
            # -- EMF correction at coverage-boundary edges
            dE = [np.zeros(m.shape) for _ in range(3)]
            for e in range(3):
                a, c_ = (e + 1) % 3, (e + 2) % 3
                n_mm = mhd.sh(mhd.sh(cov, a, -1), c_, -1)
                n_0m = mhd.sh(cov, c_, -1)
                n_m0 = mhd.sh(cov, a, -1)
                n_00 = cov
                order = [n_mm, n_0m, n_m0, n_00]
                anyc = np.zeros(m.shape, dtype=bool)
                allc = np.ones(m.shape, dtype=bool)
                for nb in order:
                    anyc |= nb >= 0
                    allc &= nb >= 0
                bnd = anyc & ~allc
                for (z, y, x) in np.argwhere(bnd):
                    owner = next(int(nb[z, y, x]) for nb in order if nb[z, y, x] >= 0)
                    ch = self.patches[owner]
                    cg = np.array([x, y, z]) + mo
                    f0 = R * cg - ch.origin()
                    f1 = f0.copy()
                    f1[e] += 1
                    enew = 0.5 * (ch.eacc[e][f0[2], f0[1], f0[0]] + ch.eacc[e][f1[2], f1[1], f1[0]])
                    dE[e][z, y, x] = enew - m.last.edges[e][z, y, x] * m.last_dt
            for d in range(3):
                a, c_ = (d + 1) % 3, (d + 2) % 3
                curl = (mhd.sh(dE[c_], a, 1) - dE[c_]) / dxc - (mhd.sh(dE[a], c_, 1) - dE[a]) / dxc
                lo_cov = mhd.sh(cov, d, -1)
                unc_face = (lo_cov < 0) & (cov < 0)
                m.faces[d] = np.where(unc_face, m.faces[d] - curl, m.faces[d])
            # -- restriction of covered cells and closure faces
            for c in m.children:
                clo = c.lo // R - mo
                chi = c.hi // R - mo
                fi = c.interior_box()[0]
                fsum = np.zeros((5,) + tuple(int(x) for x in (c.n // R)[::-1]))
                cz, cy, cx = (int(x) for x in (c.n // R)[::-1])
                for oz in (0, 1):
                    for oy in (0, 1):
                        for ox in (0, 1):
                            fsum += c.cells[:, G + oz:G + oz + 2 * cz:2, G + oy:G + oy + 2 * cy:2,
                                            G + ox:G + ox + 2 * cx:2]
                m.cells[:, clo[2]:chi[2], clo[1]:chi[1], clo[0]:chi[0]] = 0.125 * fsum
                for d in range(3):
                    a1, a2 = [a for a in range(3) if a != d]
                    ext = [cx, cy, cz]
                    ext[d] += 1
                    fs = np.zeros((ext[2], ext[1], ext[0]))
                    for t2 in (0, 1):
                        for t1 in (0, 1):
                            off = [0, 0, 0]
                            off[a1] = t1
                            off[a2] = t2
                            step = [2, 2, 2]
                            st = [G + off[a] for a in range(3)]
                            fs += c.faces[d][st[2]:st[2] + 2 * ext[2]:2, st[1]:st[1] + 2 * ext[1]:2,
                                             st[0]:st[0] + 2 * ext[0]:2][:ext[2], :ext[1], :ext[0]]
                    hi = [int(x) for x in chi]
                    hi[d] += 1
                    m.faces[d][clo[2]:hi[2], clo[1]:hi[1], clo[0]:hi[0]] = 0.25 * fs

    # ------------------------------------------------------------------ same-level synchronisation
    def sync(self, level):
        """Compare fluxes / faces shared by same-level patches; average and correct when they differ."""
        lv = self.level_patches(level)
        for p in lv:
            for q in lv:
                for s in self._images(p, q):
                    if q is p and not np.any(s):
                        continue
                    for d in range(3):
                        for p_low in (True, False):
                            plane = p.lo[d] if p_low else p.hi[d]
                            qplane = (q.hi[d] if p_low else q.lo[d]) + s[d]
                            if plane != qplane:
                                continue
                            lo = np.maximum(p.lo, q.lo + s)
                            hi = np.minimum(p.hi, q.hi + s)
                            lo[d], hi[d] = plane, plane + 1
                            if np.any(hi <= lo):
                                continue
                            pa = lo - p.origin()
                            pb = hi - p.origin()
                            qa = lo - s - q.origin()
                            qb = hi - s - q.origin()
                            psel = (slice(pa[2], pb[2]), slice(pa[1], pb[1]), slice(pa[0], pb[0]))
                            qsel = (slice(qa[2], qb[2]), slice(qa[1], qb[1]), slice(qa[0], qb[0]))
                            fp = p.last.fluxes[d][(slice(0, 5),) + psel] * p.last_dt
                            fq = q.last.fluxes[d][(slice(0, 5),) + qsel] * q.last_dt
                            diff = float(np.max(np.abs(fq - fp)))
                            self.diag["sync_flux_max"] = max(self.diag["sync_flux_max"], diff)
                            bd = float(np.max(np.abs(p.faces[d][psel] - q.faces[d][qsel])))
                            self.diag["sync_face_max"] = max(self.diag["sync_face_max"], bd)
                            if diff > 0.0:
                                dx = self.dxv(level)[d]
                                delta = 0.5 * (fq - fp)
                                if p_low:       # the face is the left face of p's first interior cell
                                    p.cells[(slice(None),) + psel] += delta / dx
                                else:           # the face is the right face of p's last interior cell
                                    cs = list(psel)
                                    cs[2 - d] = slice(pa[d] - 1, pb[d] - 1)
                                    p.cells[(slice(None),) + tuple(cs)] -= delta / dx

    # ------------------------------------------------------------------ time step
    def cfl_dt(self):
        best = math.inf
        for lv in range(self.nlevels):
            smax = 0.0
            for p in self.level_patches(lv):
                if self.physics == "isothermal":
                    sig = hydro.max_signal(p.cells, self.dxv(lv), p.interior_box(), self.cs)
                else:
                    sig = mhd.max_signal(p.cells, p.faces, self.dxv(lv), p.interior_box(), self.gamma)
                smax = max(smax, sig)
            if smax > 0.0:
                best = min(best, R ** lv * self.cfl / smax)
        return best

    # ------------------------------------------------------------------ driver
    def root_step(self, dt0=None):
        if dt0 is None:
            dt0 = self.cfl_dt()
        self._amr(0, dt0)
        return dt0

    def _amr(self, level, dt):
        nsub = 1 if level == 0 else R
        for s in range(nsub):
            self.ghost_fill(level, s)
            self.advance_level(level, dt, s)
            if level + 1 < self.nlevels:
                self._amr(level + 1, dt / R)
                self.restrict(level + 1)
            self.sync(level)

    # ------------------------------------------------------------------ diagnostics
    def leaf_mask(self, p):
        m = self._interior_mask(p)
        if p.children:
            m &= self.coverage(p) < 0
        return m

    def conservation(self):
        """Exactly rounded sums over leaf cells of (rho, m, E, B_c) * dV."""
        terms = [[] for _ in range(8)]
        for p in self.patches:
            dv = float(np.prod(self.dxv(p.level)))
            m = self.leaf_mask(p)
            bc = mhd.cell_centred_b(p.faces)
            for c in range(5):
                terms[c].append((p.cells[c][m] * dv).ravel())
            for c in range(3):
                terms[5 + c].append((bc[c][m] * dv).ravel())
        return np.array([math.fsum(np.concatenate(t)) for t in terms])

    def max_divergence(self):
        out = 0.0
        for p in self.patches:
            dv = mhd.divergence(p.faces, self.dxv(p.level))
            out = max(out, float(np.max(np.abs(dv[self._interior_mask(p)]))))
        return out


def build(spec, field=None, gamma=5.0 / 3.0, cfl=0.4, ghosts="extended", physics="mhd", cs=1.0):
    """Hierarchy from a workloads HierarchySpec (and optional initial field)."""
    h = Hierarchy(spec.root_n, gamma=gamma, cfl=cfl, ghosts=ghosts, physics=physics, cs=cs)
    for lv, lo, hi in spec.patches:
        h.add(lv, lo, hi)
    h.freeze()
    if field is not None:
        h.set_state(field)
    return h
