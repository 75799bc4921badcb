"""One substep of the unsplit MUSCL-Hancock / HLLD / constrained-transport advance.

TEST INFRASTRUCTURE ONLY (see the package docstring): float64 NumPy, written
for readability, not speed.

What the paper fixes and what it leaves open
--------------------------------------------
The paper (Sec. 2, Sec. 2.3 "Isolated Grids") fixes the structure: grids hold
cells plus ghost cells; a refined grid takes R substeps per parent step and,
with extended ghost cells, first updates a region R*n_ghost wide and then
successively smaller regions (Sec. 2.3; worked 2-D example in Sec. 4).  It
names the physics only as "hyperbolic advances" of MHD (title, abstract) and
describes no solver.  The numerical method below is therefore a stated
reading built from published methods:

  * ideal MHD, gamma-law gas, Heaviside-Lorentz units (magnetic pressure B^2/2);
  * primitive variables w = (rho, vx, vy, vz, p, Bx, By, Bz) with the
    cell-centred field the mean of the two bounding face values;
  * monotonised-central (van Leer) limited slopes of the primitives per axis;
  * conservative Hancock half step using all three axes (Toro, MUSCL-Hancock),
    face-normal field advanced half a step by the discrete Stokes update of
    edge-averaged cell EMFs;
  * HLLD approximate Riemann solver (Miyoshi & Kusano 2005, J. Comput. Phys.
    208, 315) with the face-normal field taken from the half-step face value;
  * edge EMFs by the upwinded "CT-contact" rule (Gardiner & Stone 2005,
    J. Comput. Phys. 205, 509);
  * conservative cell update and discrete Stokes update of the face field.

Array conventions: every array of a patch has the node-padded shape
(NZ+1, NY+1, NX+1), indexed [z][y][x]; cells use [0, N) per axis; the x-face
array entry [k, j, i] is the face at x = i - 1/2 (left face of cell i); the
z-edge array entry [k, j, i] is the edge at (i - 1/2, j - 1/2, k) and
cyclically for the x- and y-edges.  Stages are evaluated on whole arrays with
periodic index shifts; the wrapped values at the array border never reach the
update region because it lies at least 2 cells (the stencil depth) inside the
valid data (checked by the poison tests).
"""
from __future__ import annotations

import numpy as np

N_G = 2                      # stencil depth of one substep (cells)
DEGEN_REL = 1e-8             # HLLD star-state degeneracy threshold (relative)
BN_SKIP_REL = 1e-12          # HLLD: skip double-star states when Bn^2 <= this * (ptL + ptR)
MASS_FLUX_ZERO = 1e-12       # HLLD: a mass flux at most this * max(rho) * max(|S|) is exactly zero


class PhysicsError(RuntimeError):
    """Non-positive density or pressure, or a non-finite value, inside the region."""


# ---------------------------------------------------------------------------
# index helpers
# ---------------------------------------------------------------------------

def npax(d):
    """NumPy axis of spatial axis d (0=x, 1=y, 2=z) for a 3-D [z][y][x] array."""
    return 2 - d


def sh(a, d, s):
    """b[..., i, ...] = a[..., i + s, ...] along spatial axis d (periodic wrap)."""
    ax = a.ndim - 1 - d
    return np.roll(a, -s, axis=ax)


# ---------------------------------------------------------------------------
# pointwise physics
# ---------------------------------------------------------------------------

def cell_centred_b(faces):
    """Cell-centred field: mean of the two bounding face values per axis."""
    return np.stack([0.5 * (faces[d] + sh(faces[d], d, 1)) for d in range(3)])


def prim_from_cons(u, bc, gamma):
    """w = (rho, v, p, B) from conserved (rho, m, E) and the cell-centred field."""
    rho = u[0]
    v = u[1:4] / rho
    kin = 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / rho
    mag = 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)
    p = (gamma - 1.0) * (u[4] - kin - mag)
    return np.concatenate([rho[None], v, p[None], bc])


def cons_from_prim(w, gamma):
    """Eight conserved components (rho, m, E, B) from primitives."""
    rho, vx, vy, vz, p, bx, by, bz = w
    e = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, e, bx, by, bz])


def flux(w, d, gamma):
    """Ideal-MHD flux along axis d of the eight conserved components."""
    rho, p = w[0], w[4]
    v = w[1:4]
    b = w[5:8]
    un, bn = v[d], b[d]
    b2 = b[0] ** 2 + b[1] ** 2 + b[2] ** 2
    pt = p + 0.5 * b2
    e = p / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) + 0.5 * b2
    vb = v[0] * b[0] + v[1] * b[1] + v[2] * b[2]
    f = np.empty((8,) + rho.shape)
    f[0] = rho * un
    for c in range(3):
        f[1 + c] = rho * v[c] * un - b[c] * bn
    f[1 + d] += pt
    f[4] = (e + pt) * un - bn * vb
    for c in range(3):
        f[5 + c] = b[c] * un - bn * v[c]
    f[5 + d] = 0.0
    return f


def fast_speed(rho, p, b2, bn2, gamma):
    """Fast magnetosonic speed along a direction with normal field squared bn2."""
    a2 = gamma * p / rho
    s = a2 + b2 / rho
    disc = np.maximum(s * s - 4.0 * a2 * bn2 / rho, 0.0)
    return np.sqrt(0.5 * (s + np.sqrt(disc)))


def mc_slope(dm, dp):
    """Monotonised-central limited slope: minmod(2 dm, 2 dp, (dm + dp)/2)."""
    same = dm * dp > 0.0
    mag = np.minimum(np.minimum(2.0 * np.abs(dm), 2.0 * np.abs(dp)), 0.5 * np.abs(dm + dp))
    return np.where(same, np.sign(dm) * mag, 0.0)


# ---------------------------------------------------------------------------
# HLLD (Miyoshi & Kusano 2005)
# ---------------------------------------------------------------------------

def hlld(wl, wr, bn, d, gamma):
    """HLLD flux across a face normal to axis d.

    wl, wr: primitive states (8, ...) left and right of the face; their
    normal field components are ignored and ``bn`` is used for both.
    Returns the eight-component flux in the global component order.
    Region selection: F_L if S_L >= 0, else F*_L if S*_L >= 0, else F**_L if
    S_M >= 0, else F**_R if S*_R >= 0, else F*_R if S_R >= 0, else F_R (ties
    go to the left-hand region).  Degenerate star states (Miyoshi & Kusano's
    vanishing denominator) keep the transverse velocity and field unchanged:
    with S_M = u the general formulas tend to exactly these values as the
    transverse field vanishes, so the switch introduces no jump;
    when Bn^2 is negligible against the total pressures the rotational waves
    collapse onto S_M and the double-star states are skipped.
    A mass flux no larger than MASS_FLUX_ZERO * max(rho_L, rho_R) *
    max(|S_L|, |S_R|) is set to exactly zero: it vanishes in exact arithmetic
    (a stagnant face ahead of a flow front), and the edge EMFs choose their
    upwind side by its sign, a choice that jumps at zero.
    """
    t1, t2 = (d + 1) % 3, (d + 2) % 3
    g1 = gamma - 1.0

    def local(w):
        return (w[0], w[1 + d], w[1 + t1], w[1 + t2], w[4], w[5 + t1], w[5 + t2])

    rl, ul, vl, zl, pl, byl, bzl = local(wl)
    rr, ur, vr, zr, pr, byr, bzr = local(wr)
    bn2 = bn * bn
    b2l = bn2 + byl * byl + bzl * bzl
    b2r = bn2 + byr * byr + bzr * bzr
    cfl = fast_speed(rl, pl, b2l, bn2, gamma)
    cfr = fast_speed(rr, pr, b2r, bn2, gamma)
    cmax = np.maximum(cfl, cfr)
    sl = np.minimum(ul, ur) - cmax
    sr = np.maximum(ul, ur) + cmax
    ptl = pl + 0.5 * b2l
    ptr = pr + 0.5 * b2r
    el = pl / g1 + 0.5 * rl * (ul * ul + vl * vl + zl * zl) + 0.5 * b2l
    er = pr / g1 + 0.5 * rr * (ur * ur + vr * vr + zr * zr) + 0.5 * b2r
    vbl = ul * bn + vl * byl + zl * bzl
    vbr = ur * bn + vr * byr + zr * bzr

    ul_ = np.stack([rl, rl * ul, rl * vl, rl * zl, el, byl, bzl])
    ur_ = np.stack([rr, rr * ur, rr * vr, rr * zr, er, byr, bzr])
    fl = np.stack([rl * ul, rl * ul * ul + ptl - bn2, rl * ul * vl - bn * byl, rl * ul * zl - bn * bzl,
                   (el + ptl) * ul - bn * vbl, byl * ul - bn * vl, bzl * ul - bn * zl])
    fr = np.stack([rr * ur, rr * ur * ur + ptr - bn2, rr * ur * vr - bn * byr, rr * ur * zr - bn * bzr,
                   (er + ptr) * ur - bn * vbr, byr * ur - bn * vr, bzr * ur - bn * zr])

    sdl = sl - ul
    sdr = sr - ur
    den = sdr * rr - sdl * rl
    sm = (sdr * rr * ur - sdl * rl * ul - ptr + ptl) / den
    pts = (sdr * rr * ptl - sdl * rl * ptr + rl * rr * sdr * sdl * (ur - ul)) / den

    def star(r, u, v, z, by, bz, e, pt, vb, s, sd):
        rs = r * sd / (s - sm)
        dn = r * sd * (s - sm) - bn2
        degen = np.abs(dn) <= DEGEN_REL * r * sd * sd
        dn_safe = np.where(degen, 1.0, dn)
        vs = np.where(degen, v, v - bn * by * (sm - u) / dn_safe)
        zs = np.where(degen, z, z - bn * bz * (sm - u) / dn_safe)
        num = r * sd * sd - bn2
        bys = np.where(degen, by, by * num / dn_safe)
        bzs = np.where(degen, bz, bz * num / dn_safe)
        vbs = sm * bn + vs * bys + zs * bzs
        es = (sd * e - pt * u + pts * sm + bn * (vb - vbs)) / (s - sm)
        return rs, vs, zs, bys, bzs, es, vbs

    rls, vls, zls, byls, bzls, els, vbls = star(rl, ul, vl, zl, byl, bzl, el, ptl, vbl, sl, sdl)
    rrs, vrs, zrs, byrs, bzrs, ers, vbrs = star(rr, ur, vr, zr, byr, bzr, er, ptr, vbr, sr, sdr)

    usl = np.stack([rls, rls * sm, rls * vls, rls * zls, els, byls, bzls])
    usr = np.stack([rrs, rrs * sm, rrs * vrs, rrs * zrs, ers, byrs, bzrs])
    fsl = fl + sl * (usl - ul_)
    fsr = fr + sr * (usr - ur_)

    sql = np.sqrt(rls)
    sqr = np.sqrt(rrs)
    sgn = np.sign(bn)
    abn = np.abs(bn)
    ssl = sm - abn / sql
    ssr = sm + abn / sqr
    inv = 1.0 / (sql + sqr)
    vss = (sql * vls + sqr * vrs + (byrs - byls) * sgn) * inv
    zss = (sql * zls + sqr * zrs + (bzrs - bzls) * sgn) * inv
    byss = (sql * byrs + sqr * byls + sql * sqr * (vrs - vls) * sgn) * inv
    bzss = (sql * bzrs + sqr * bzls + sql * sqr * (zrs - zls) * sgn) * inv
    vbss = sm * bn + vss * byss + zss * bzss
    elss = els - sql * (vbls - vbss) * sgn
    erss = ers + sqr * (vbrs - vbss) * sgn
    ussl = np.stack([rls, rls * sm, rls * vss, rls * zss, elss, byss, bzss])
    ussr = np.stack([rrs, rrs * sm, rrs * vss, rrs * zss, erss, byss, bzss])
    fssl = fsl + ssl * (ussl - usl)
    fssr = fsr + ssr * (ussr - usr)

    skip = bn2 <= BN_SKIP_REL * (ptl + ptr)
    f = np.where(sl >= 0.0, fl,
        np.where(skip,
                 np.where(sm >= 0.0, fsl, np.where(sr >= 0.0, fsr, fr)),
                 np.where(ssl >= 0.0, fsl,
                 np.where(sm >= 0.0, fssl,
                 np.where(ssr >= 0.0, fssr,
                 np.where(sr >= 0.0, fsr, fr))))))
    out = np.zeros((8,) + rl.shape)
    scale = np.maximum(rl, rr) * np.maximum(np.abs(sl), np.abs(sr))
    out[0] = np.where(np.abs(f[0]) <= MASS_FLUX_ZERO * scale, 0.0, f[0])
    out[1 + d] = f[1]
    out[1 + t1] = f[2]
    out[1 + t2] = f[3]
    out[4] = f[4]
    out[5 + d] = 0.0
    out[5 + t1] = f[5]
    out[5 + t2] = f[6]
    return out


# ---------------------------------------------------------------------------
# the substep
# ---------------------------------------------------------------------------

def grow(box, g):
    lo, hi = box
    return (tuple(x - g for x in lo), tuple(x + g for x in hi))


def _sel(box):
    (x0, y0, z0), (x1, y1, z1) = box
    return (slice(z0, z1), slice(y0, y1), slice(x0, x1))


def _face_sel(box, d):
    """Faces of the cells of ``box`` normal to axis d (closure along d)."""
    lo, hi = box
    hi = list(hi)
    hi[d] += 1
    return _sel((lo, tuple(hi)))


def _edge_sel(box, e):
    """Edges along axis e bounding the faces of ``box`` (closure across e)."""
    lo, hi = box
    hi = list(hi)
    for a in range(3):
        if a != e:
            hi[a] += 1
    return _sel((lo, tuple(hi)))


def _check(name, arrs, sel):
    for a in arrs:
        v = a[(slice(None),) + sel] if a.ndim == 4 else a[sel]
        if not np.all(np.isfinite(v)):
            raise PhysicsError(f"{name}: non-finite value")
    return True


def edge_emf(ef_a, ef_b, eref, fa_rho, fb_rho, a, b):
    """CT-contact EMF along axis e = third axis of (a, b), on the edge array.

    ef_a: EMF component e carried by the faces normal to a (stored at the
    left face of each cell); ef_b: the same component on the faces normal to
    b; eref: the cell-centred reference EMF at the half step; fa_rho, fb_rho:
    mass fluxes through the a- and b-faces (upwind selectors).  The edge at
    array index (i_a, i_b) sits at (i_a - 1/2, i_b - 1/2) in the (a, b) plane.
    Each of the four face EMFs is carried to the edge with a gradient taken
    on the upwind side of the face's transverse mass flux (average when the
    mass flux vanishes), following Gardiner & Stone (2005).
    """
    # face values adjacent to edge (a-1/2, b-1/2)
    ea_bm = sh(ef_a, b, -1)      # a-face at (a-1/2, b-1)
    ea_b0 = ef_a                 # a-face at (a-1/2, b)
    eb_am = sh(ef_b, a, -1)      # b-face at (a-1, b-1/2)
    eb_a0 = ef_b                 # b-face at (a, b-1/2)
    r_mm = sh(sh(eref, a, -1), b, -1)   # cell (a-1, b-1)
    r_0m = sh(eref, b, -1)               # cell (a,   b-1)
    r_m0 = sh(eref, a, -1)               # cell (a-1, b)
    r_00 = eref                          # cell (a,   b)

    def upwind(flux, minus_val, plus_val):
        return np.where(flux > 0.0, minus_val, np.where(flux < 0.0, plus_val, 0.5 * (minus_val + plus_val)))

    # d/db between face centre b and the edge, at a-1/2: upwind by the a-face mass flux at (a-1/2, b)
    d_b_upper = upwind(fa_rho, r_m0 - eb_am, r_00 - eb_a0)
    # d/db between cell b-1 and the edge: upwind by the a-face mass flux at (a-1/2, b-1)
    d_b_lower = upwind(sh(fa_rho, b, -1), eb_am - r_mm, eb_a0 - r_0m)
    # d/da between edge and centre a, at b-1/2: upwind by the b-face mass flux at (a, b-1/2)
    d_a_upper = upwind(fb_rho, r_0m - ea_bm, r_00 - ea_b0)
    # d/da between cell a-1 and the edge: upwind by the b-face mass flux at (a-1, b-1/2)
    d_a_lower = upwind(sh(fb_rho, a, -1), ea_bm - r_mm, ea_b0 - r_m0)
    return 0.25 * (ea_bm + ea_b0 + eb_am + eb_a0) + 0.25 * (d_b_lower - d_b_upper) + 0.25 * (d_a_lower - d_a_upper)


class StepResult:
    """Output of one substep: new arrays plus the fluxes and EMFs it used."""

    def __init__(self, cells, faces, fluxes, edges, max_signal=None):
        self.cells = cells          # (5, ...) conserved after the update (outside the region: input)
        self.faces = faces          # [bx, by, bz] after the update (outside the region closure: input)
        self.fluxes = fluxes        # per axis d: (8, ...) flux at the left face of each cell
        self.edges = edges          # per axis e: edge EMF array


def advance(cells, faces, dx, dt, region, gamma):
    """Advance a padded patch by dt over ``region`` (cell box in padded indices).

    Cells inside the region and faces on the closure of the region are updated;
    everything else is returned unchanged.  Valid input is required on the
    region grown by N_G cells (and the faces of those cells).
    """
    dx = np.asarray(dx, dtype=np.float64)
    u = cells
    b = faces
    rp2 = grow(region, 2)
    with np.errstate(all='ignore'):
        bc = cell_centred_b(b)
        w = prim_from_cons(u, bc, gamma)
        s_w = w[(slice(None),) + _sel(rp2)]
        if not (np.all(np.isfinite(s_w)) and np.all(s_w[0] > 0) and np.all(s_w[4] > 0)):
            raise PhysicsError("cell state: rho<=0, p<=0 or non-finite")

        # limited slopes per axis
        slope = [mc_slope(w - sh(w, d, -1), sh(w, d, 1) - w) for d in range(3)]

        # conservative Hancock half step from all three axes
        du = np.zeros((8,) + u.shape[1:])
        for d in range(3):
            fp = flux(w + 0.5 * slope[d], d, gamma)
            fm = flux(w - 0.5 * slope[d], d, gamma)
            du -= (0.5 * dt / dx[d]) * (fp - fm)

        # face-normal field at the half step from edge-averaged cell EMFs at t^n
        v = w[1:4]
        ec = -np.cross(v, bc, axis=0)              # cell EMF, (3, ...)
        ebar = []
        for e in range(3):
            a, c = (e + 1) % 3, (e + 2) % 3
            ebar.append(0.25 * (ec[e] + sh(ec[e], a, -1) + sh(ec[e], c, -1) + sh(sh(ec[e], a, -1), c, -1)))
        bh = []
        for d in range(3):
            a, c = (d + 1) % 3, (d + 2) % 3
            # curl_d E = dE_c/da - dE_a/dc  (d, a, c cyclic)
            curl = (sh(ebar[c], a, 1) - ebar[c]) / dx[a] - (sh(ebar[a], c, 1) - ebar[a]) / dx[c]
            bh.append(b[d] - 0.5 * dt * curl)

        # half-step cell state and CT reference EMF
        uh = np.concatenate([u, bc]) + du
        vh = uh[1:4] / uh[0]
        bch = cell_centred_b(bh)
        eref = -np.cross(vh, bch, axis=0)

        # face states at the half step and HLLD fluxes
        fl = []
        for d in range(3):
            up = cons_from_prim(w + 0.5 * slope[d], gamma) + du
            um = cons_from_prim(w - 0.5 * slope[d], gamma) + du
            wp = prim_from_cons(up[:5], up[5:], gamma)
            wm = prim_from_cons(um[:5], um[5:], gamma)
            wl = sh(wp, d, -1)       # + state of the cell on the left of face i-1/2
            wr = wm
            # check the states of the faces whose fluxes feed the region and its edges
            flo = [x - 1 for x in region[0]]
            fhi = [x + 1 for x in region[1]]
            flo[d] += 1
            fsel = _sel((tuple(flo), tuple(fhi)))
            for chk in (wl, wr):
                cc = chk[(slice(None),) + fsel]
                if not (np.all(np.isfinite(cc)) and np.all(cc[0] > 0) and np.all(cc[4] > 0)):
                    raise PhysicsError("face state: rho<=0, p<=0 or non-finite")
            fl.append(hlld(wl, wr, bh[d], d, gamma))

        # CT-contact edge EMFs
        edges = []
        for e in range(3):
            a, c = (e + 1) % 3, (e + 2) % 3
            # EMF component e on faces normal to a: E_e = -(F_a)[B_c] ; normal to c: E_e = +(F_c)[B_a]
            ef_a = -fl[a][5 + c]
            ef_c = fl[c][5 + a]
            edges.append(edge_emf(ef_a, ef_c, eref[e], fl[a][0], fl[c][0], a, c))

        # conservative update and Stokes update of the faces
        new_u = u.copy()
        div = np.zeros_like(u)
        for d in range(3):
            div += (sh(fl[d][:5], d, 1) - fl[d][:5]) / dx[d]
        sel = _sel(region)
        new_u[(slice(None),) + sel] = u[(slice(None),) + sel] - dt * div[(slice(None),) + sel]
        new_b = [x.copy() for x in b]
        for d in range(3):
            a, c = (d + 1) % 3, (d + 2) % 3
            curl = (sh(edges[c], a, 1) - edges[c]) / dx[a] - (sh(edges[a], c, 1) - edges[a]) / dx[c]
            fs = _face_sel(region, d)
            new_b[d][fs] = b[d][fs] - dt * curl[fs]
    res_sel = (slice(None),) + sel
    if not np.all(np.isfinite(new_u[res_sel])):
        raise PhysicsError("updated state non-finite")
    return StepResult(new_u, new_b, fl, edges)


def max_signal(cells, faces, dx, box, gamma):
    """max over the cells of ``box`` of sum_d (|v_d| + c_f,d) / dx_d."""
    with np.errstate(all='ignore'):
        bc = cell_centred_b(faces)
        w = prim_from_cons(cells, bc, gamma)
    sel = (slice(None),) + _sel(box)
    w = w[sel]
    b2 = w[5] ** 2 + w[6] ** 2 + w[7] ** 2
    tot = np.zeros_like(w[0])
    for d in range(3):
        tot += (np.abs(w[1 + d]) + fast_speed(w[0], w[4], b2, w[5 + d] ** 2, gamma)) / dx[d]
    return float(np.max(tot))


def divergence(faces, dx):
    """Discrete divergence of the face field per cell (cell-shaped array)."""
    return sum((sh(faces[d], d, 1) - faces[d]) / dx[d] for d in range(3))
