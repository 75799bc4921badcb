"""Seeded synthetic initial states for ghost-padded patches.

This module is shared by the CPU oracle and the HIP path as their common
source of inputs.  It holds none of the solver's arithmetic: it only builds
initial conditions (smooth random fields, an off-centre blast, a low-beta
variant, the Brio-Wu shock tube) on a patch's padded index box.

Conventions (shared with the library's memory layout):
  * a patch at level ``l`` covers the index box [lo, hi) of the level-l grid,
    whose cells have width h = 1 / (root_n * 2**l) on the unit cube;
  * arrays are padded by ``G`` ghost cells on every side, indexed [z][y][x]
    with x fastest;
  * every array of a patch uses the same node-padded shape
    (NZ+1, NY+1, NX+1) with NX = nx + 2G: cells use [0, NX) per axis and the
    trailing plane/row/column is unused; the x-face array ``bx[k, j, i]`` is
    the face at x = (i - 1/2) h (left face of cell i), likewise for y and z;
  * conserved cell variables are (rho, m_x, m_y, m_z, E); face variables are
    the face-normal magnetic field components (b_x, b_y, b_z).

Smooth fields are exact cell averages (for rho and momentum) and exact face
averages (for b, obtained by Stokes' theorem from exact edge averages of a
vector potential), so the data are consistent across refinement levels and
the discrete divergence of b vanishes to round-off.  Total energy is built
from a uniform pressure p0 with the ideal-gas closure in Heaviside-Lorentz
units (magnetic pressure |B|^2/2), using the cell-centred field taken as the
mean of the two bounding face values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

G = 4  # allocated ghost cells per side (= refinement ratio 2 x stencil depth 2)


def padded_shape(n):
    """Node-padded array shape (z, y, x) for a patch with interior sizes n=(nx,ny,nz)."""
    nx, ny, nz = n
    return (nz + 2 * G + 1, ny + 2 * G + 1, nx + 2 * G + 1)


# ----------------------------------------------------------------------------
# random Fourier series with exact cell / face / edge averages
# ----------------------------------------------------------------------------

def _half_modes(kmax):
    """Integer wave vectors with 0 < |k|_2 <= kmax, one of each +-k pair."""
    ks = []
    r = int(math.floor(kmax))
    for kz in range(-r, r + 1):
        for ky in range(-r, r + 1):
            for kx in range(-r, r + 1):
                if kx * kx + ky * ky + kz * kz == 0 or kx * kx + ky * ky + kz * kz > kmax * kmax:
                    continue
                # keep the half space (first nonzero of (kz, ky, kx) positive)
                first = kz if kz != 0 else (ky if ky != 0 else kx)
                if first > 0:
                    ks.append((kx, ky, kz))
    return np.array(ks, dtype=np.int64)


@dataclass
class Series:
    """f(x) = Re sum_k c_k exp(2 pi i k.x) over a half set of modes."""
    k: np.ndarray          # (M, 3) integer wave vectors (x, y, z)
    c: np.ndarray          # (M,) complex coefficients

    def rms(self):
        # mean over the unit cube of (Re sum c e^{i..})^2 = 1/2 sum |c|^2
        return math.sqrt(0.5 * float(np.sum(np.abs(self.c) ** 2)))


def random_series(rng, kmax=4.0, ncomp=1):
    ks = _half_modes(kmax)
    out = []
    for _ in range(ncomp):
        c = rng.standard_normal(len(ks)) + 1j * rng.standard_normal(len(ks))
        out.append(Series(ks, c))
    return out


def _axis_factor(k1d, pos, h, averaged):
    """(K, P) matrix exp(2 pi i k x) times sinc(k h) when averaged along this axis."""
    e = np.exp(2j * np.pi * np.outer(k1d, pos))
    if averaged:
        e = e * np.sinc(k1d * h)[:, None]
    return e


def eval_series(s: Series, xs, ys, zs, h, avg=(True, True, True)):
    """Evaluate the series at the tensor grid (zs, ys, xs); averages along axes with avg[d].

    Every output value is formed by the same fixed sequence of operations on
    its own three coordinates, so equal coordinates give bitwise equal values
    whatever the array shape (patches that share a face or a periodic image
    receive identical data).
    """
    kmin = int(s.k.min())
    kmax = int(s.k.max())
    kr = np.arange(kmin, kmax + 1)
    nk = len(kr)
    coef = np.zeros((nk, nk, nk), dtype=np.complex128)  # [kz, ky, kx]
    np.add.at(coef, (s.k[:, 2] - kmin, s.k[:, 1] - kmin, s.k[:, 0] - kmin), s.c)
    Ex = _axis_factor(kr, xs, h[0], avg[0])
    Ey = _axis_factor(kr, ys, h[1], avg[1])
    Ez = _axis_factor(kr, zs, h[2], avg[2])
    t1 = np.zeros((len(zs), nk, nk), dtype=np.complex128)       # [z, ky, kx]
    for a in range(nk):
        t1 += Ez[a][:, None, None] * coef[a][None, :, :]
    t2 = np.zeros((len(zs), len(ys), nk), dtype=np.complex128)  # [z, y, kx]
    for b in range(nk):
        t2 += t1[:, b, None, :] * Ey[b][None, :, None]
    out = np.zeros((len(zs), len(ys), len(xs)))
    for c in range(nk):
        out += (t2[:, :, c, None] * Ex[c][None, None, :]).real
    return out


# ----------------------------------------------------------------------------
# patch state container
# ----------------------------------------------------------------------------

@dataclass
class PatchState:
    cells: np.ndarray      # (5, NZ+1, NY+1, NX+1) float64
    faces: list            # [bx, by, bz], each (NZ+1, NY+1, NX+1) float64


def _coords(level, root_n, lo, hi):
    """Cell-centre and face coordinates along each axis of the padded box."""
    h = [1.0 / (root_n[d] * 2 ** level) for d in range(3)]
    centres, lefts = [], []
    for d in range(3):
        n_l = root_n[d] * 2 ** level
        # periodic images share one reduced index, hence bitwise identical data
        idx = np.mod(np.arange(lo[d] - G, hi[d] + G + 1), n_l).astype(np.float64)  # node-padded length
        centres.append((idx + 0.5) * h[d])
        lefts.append(idx * h[d])
    return h, centres, lefts


def _total_energy(rho, mom, bc, p, gamma):
    return p / (gamma - 1.0) + 0.5 * (mom[0] ** 2 + mom[1] ** 2 + mom[2] ** 2) / rho \
        + 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)


def _cell_mean_of_faces(faces):
    bx, by, bz = faces
    out = []
    a = np.full_like(bx, np.nan)
    a[:, :, :-1] = 0.5 * (bx[:, :, :-1] + bx[:, :, 1:])
    out.append(a)
    a = np.full_like(by, np.nan)
    a[:, :-1, :] = 0.5 * (by[:, :-1, :] + by[:, 1:, :])
    out.append(a)
    a = np.full_like(bz, np.nan)
    a[:-1, :, :] = 0.5 * (bz[:-1, :, :] + bz[1:, :, :])
    out.append(a)
    return out


class SmoothField:
    """Smooth random MHD state: rho = 1 + A_rho n(x), p = p0, m and dB random, B0 uniform."""

    def __init__(self, seed, a_rho=0.1, v_rms=0.1, db_rms=0.1, b0=(1.0, 0.0, 0.0),
                 p0=1.0, gamma=5.0 / 3.0, kmax=4.0):
        rng = np.random.Generator(np.random.PCG64(seed))
        (self.n,) = random_series(rng, kmax, 1)
        self.m = random_series(rng, kmax, 3)
        self.a = random_series(rng, kmax, 3)  # vector potential components
        self.a_rho = a_rho / self.n.rms()
        vr = math.sqrt(sum(s.rms() ** 2 for s in self.m))
        self.m_scale = v_rms / vr
        # rms of curl A = sqrt(1/2 sum_k |2 pi k x a_k|^2)
        ks = self.a[0].k.astype(np.float64)
        ac = np.stack([s.c for s in self.a], axis=1)  # (M, 3)
        curl = 2j * np.pi * np.cross(ks, ac)
        crms = math.sqrt(0.5 * float(np.sum(np.abs(curl) ** 2)))
        self.a_scale = db_rms / crms
        self.b0 = tuple(float(b) for b in b0)
        self.p0 = p0
        self.gamma = gamma

    def patch(self, level, root_n, lo, hi):
        h, c, l = _coords(level, root_n, lo, hi)
        xs, ys, zs = c
        xl, yl, zl = l
        rho = 1.0 + self.a_rho * eval_series(self.n, xs, ys, zs, h)
        mom = [self.m_scale * eval_series(s, xs, ys, zs, h) for s in self.m]
        # exact edge averages of A: A_x on x-edges centred (x_c, y_l, z_l), etc.
        ax = self.a_scale * eval_series(self.a[0], xs, yl, zl, h, avg=(True, False, False))
        ay = self.a_scale * eval_series(self.a[1], xl, ys, zl, h, avg=(False, True, False))
        az = self.a_scale * eval_series(self.a[2], xl, yl, zs, h, avg=(False, False, True))
        shape = rho.shape
        nan = np.full(shape, np.nan)
        # face average of curl A by Stokes over the face perimeter
        bx = nan.copy()
        bx[:-1, :-1, :] = (az[:-1, 1:, :] - az[:-1, :-1, :]) / h[1] - (ay[1:, :-1, :] - ay[:-1, :-1, :]) / h[2]
        by = nan.copy()
        by[:-1, :, :-1] = (ax[1:, :, :-1] - ax[:-1, :, :-1]) / h[2] - (az[:-1, :, 1:] - az[:-1, :, :-1]) / h[0]
        bz = nan.copy()
        bz[:, :-1, :-1] = (ay[:, :-1, 1:] - ay[:, :-1, :-1]) / h[0] - (ax[:, 1:, :-1] - ax[:, :-1, :-1]) / h[1]
        bx += self.b0[0]
        by += self.b0[1]
        bz += self.b0[2]
        faces = [bx, by, bz]
        bc = _cell_mean_of_faces(faces)
        e = _total_energy(rho, mom, bc, self.p0, self.gamma)
        cells = np.stack([rho, mom[0], mom[1], mom[2], e])
        return _clean(PatchState(cells, faces))


class Blast:
    """Off-centre pressure blast: p = p_in inside |x - c| < r, p_out outside, rho = 1, v = 0, uniform B."""

    def __init__(self, centre, radius=0.1, p_in=100.0, p_out=1.0, b=(1 / math.sqrt(2), 1 / math.sqrt(2), 0.0),
                 gamma=5.0 / 3.0):
        self.c = np.asarray(centre, dtype=np.float64)
        self.r = radius
        self.p_in, self.p_out = p_in, p_out
        self.b = tuple(float(x) for x in b)
        self.gamma = gamma

    def patch(self, level, root_n, lo, hi):
        h, c, _ = _coords(level, root_n, lo, hi)
        zz, yy, xx = np.meshgrid(c[2], c[1], c[0], indexing='ij')
        # periodic minimum-image distance to the centre
        dx = [(a - self.c[d] + 0.5) % 1.0 - 0.5 for d, a in enumerate((xx, yy, zz))]
        r2 = dx[0] ** 2 + dx[1] ** 2 + dx[2] ** 2
        p = np.where(r2 < self.r * self.r, self.p_in, self.p_out)
        rho = np.ones_like(p)
        mom = [np.zeros_like(p) for _ in range(3)]
        faces = [np.full_like(p, self.b[d]) for d in range(3)]
        bc = [np.full_like(p, self.b[d]) for d in range(3)]
        e = _total_energy(rho, mom, bc, p, self.gamma)
        return _clean(PatchState(np.stack([rho, mom[0], mom[1], mom[2], e]), faces))


class PlaneRiemann:
    """Plane-parallel two-state problem along x on a doubled periodic domain [L | R | L].

    States are given as primitive tuples (rho, vx, vy, vz, p, Bx, By, Bz); cells with
    centre in [1/4, 3/4) take the right state.  Bx must be equal on both sides.
    """

    def __init__(self, left, right, gamma):
        assert left[5] == right[5]
        self.l, self.r, self.gamma = left, right, gamma

    def patch(self, level, root_n, lo, hi):
        h, c, _ = _coords(level, root_n, lo, hi)
        zz, yy, xx = np.meshgrid(c[2], c[1], c[0], indexing='ij')
        x = xx % 1.0
        inside = (x >= 0.25) & (x < 0.75)
        def pick(q):
            return np.where(inside, self.r[q], self.l[q])
        rho = pick(0)
        vel = [pick(1), pick(2), pick(3)]
        p = pick(4)
        bcell = [pick(5), pick(6), pick(7)]
        mom = [rho * v for v in vel]
        # face values: By, Bz are constant inside a cell column in x; y/z faces take the cell value
        faces = [np.full_like(rho, self.l[5]), bcell[1].copy(), bcell[2].copy()]
        e = _total_energy(rho, mom, bcell, p, self.gamma)
        return _clean(PatchState(np.stack([rho, mom[0], mom[1], mom[2], e]), faces))


def _clean(ps: PatchState) -> PatchState:
    """Zero the unused trailing node-padding entries so arrays are finite everywhere."""
    c = ps.cells
    c[:, -1, :, :] = 0.0
    c[:, :, -1, :] = 0.0
    c[:, :, :, -1] = 0.0
    bx, by, bz = ps.faces
    bx[-1, :, :] = 0.0
    bx[:, -1, :] = 0.0
    by[-1, :, :] = 0.0
    by[:, :, -1] = 0.0
    bz[:, -1, :] = 0.0
    bz[:, :, -1] = 0.0
    for a in (c, bx, by, bz):
        np.nan_to_num(a, copy=False, nan=0.0)
    return ps


def low_beta(seed, beta=1e-3, p0=1.0, gamma=5.0 / 3.0):
    """Smooth field with B0 = sqrt(2 p0 / beta) along x and 1% density noise."""
    b0 = math.sqrt(2.0 * p0 / beta)
    return SmoothField(seed, a_rho=0.01, b0=(b0, 0.0, 0.0), p0=p0, gamma=gamma)


class Uniform:
    """Spatially uniform state from primitives (rho, v, p, B)."""

    def __init__(self, rho, v, p, b, gamma=5.0 / 3.0):
        self.rho, self.v, self.p, self.b, self.gamma = rho, tuple(v), p, tuple(b), gamma

    def patch(self, level, root_n, lo, hi):
        shape = tuple(int(hi[a] - lo[a]) + 2 * G + 1 for a in (2, 1, 0))
        rho = np.full(shape, float(self.rho))
        mom = [rho * x for x in self.v]
        faces = [np.full(shape, float(x)) for x in self.b]
        e = _total_energy(rho, mom, faces, np.full(shape, float(self.p)), self.gamma)
        return _clean(PatchState(np.stack([rho, mom[0], mom[1], mom[2], e]), faces))


class PlaneProfile:
    """Plane-parallel state along x from point values at cell centres.

    ``prims(x)`` returns (rho, vx, vy, vz, p, By, Bz) arrays for positions x in
    [0, 1); Bx is the constant ``bx``.  y- and z-faces take the value of their
    cell column, so the data are exactly invariant along y and z.
    """

    def __init__(self, prims, bx, gamma):
        self.prims, self.bx, self.gamma = prims, float(bx), gamma

    def patch(self, level, root_n, lo, hi):
        h, c, _ = _coords(level, root_n, lo, hi)
        x = c[0] % 1.0
        rho, vx, vy, vz, p, by, bz = (np.asarray(a, dtype=np.float64) for a in self.prims(x))
        shape = (len(c[2]), len(c[1]), len(c[0]))

        def bc3(a):
            return np.broadcast_to(a, shape).copy()

        rho, vx, vy, vz, p, by, bz = (bc3(a) for a in (rho, vx, vy, vz, p, by, bz))
        mom = [rho * vx, rho * vy, rho * vz]
        bxa = np.full(shape, self.bx)
        faces = [bxa, by.copy(), bz.copy()]
        e = _total_energy(rho, mom, [bxa, by, bz], p, self.gamma)
        return _clean(PatchState(np.stack([rho, mom[0], mom[1], mom[2], e]), faces))


class LinearWave:
    """U = U0 + eps * vec * cos(2 pi (k.x) + phase) in exact cell averages; B via a vector potential.

    u0, vec: eight conserved components (rho, m, E, B); the field part of
    ``vec`` must be orthogonal to k so that a vector potential exists.
    """

    def __init__(self, u0, vec, eps, k, phase=0.0):
        self.u0 = np.asarray(u0, dtype=np.float64)
        self.vec = np.asarray(vec, dtype=np.float64)
        self.eps = float(eps)
        self.k = np.asarray(k, dtype=np.int64)
        self.phase = float(phase)
        kk = self.k.astype(np.float64)
        db = self.vec[5:8] * self.eps
        a0 = np.cross(db, kk) / (2.0 * np.pi * float(kk @ kk))
        rot = np.exp(1j * self.phase)
        self.cell_series = [Series(self.k[None, :], np.array([self.eps * self.vec[c] * rot])) for c in range(5)]
        # sin(theta + phase) = Re(-i e^{i theta} e^{i phase})
        self.a_series = [Series(self.k[None, :], np.array([-1j * a0[c] * rot])) for c in range(3)]

    def patch(self, level, root_n, lo, hi):
        h, c, l = _coords(level, root_n, lo, hi)
        xs, ys, zs = c
        xl, yl, zl = l
        cells = np.stack([self.u0[q] + eval_series(self.cell_series[q], xs, ys, zs, h) for q in range(5)])
        ax = eval_series(self.a_series[0], xs, yl, zl, h, avg=(True, False, False))
        ay = eval_series(self.a_series[1], xl, ys, zl, h, avg=(False, True, False))
        az = eval_series(self.a_series[2], xl, yl, zs, h, avg=(False, False, True))
        shape = cells.shape[1:]
        bx = np.full(shape, np.nan)
        bx[:-1, :-1, :] = (az[:-1, 1:, :] - az[:-1, :-1, :]) / h[1] - (ay[1:, :-1, :] - ay[:-1, :-1, :]) / h[2]
        by = np.full(shape, np.nan)
        by[:-1, :, :-1] = (ax[1:, :, :-1] - ax[:-1, :, :-1]) / h[2] - (az[:-1, :, 1:] - az[:-1, :, :-1]) / h[0]
        bz = np.full(shape, np.nan)
        bz[:, :-1, :-1] = (ay[:, :-1, 1:] - ay[:, :-1, :-1]) / h[0] - (ax[:, 1:, :-1] - ax[:, :-1, :-1]) / h[1]
        faces = [bx + self.u0[5], by + self.u0[6], bz + self.u0[7]]
        return _clean(PatchState(cells, faces))


class Isothermal:
    """The density and momentum of another field's state for the isothermal hydro workload: the
    energy slot and the face fields are zero (no solver arithmetic, only a copy of the arrays)."""

    def __init__(self, base):
        self.base = base

    def patch(self, level, root_n, lo, hi):
        st = self.base.patch(level, root_n, lo, hi)
        cells = st.cells.copy()
        cells[4] = 0.0
        return PatchState(cells, [np.zeros_like(f) for f in st.faces])
