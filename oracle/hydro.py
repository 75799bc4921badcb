"""One substep of the unsplit MUSCL-Hancock advance of isothermal hydrodynamics.

TEST INFRASTRUCTURE ONLY (see the package docstring): float64 NumPy.

The paper counts the isothermal hydrodynamic state (density and the three
momentum components) in its memory estimate of a grid (Sec. 3) and names no
solver for it.  This module is the second workload of the library, a reading
built on the same framework as the MHD scheme of ``mhd.py``:

  * isothermal gas: p = c_s^2 rho with a given sound speed c_s; no energy
    equation and no magnetic field (the patch arrays keep the layout of the
    MHD state: the energy slot and the face fields stay zero);
  * primitive variables (rho, v, p) with MC-limited slopes per axis, the
    conservative Hancock half step from all three axes and face states
    U(w +- s/2) + dU, exactly as in ``mhd.advance``;
  * HLLC-type Riemann solver for the isothermal system (the isothermal HLLD
    of Mignone 2007 with zero field): wave speeds S_L = min(u) - c_s and
    S_R = max(u) + c_s; mass and normal-momentum fluxes are the HLL fluxes;
    the contact speed is S_M = F_rho / rho_hll, and the transverse momentum
    fluxes are F_rho times the transverse velocity of the side S_M comes
    from (left for S_M >= 0).  An isolated stationary or moving shear wave
    is thus resolved exactly;
  * conservative cell update; no constrained transport is needed (B = 0).
"""
from __future__ import annotations

import numpy as np

from . import mhd
from .mhd import N_G, PhysicsError, StepResult, _face_sel, _sel, grow, mc_slope, sh


def prim_from_cons(u, cs2):
    """w = (rho, v, p, B = 0) from conserved (rho, m, E unused)."""
    rho = u[0]
    v = u[1:4] / rho
    z = np.zeros_like(rho)
    return np.concatenate([rho[None], v, (cs2 * rho)[None], z[None], z[None], z[None]])


def cons_from_prim(w):
    """Eight conserved components (rho, m, E = 0, B = 0) from primitives."""
    rho = w[0]
    z = np.zeros_like(rho)
    return np.stack([rho, rho * w[1], rho * w[2], rho * w[3], z, z, z, z])


def flux(w, d, cs2):
    """Isothermal flux along axis d (energy and field components zero)."""
    rho = w[0]
    un = w[1 + d]
    f = np.zeros((8,) + rho.shape)
    f[0] = rho * un
    for c in range(3):
        f[1 + c] = rho * w[1 + c] * un
    f[1 + d] += cs2 * rho
    return f


def hllc(wl, wr, d, cs):
    """Isothermal HLLC flux across a face normal to axis d (ties go to the left side)."""
    cs2 = cs * cs
    rl, ul = wl[0], wl[1 + d]
    rr, ur = wr[0], wr[1 + d]
    sl = np.minimum(ul, ur) - cs
    sr = np.maximum(ul, ur) + cs
    fl = flux(wl, d, cs2)
    fr = flux(wr, d, cs2)
    with np.errstate(all='ignore'):
        inv = 1.0 / (sr - sl)
        f_rho = (sr * fl[0] - sl * fr[0] + sl * sr * (rr - rl)) * inv
        f_mn = (sr * fl[1 + d] - sl * fr[1 + d] + sl * sr * (rr * ur - rl * ul)) * inv
        rho_hll = (sr * rr - sl * rl - (fr[0] - fl[0])) * inv
        sm = f_rho / rho_hll
    star = np.zeros_like(fl)
    star[0] = f_rho
    star[1 + d] = f_mn
    for c in range(3):
        if c != d:
            star[1 + c] = f_rho * np.where(sm >= 0.0, wl[1 + c], wr[1 + c])
    return np.where(sl >= 0.0, fl, np.where(sr <= 0.0, fr, star))


def advance(cells, faces, dx, dt, region, cs):
    """Advance a padded patch by dt over ``region`` (cell box in padded indices); the faces (zero
    field) are returned unchanged.  Same conventions and validity rules as ``mhd.advance``."""
    dx = np.asarray(dx, dtype=np.float64)
    cs2 = cs * cs
    u = cells
    with np.errstate(all='ignore'):
        w = prim_from_cons(u, cs2)
        s_w = w[(slice(None),) + _sel(grow(region, 2))]
        if not (np.all(np.isfinite(s_w[:4])) and np.all(s_w[0] > 0)):
            raise PhysicsError("cell state: rho<=0 or non-finite")
        slope = [mc_slope(w - sh(w, d, -1), sh(w, d, 1) - w) for d in range(3)]
        du = np.zeros((8,) + u.shape[1:])
        for d in range(3):
            du -= (0.5 * dt / dx[d]) * (flux(w + 0.5 * slope[d], d, cs2) - flux(w - 0.5 * slope[d], d, cs2))
        fl = []
        for d in range(3):
            up = cons_from_prim(w + 0.5 * slope[d]) + du
            um = cons_from_prim(w - 0.5 * slope[d]) + du
            wp = prim_from_cons(up[:5], cs2)
            wm = prim_from_cons(um[:5], cs2)
            wl = sh(wp, d, -1)
            wr = wm
            flo = [x - 1 for x in region[0]]
            fhi = [x + 1 for x in region[1]]
            flo[d] += 1
            fsel = _sel((tuple(flo), tuple(fhi)))
            for chk in (wl, wr):
                cc = chk[(slice(None),) + fsel]
                if not (np.all(np.isfinite(cc[:4])) and np.all(cc[0] > 0)):
                    raise PhysicsError("face state: rho<=0 or non-finite")
            fl.append(hllc(wl, wr, d, cs))
        new_u = u.copy()
        div = np.zeros_like(u)
        for d in range(3):
            div += (sh(fl[d][:5], d, 1) - fl[d][:5]) / dx[d]
        sel = _sel(region)
        new_u[(slice(None),) + sel] = u[(slice(None),) + sel] - dt * div[(slice(None),) + sel]
    if not np.all(np.isfinite(new_u[(slice(None),) + sel])):
        raise PhysicsError("updated state non-finite")
    edges = [np.zeros(u.shape[1:]) for _ in range(3)]
    return StepResult(new_u, [f.copy() for f in faces], fl, edges)


def max_signal(cells, dx, box, cs):
    """max over the cells of ``box`` of sum_d (|v_d| + c_s) / dx_d."""
    sel = _sel(box)
    with np.errstate(all='ignore'):
        v = cells[1:4][(slice(None),) + sel] / cells[0][sel]
    tot = sum((np.abs(v[d]) + cs) / dx[d] for d in range(3))
    return float(np.max(tot))
