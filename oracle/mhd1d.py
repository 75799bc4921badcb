"""The same MUSCL-Hancock / HLLD scheme in one dimension (x), with cell-centred B.

TEST INFRASTRUCTURE ONLY.  In one dimension the normal field Bx is constant
and the transverse field is an ordinary conserved cell variable, so no
constrained transport is involved.  A three-dimensional run of the CT scheme
on plane-parallel data along x must reduce to this scheme: the upwinded
CT-contact edge EMF collapses onto the 1-D Godunov flux of the transverse
field, while a plain arithmetic mean of the face EMFs would not.
"""
from __future__ import annotations

import numpy as np

from .mhd import cons_from_prim, flux, hlld, mc_slope, prim_from_cons


def _sh(a, s):
    return np.roll(a, -s, axis=-1)


def advance_1d(u8, dx, dt, gamma):
    """One step of a periodic 1-D line.  u8: (8, N) = (rho, m, E, Bx, By, Bz)."""
    w = prim_from_cons(u8[:5], u8[5:], gamma)
    s = mc_slope(w - _sh(w, -1), _sh(w, 1) - w)
    du = -(0.5 * dt / dx) * (flux(w + 0.5 * s, 0, gamma) - flux(w - 0.5 * s, 0, gamma))
    up = cons_from_prim(w + 0.5 * s, gamma) + du
    um = cons_from_prim(w - 0.5 * s, gamma) + du
    wp = prim_from_cons(up[:5], up[5:], gamma)
    wm = prim_from_cons(um[:5], um[5:], gamma)
    bn = u8[5]
    f = hlld(_sh(wp, -1), wm, bn, 0, gamma)     # flux at the left face of each cell
    out = u8.copy()
    out -= (dt / dx) * (_sh(f, 1) - f)
    out[5] = u8[5]
    return out
