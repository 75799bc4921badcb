"""Pins of the oracle's isothermal hydro scheme (the second workload) against what the mathematics
fixes: Riemann-solver consistency, symmetry and upwinding, exact resolution of isolated shear waves
(stationary and moving), the exact isothermal Riemann problem, second-order acoustic waves,
conservation across levels and the positivity rule of its prolongation."""
import math

import numpy as np
import pytest

from oracle import amr, hydro
from workloads import hierarchies as H
from workloads.fields import G, Isothermal, LinearWave, PlaneRiemann, SmoothField, Uniform

CS = 0.7


def _states(rng, n):
    rho = rng.uniform(0.3, 3.0, n)
    v = rng.uniform(-2.0, 2.0, (3, n))
    z = np.zeros(n)
    return np.concatenate([rho[None], v, (CS * CS * rho)[None], z[None], z[None], z[None]])


def test_hllc_consistency():
    rng = np.random.default_rng(3)
    w = _states(rng, 2000)
    for d in range(3):
        f = hydro.hllc(w, w, d, CS)
        ref = hydro.flux(w, d, CS * CS)
        assert np.max(np.abs(f - ref) / (1.0 + np.abs(ref))) < 1e-14


def test_hllc_mirror_symmetry():
    rng = np.random.default_rng(4)
    wl, wr = _states(rng, 2000), _states(rng, 2000)
    for d in range(3):
        f = hydro.hllc(wl, wr, d, CS)
        ml, mr = wr.copy(), wl.copy()
        ml[1 + d] *= -1
        mr[1 + d] *= -1
        g = hydro.hllc(ml, mr, d, CS)
        sign = -np.ones(8)
        sign[1 + d] = 1.0
        # ties of S_M at exactly zero have measure zero in random states
        assert np.max(np.abs(g - sign[:, None] * f)) < 1e-12


def test_hllc_supersonic_upwind():
    wl = np.array([1.0, 3.0, 0.2, -0.1, CS * CS, 0, 0, 0])[:, None]
    wr = np.array([0.4, 2.5, -0.3, 0.4, 0.4 * CS * CS, 0, 0, 0])[:, None]
    assert np.array_equal(hydro.hllc(wl, wr, 0, CS), hydro.flux(wl, 0, CS * CS))
    ml, mr = wr.copy(), wl.copy()
    ml[1] *= -1
    mr[1] *= -1
    assert np.array_equal(hydro.hllc(ml, mr, 0, CS), hydro.flux(mr, 0, CS * CS))


@pytest.mark.parametrize("u", [0.0, 0.3, -0.45])
def test_hllc_isolated_shear_wave(u):
    """Equal density and normal velocity, jumping transverse velocities: the exact flux is that of the
    side the wave comes from (the wave moves with u; at u = 0 the left side by the tie rule)."""
    wl = np.array([1.2, u, 0.5, -0.2, 1.2 * CS * CS, 0, 0, 0])[:, None]
    wr = np.array([1.2, u, -0.7, 0.9, 1.2 * CS * CS, 0, 0, 0])[:, None]
    f = hydro.hllc(wl, wr, 0, CS)
    up = wl if u >= 0.0 else wr
    assert np.max(np.abs(f - hydro.flux(up, 0, CS * CS))) < 1e-14


def _star(left, right, cs):
    """Star density and velocity of the isothermal Riemann problem (states (rho, u, ...))."""
    rl, ul = left[0], left[1]
    rr, ur = right[0], right[1]

    def f(r, rk):
        return cs * (r - rk) / math.sqrt(r * rk) if r > rk else cs * math.log(r / rk)

    lo, hi = 1e-10, 1e3 * max(rl, rr)
    for _ in range(200):             # bisection on the increasing function f_L + f_R + du
        mid = math.sqrt(lo * hi)
        if f(mid, rl) + f(mid, rr) + (ur - ul) > 0.0:
            hi = mid
        else:
            lo = mid
    rs = math.sqrt(lo * hi)
    return rs, 0.5 * (ul + ur) + 0.5 * (f(rs, rr) - f(rs, rl))


def _exact_riemann(left, right, xi, cs):
    """Exact solution (rho, u, v_t) of the isothermal Riemann problem at x/t = xi (states (rho, u, v_t))."""
    rl, ul, vl = left
    rr, ur, vr = right
    rs, us = _star(left, right, cs)
    out = np.zeros((3,) + np.shape(xi))
    for idx, x in np.ndenumerate(np.asarray(xi, dtype=float)):
        vt = vl if x < us else vr
        if x < us:
            if rs > rl:
                r, u = (rl, ul) if x < ul - cs * math.sqrt(rs / rl) else (rs, us)
            elif x < ul - cs:
                r, u = rl, ul
            elif x > us - cs:
                r, u = rs, us
            else:
                u = x + cs
                r = rl * math.exp((ul - u) / cs)
        else:
            if rs > rr:
                r, u = (rr, ur) if x > ur + cs * math.sqrt(rs / rr) else (rs, us)
            elif x > ur + cs:
                r, u = rr, ur
            elif x < us + cs:
                r, u = rs, us
            else:
                u = x - cs
                r = rr * math.exp((u - ur) / cs)
        out[(slice(None),) + idx] = (r, u, vt)
    return out


def test_exact_riemann_helper_satisfies_the_wave_relations():
    """The test's own exact solver: across its right shock the isothermal Rankine-Hugoniot conditions
    hold, across its left rarefaction the Riemann invariant u + c_s ln(rho) is constant."""
    left, right = (2.0, 0.1, 0.3), (0.5, -0.2, -0.2)
    rs, us = _star(left, right, CS)
    assert rs < left[0] and rs > right[0]          # rarefaction to the left, shock to the right
    s = right[1] + CS * math.sqrt(rs / right[0])
    mass = s * (rs - right[0]) - (rs * us - right[0] * right[1])
    mom = s * (rs * us - right[0] * right[1]) - ((rs * us * us + CS * CS * rs) - (right[0] * right[1] ** 2 + CS * CS * right[0]))
    assert abs(mass) < 1e-12 and abs(mom) < 1e-12
    assert abs((us + CS * math.log(rs)) - (left[1] + CS * math.log(left[0]))) < 1e-12


def _shock_tube(n, t_end, left, right):
    """Doubled periodic domain [L | R | L] along x on an n x 4 x 4 patch, run to t_end (CFL steps)."""
    spec = H.HierarchySpec(root_n=(n, 4, 4), patches=[(0, (0, 0, 0), (n, 4, 4))])
    lp = (left[0], left[1], left[2], 0.0, left[0] * CS * CS, 0.0, 0.0, 0.0)
    rp = (right[0], right[1], right[2], 0.0, right[0] * CS * CS, 0.0, 0.0, 0.0)
    h = amr.build(spec, Isothermal(PlaneRiemann(lp, rp, 5.0 / 3.0)), physics="isothermal", cs=CS)
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(h.cfl_dt(), t_end - t)
        h.root_step(dt)
        t += dt
    p = h.patches[0]
    return p.cells[:, G + 1, G + 2, G:G + n]


def test_shock_tube_converges_to_the_exact_isothermal_solution():
    """Density of a shock-plus-rarefaction tube against the exact solution: L1 error shrinks at about
    first order (discontinuous solution) and is small at 256 cells."""
    left, right = (2.5, 0.0, 0.4), (0.5, 0.0, -0.3)
    t_end = 0.08
    errs = []
    for n in (64, 128, 256):
        line = _shock_tube(n, t_end, left, right)
        x = (np.arange(n) + 0.5) / n
        ex1 = _exact_riemann(left, right, (x - 0.25) / t_end, CS)
        ex2 = _exact_riemann(right, left, (x - 0.75) / t_end, CS)
        rho = np.where(x < 0.5, ex1[0], ex2[0])
        errs.append(np.mean(np.abs(line[0] - rho)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 0.6, (errs, orders)
    assert errs[-1] < 0.02 * (left[0] - right[0]), errs


def _acoustic_errors(k, ns, t_end=0.1):
    kk = np.asarray(k, dtype=np.float64)
    nh = kk / np.linalg.norm(kk)
    rho0, v0 = 1.0, np.array([0.2, -0.1, 0.05])
    u0 = np.array([rho0, *(rho0 * v0), 0.0, 0.0, 0.0, 0.0])
    ev = np.array([1.0, *(v0 + CS * nh), 0.0, 0.0, 0.0, 0.0])   # right-going isothermal acoustic mode
    lam = float(v0 @ nh) + CS
    eps = 1e-6
    errs = []
    for n in ns:
        root = (n, n, 4)
        spec = H.HierarchySpec(root_n=root, patches=[(0, (0, 0, 0), root)])
        h = amr.build(spec, LinearWave(u0, ev, eps, k), physics="isothermal", cs=CS)
        nst = int(math.ceil(t_end / h.cfl_dt()))
        for _ in range(nst):
            h.root_step(t_end / nst)
        ref = LinearWave(u0, ev, eps, k, -2 * np.pi * np.linalg.norm(kk) * lam * t_end).patch(0, root, (0, 0, 0), root)
        sl = (slice(G, G + 4), slice(G, G + n), slice(G, G + n))
        p = h.patches[0]
        errs.append(sum(np.mean(np.abs(p.cells[q][sl] - ref.cells[q][sl])) for q in range(4)) / eps)
    return errs


def test_acoustic_wave_second_order():
    errs = _acoustic_errors((1, 1, 0), [16, 32, 64])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] > 1.9, (errs, orders)


def test_three_level_conservation_and_sync():
    o = amr.build(H.small_three_level(), Isothermal(SmoothField(33)), physics="isothermal", cs=CS)
    c0 = o.conservation()
    scale = sum(abs(x) for x in c0[:4])
    for _ in range(2):
        o.root_step()
    c1 = o.conservation()
    assert np.all(np.abs(c1[:4] - c0[:4]) <= 1e-14 * scale)
    assert c1[4] == 0.0 and np.all(c1[5:] == 0.0)
    assert o.diag["sync_flux_max"] == 0.0


def test_isothermal_prolongation_fallback_acts_on_density_only():
    """A density slope that would make a child's density negative hands all 8 children the coarse
    values; a steep momentum (unphysical for the MHD energy rule) is fine for isothermal gas."""
    o = amr.build(H.small_two_level(), Uniform(1.0, (0, 0, 0), 1.0, (0, 0, 0)), physics="isothermal", cs=CS)
    m = o.patches[0]
    m.cells[4] = 0.0
    for d in range(3):
        m.faces[d][...] = 0.0
    for i, (r, mx) in enumerate(((1.0, 0.0), (0.05, 3.0), (1.0, 6.0))):
        m.cells[0, G + 4, G + 4, G + i] = r
        m.cells[1, G + 5, G + 4, G + i] = mx
    m.old_cells, m.old_faces = m.cells.copy(), [f.copy() for f in m.faces]
    p = o.patches[1]
    o._prolong(p)
    po = p.origin()

    def children(cx, cy, cz):
        f = 2 * np.array([cx, cy, cz]) - po
        return p.cells[:, f[2]:f[2] + 2, f[1]:f[1] + 2, f[0]:f[0] + 2]

    dens = children(1, 4, 4)
    assert np.all(dens[0] == 0.05)
    mom = children(1, 4, 5)
    assert np.ptp(mom[1]) > 1.0
