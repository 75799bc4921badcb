"""Pins of the oracle's single-patch scheme against what the mathematics fixes.

Each test targets a property a plausible mistake would break: Riemann-solver
consistency and symmetry, exact resolution of isolated discontinuities, the
limiter's definition, the stencil depth that sets the extended-ghost width,
discrete conservation and divergence preservation, the dimensional reduction
that singles out the upwinded CT-contact EMF, and second-order convergence on
linear waves (grid-aligned and oblique).
"""
import math

import numpy as np
import pytest

from oracle import amr, mhd, mhd1d
from workloads import hierarchies as H
from workloads.fields import G, LinearWave, PlaneProfile, SmoothField

GAM = 5.0 / 3.0


def _states(rng, n):
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.uniform(-1.0, 1.0, (3, n))
    p = rng.uniform(0.2, 2.0, n)
    b = rng.uniform(-1.5, 1.5, (3, n))
    return np.concatenate([rho[None], v, p[None], b])


def test_hlld_consistency():
    """F_HLLD(U, U) equals the physical flux F(U) for every axis."""
    rng = np.random.default_rng(0)
    w = _states(rng, 2000)
    for d in range(3):
        f = mhd.hlld(w, w, w[5 + d], d, GAM)
        ref = mhd.flux(w, d, GAM)
        assert np.max(np.abs(f - ref) / (1.0 + np.abs(ref))) < 1e-13


def test_hlld_mirror_symmetry():
    """Reflection x -> -x (swap sides, negate u_n and B_n) maps the flux by the parity signs."""
    rng = np.random.default_rng(1)
    wl = _states(rng, 2000)
    wr = _states(rng, 2000)
    bn = rng.uniform(-1.5, 1.5, 2000)
    for d in range(3):
        f = mhd.hlld(wl, wr, bn, d, GAM)
        ml, mr = wr.copy(), wl.copy()
        ml[1 + d] *= -1
        mr[1 + d] *= -1
        g = mhd.hlld(ml, mr, -bn, d, GAM)
        sign = -np.ones(8)
        sign[1 + d] = 1.0
        assert np.max(np.abs(g - sign[:, None] * f)) < 1e-12


def test_hlld_supersonic_upwind():
    """All waves moving right: the flux is exactly the left physical flux."""
    w = np.array([1.0, 10.0, 0.1, 0.2, 1.0, 0.5, 0.3, 0.1])[:, None]
    wr = np.array([0.5, 9.0, 0.0, 0.1, 0.7, 0.5, 0.2, 0.0])[:, None]
    f = mhd.hlld(w, wr, np.array([0.5]), 0, GAM)
    assert np.array_equal(f, mhd.flux(w, 0, GAM))


@pytest.mark.parametrize("bn", [0.0, 0.8])
def test_hlld_isolated_contact(bn):
    """A stationary contact (Bn != 0) or tangential discontinuity (Bn = 0) is resolved exactly."""
    wl = np.array([1.0, 0.0, 0.3, -0.2, 1.0, bn, 0.5, 0.4])[:, None]
    wr = wl.copy()
    wr[0] = 0.3
    if bn == 0.0:
        # tangential discontinuity: v_t and B_t may jump, total pressure continuous
        wr[2], wr[3], wr[6], wr[7] = -0.4, 0.6, 0.2, -0.3
        pt = wl[4] + 0.5 * (wl[6] ** 2 + wl[7] ** 2)
        wr[4] = pt - 0.5 * (wr[6] ** 2 + wr[7] ** 2)
    f = mhd.hlld(wl, wr, np.array([bn]), 0, GAM)
    ref = mhd.flux(wl, 0, GAM)
    assert abs(f[0, 0]) < 1e-15
    assert np.max(np.abs(f - ref)) < 1e-14


def test_hlld_rotational_discontinuity():
    """A stationary rotational discontinuity (u_n = Bn / sqrt(rho)) is resolved exactly."""
    rho, p, bn, bt = 1.3, 0.8, 0.9, 0.7
    un = bn / math.sqrt(rho)
    v0 = np.array([0.1, -0.2])
    out = []
    for th in (0.3, 2.1):
        btv = bt * np.array([math.cos(th), math.sin(th)])
        vt = v0 + btv / math.sqrt(rho)
        out.append(np.array([rho, un, vt[0], vt[1], p, bn, btv[0], btv[1]])[:, None])
    wl, wr = out
    f = mhd.hlld(wl, wr, np.array([bn]), 0, GAM)
    fl = mhd.flux(wl, 0, GAM)
    fr = mhd.flux(wr, 0, GAM)
    assert np.max(np.abs(fl - fr)) < 1e-14           # it is a stationary discontinuity
    assert np.max(np.abs(f - fl)) < 1e-13


def test_mc_limiter_cases():
    dm = np.array([1.0, 1.0, 1.0, 0.0, -1.0, 2.0, -3.0, 1.0])
    dp = np.array([1.0, 3.0, -1.0, 1.0, -0.2, 0.5, -3.0, 0.0])
    want = np.array([1.0, 2.0, 0.0, 0.0, -0.4, 1.0, -3.0, 0.0])
    assert np.array_equal(mhd.mc_slope(dm, dp), want)


def _random_patch(n, seed):
    fld = SmoothField(seed)
    st = fld.patch(0, (n, n, n), (0, 0, 0), (n, n, n))
    return st.cells, st.faces


def test_stencil_depth_is_two():
    """Perturbing one cell changes the update only within a box of radius 2 (n_g = 2), and at radius 2."""
    n = 12
    cells, faces = _random_patch(n, 5)
    dx = [1.0 / n] * 3
    region = ((2, 2, 2), (n + 2 * G - 2,) * 3)
    base = mhd.advance(cells, faces, dx, 1e-3, region, GAM)
    c = n // 2 + G
    pert = cells.copy()
    pert[0, c, c, c] *= 1.01
    res = mhd.advance(pert, faces, dx, 1e-3, region, GAM)
    changed = np.argwhere(np.any(res.cells != base.cells, axis=0))
    r = np.max(np.abs(changed - c), axis=1)
    assert r.max() == 2
    # and a face value perturbation: radius 2 around its two cells for the faces too
    fp = [f.copy() for f in faces]
    fp[0][c, c, c] += 1e-3
    res2 = mhd.advance(cells, fp, dx, 1e-3, region, GAM)
    ch = np.argwhere(np.any(res2.cells != base.cells, axis=0))
    lo = np.array([c, c, c - 1])
    hi = np.array([c, c, c])
    dist = np.maximum(lo - ch, 0) + np.maximum(ch - hi, 0)
    assert dist.max() == 2


def _periodic_single(n, fld, steps, dt=None):
    h = amr.build(H.single_patch(n), fld)
    for _ in range(steps):
        h.root_step(dt)
    return h


def test_periodic_conservation_and_divergence():
    n = 16
    fld = SmoothField(1112)
    h = amr.build(H.single_patch(n), fld)
    c0 = h.conservation()
    scale = [math.fsum(np.abs(h.patches[0].cells[q]).ravel()) / n ** 3 for q in range(5)]
    for _ in range(3):
        h.root_step()
    c1 = h.conservation()
    for q in range(5):
        assert abs(c1[q] - c0[q]) <= 1e-14 * max(scale[q], 1e-300) * 10
    assert h.max_divergence() < 1e-12


def _plane_profile():
    def prims(x):
        s, c = np.sin(2 * np.pi * x), np.cos(2 * np.pi * x)
        return (1 + 0.2 * s, 0.1 * c, 0.05 * np.sin(4 * np.pi * x), 0.02 * c, 1 + 0.1 * c, 0.4 * s + 0.3, 0.2 * c)
    return PlaneProfile(prims, 0.7, GAM)


def _line_of(p, n):
    return np.concatenate([p.cells[:, G + 1, G + 2, G:G + n],
                           np.stack([p.faces[0][G + 1, G + 2, G:G + n], p.faces[1][G + 1, G + 2, G:G + n],
                                     p.faces[2][G + 1, G + 2, G:G + n]])])


def test_dimensional_reduction_to_1d(monkeypatch):
    """A plane-parallel 3-D CT run equals the 1-D Godunov scheme; a plain mean of face EMFs does not."""
    n, dt, steps = 32, 0.002, 5

    def run3d():
        h = amr.build(H.HierarchySpec(root_n=(n, 4, 4), patches=[(0, (0, 0, 0), (n, 4, 4))]), _plane_profile())
        p = h.patches[0]
        line = _line_of(p, n)
        for _ in range(steps):
            h.root_step(dt)
        return h.patches[0], line

    p, line = run3d()
    for _ in range(steps):
        line = mhd1d.advance_1d(line, 1.0 / n, dt, GAM)
    interior = p.cells[:, G:G + 4, G:G + 4, G:G + n]
    assert np.array_equal(interior, np.broadcast_to(interior[:, :1, :1, :], interior.shape))
    got = _line_of(p, n)
    err = np.max(np.abs(got - line))
    assert err < 1e-13

    # the arithmetic-mean EMF (no upwinded corner terms) breaks the reduction
    def mean_only(ef_a, ef_b, eref, fa, fb, a, b):
        return 0.25 * (mhd.sh(ef_a, b, -1) + ef_a + mhd.sh(ef_b, a, -1) + ef_b)

    monkeypatch.setattr(mhd, "edge_emf", mean_only)
    p2, _ = run3d()
    assert np.max(np.abs(_line_of(p2, n) - line)) > 1e-6


def _jacobian(u, nhat):
    """Numerical Jacobian of the projected flux sum_d n_d F_d with respect to the 8 conserved components."""
    def f(uv):
        w = mhd.prim_from_cons(uv[:5, None], uv[5:, None], GAM)
        return sum(nhat[d] * mhd.flux(w, d, GAM)[:, 0] for d in range(3))
    jac = np.zeros((8, 8))
    for j in range(8):
        h = 1e-6 * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        jac[:, j] = (f(up) - f(um)) / (2 * h)
    return jac


def _wave_errors(k, mode, ns, shape_z=None, t_end=0.08):
    """L1 errors (summed over the 8 fields, relative to the amplitude) of a linear wave at several resolutions."""
    kk = np.asarray(k, dtype=np.float64)
    nhat = kk / np.linalg.norm(kk)
    rho0, p0 = 1.0, 1.0 / GAM
    b0 = np.array([1.0, math.sqrt(2.0), 0.5])
    v0 = np.zeros(3)
    w0 = np.concatenate([[rho0], v0, [p0], b0])[:, None]
    u0 = mhd.cons_from_prim(w0, GAM)[:, 0]
    jac = _jacobian(u0, nhat)
    lam, vec = np.linalg.eig(jac)
    lam, vec = lam.real, vec.real
    order = np.argsort(lam)
    idx = order[-1] if mode == "fast" else order[-2]   # fastest, or the Alfven wave next to it
    lam_w = lam[idx]
    ev = vec[:, idx] / np.max(np.abs(vec[:, idx]))
    ev[5:8] -= nhat * (ev[5:8] @ nhat)                  # field perturbation orthogonal to k
    eps = 1e-6
    errs = []
    for n in ns:
        root = (n, n, shape_z if shape_z else n)
        spec = H.HierarchySpec(root_n=root, patches=[(0, (0, 0, 0), root)])
        h = amr.build(spec, LinearWave(u0, ev, eps, k))
        dt_cfl = h.cfl_dt()
        nst = int(math.ceil(t_end / dt_cfl))
        dt = t_end / nst
        for _ in range(nst):
            h.root_step(dt)
        phase = -2 * np.pi * np.linalg.norm(kk) * lam_w * t_end
        ref = LinearWave(u0, ev, eps, k, phase).patch(0, root, (0, 0, 0), root)
        p = h.patches[0]
        sl = (slice(G, G + root[2]), slice(G, G + root[1]), slice(G, G + root[0]))
        e = sum(np.mean(np.abs(p.cells[q][sl] - ref.cells[q][sl])) for q in range(5))
        e += sum(np.mean(np.abs(p.faces[d][sl] - ref.faces[d][sl])) for d in range(3))
        errs.append(e / eps)
    return errs


@pytest.mark.parametrize("k,mode,zn", [((1, 1, 0), "fast", 4), ((1, 1, 0), "alfven", 4), ((1, 0, 0), "alfven", 4)])
def test_linear_wave_second_order(k, mode, zn):
    errs = _wave_errors(k, mode, [16, 32, 64], shape_z=zn)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 1.9, (errs, orders)


@pytest.mark.slow
def test_linear_wave_second_order_fully_oblique():
    errs = _wave_errors((1, 1, 1), "fast", [8, 16, 32])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 1.9, (errs, orders)


def _brio_wu_line(n, t_end):
    gam = 2.0
    x = (np.arange(n) + 0.5) / n
    inside = (x >= 0.25) & (x < 0.75)
    rho = np.where(inside, 0.125, 1.0)
    p = np.where(inside, 0.1, 1.0)
    by = np.where(inside, -1.0, 1.0)
    w = np.stack([rho, 0 * x, 0 * x, 0 * x, p, 0.75 + 0 * x, by, 0 * x])
    u = mhd.cons_from_prim(w, gam)
    dx = 1.0 / n
    nst = int(math.ceil(t_end / (0.2 * dx)))
    dt = t_end / nst
    for _ in range(nst):
        u = mhd1d.advance_1d(u, dx, dt, gam)
    return u


def test_brio_wu_self_convergence():
    """L1 self-convergence of the shock tube (doubled periodic domain) is about first order."""
    t_end = 0.05
    ref_n = 4096
    ref = _brio_wu_line(ref_n, t_end)
    errs = []
    for n in (64, 128, 256):
        u = _brio_wu_line(n, t_end)
        r = ref.reshape(8, n, ref_n // n).mean(axis=2)
        errs.append(np.mean(np.abs(u[0] - r[0])))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 0.6, (errs, orders)


def _degenerate_family(eps, shear):
    """States at HLLD's degenerate limit as eps -> 0: normal field dominant over sound
    (Bn^2 / rho > gamma p / rho), transverse field eps on both sides, equal rho, u_n and
    total pressure (so the contact speed equals u_n and both star-state denominators
    rho (S - u)(S - S_M) - Bn^2 shrink like eps^2).  ``shear`` jumps the transverse velocity."""
    wl = np.array([1.0, 0.2, 0.1, -0.05, 0.1, 1.0, eps, 0.5 * eps])[:, None]
    wr = wl.copy()
    if shear:
        wr[2], wr[3] = -0.3, 0.25
    return wl, wr


@pytest.mark.parametrize("shear", [False, True])
def test_hlld_degenerate_branch_is_the_limit_of_the_general_formulas(monkeypatch, shear):
    """Miyoshi & Kusano's star-state formulas for v*_t and B*_t become 0/0 when the
    Alfven and fast waves coincide (B_t -> 0 with Bn^2 >= gamma p).  With S_M = u their
    limits are v*_t = v_t and B*_t = B_t, so the degenerate branch must agree with the
    general formulas on both sides of its threshold and for both signs of B_t (no jump),
    and consistency F(U, U) = F(U) must hold there."""
    eps = np.concatenate([np.geomspace(3e-3, 1e-6, 40), -np.geomspace(3e-3, 1e-6, 40)])
    f_branch, f_general = [], []
    for e in eps:
        wl, wr = _degenerate_family(e, shear)
        f_branch.append(mhd.hlld(wl, wr, wl[5], 0, GAM)[:, 0])
        if not shear:
            ref = mhd.flux(wl, 0, GAM)[:, 0]
            assert np.max(np.abs(f_branch[-1] - ref) / (1.0 + np.abs(ref))) < 1e-13
    monkeypatch.setattr(mhd, "DEGEN_REL", 0.0)     # general formulas everywhere (den != 0 here)
    for e in eps:
        wl, wr = _degenerate_family(e, shear)
        f_general.append(mhd.hlld(wl, wr, wl[5], 0, GAM)[:, 0])
    f_branch, f_general = np.array(f_branch), np.array(f_general)
    # the smallest |eps| lie well inside the threshold: |den| / (rho (S - u)^2) ~ 1.2 eps^2 < 1e-8
    assert np.max(np.abs(f_branch - f_general)) < 1e-11
    # and the flux is a smooth function of eps across the threshold (|eps| ~ 1e-4)
    for sgn in (slice(0, 40), slice(40, 80)):
        fb = f_branch[sgn]
        steps = np.max(np.abs(np.diff(fb, axis=0)), axis=1)
        de = np.abs(np.diff(eps[sgn]))
        assert np.all(steps <= 10.0 * de + 1e-13), np.max(steps / de)


def test_hlld_degenerate_branch_taken():
    """Below the threshold the star states must come from the degenerate branch: a branch that
    returned different transverse values would change the flux by O(1)."""
    wl, wr = _degenerate_family(1e-6, True)
    f = mhd.hlld(wl, wr, wl[5], 0, GAM)
    # the flux sits between the two physical fluxes' transverse momenta in magnitude (finite, bounded)
    assert np.all(np.isfinite(f))
    fl, fr = mhd.flux(wl, 0, GAM), mhd.flux(wr, 0, GAM)
    assert np.all(np.abs(f) <= np.maximum(np.abs(fl), np.abs(fr)) + 2.0)


def test_fast_speed_is_the_flux_jacobian_spectral_radius():
    """For random states and directions n the largest and smallest eigenvalues of the projected
    flux Jacobian sum_d n_d dF_d/dU are v.n +- c_f(n), with c_f taken with Bn = B.n."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        rho = rng.uniform(0.3, 3.0)
        v = rng.uniform(-1.0, 1.0, 3)
        p = rng.uniform(0.05, 3.0)
        b = rng.uniform(-2.0, 2.0, 3)
        nh = rng.normal(size=3)
        nh /= np.linalg.norm(nh)
        w = np.concatenate([[rho], v, [p], b])[:, None]
        u = mhd.cons_from_prim(w, GAM)[:, 0]
        lam = np.linalg.eigvals(_jacobian(u, nh)).real
        vn = float(v @ nh)
        bn = float(b @ nh)
        cf = float(mhd.fast_speed(rho, p, float(b @ b), bn * bn, GAM))
        scale = abs(vn) + cf
        assert abs(lam.max() - (vn + cf)) < 1e-6 * scale, (lam, vn, cf)
        assert abs(lam.min() - (vn - cf)) < 1e-6 * scale, (lam, vn, cf)


def test_hlld_mass_flux_round_off_is_exactly_zero():
    """States at rest whose pressures or densities differ by a few ulps (a stagnant face just ahead of
    a flow front) have a mass flux that vanishes in exact arithmetic: it must come out exactly 0.0 in
    either orientation, so that the sign-upwinded edge EMF takes the average; a genuine flow of
    1e-9 of the signal speed is kept."""
    w = np.array([1.0, 0.0, 0.0, 0.0, 1.0, 0.7, 0.7, 0.0])[:, None]
    for k in range(1, 6):
        wr = w.copy()
        wr[4] = np.nextafter(1.0, 2.0) + k * 2.0 ** -52
        wr[0] = 1.0 - k * 2.0 ** -53
        for d in range(3):
            f1 = mhd.hlld(w, wr, w[5 + d], d, GAM)
            f2 = mhd.hlld(wr, w, w[5 + d], d, GAM)
            assert f1[0, 0] == 0.0 and f2[0, 0] == 0.0
    cf = float(mhd.fast_speed(1.0, 1.0, 0.98, 0.49, GAM))
    slow = w.copy()
    slow[1] = 1e-9 * cf
    f = mhd.hlld(slow, slow, w[5], 0, GAM)
    assert abs(f[0, 0] - 1e-9 * cf) < 1e-22
