// gfx950 kernels of the AMR MHD hot path.
//
// Advance of a ghost-padded patch by one substep (unsplit MUSCL-Hancock
// predictor, HLLD fluxes after Miyoshi & Kusano 2005, upwinded CT-contact
// edge EMFs after Gardiner & Stone 2005), staged through per-patch
// intermediate arrays so that every quantity is computed once per cell,
// face or edge of the region that needs it.  Stage regions follow the
// extended-ghost rule of the paper (Sec. 2.3): for an update region W, the
// primitives cover W grown by 2 cells, the half-step state W grown by 1, the
// face fluxes the faces of W plus one transverse layer, the edge EMFs the
// edges of W's faces.
//
// The first three stages (primitives, half-step face field, Hancock
// predictor) also exist fused in one LDS-tiled kernel with bit-identical
// results; which one runs, and its tile shape, is chosen per level.
//
// Every stage kernel walks a list of (patch, region) tasks: block b finds its
// task by binary search over the tasks' first blocks, so one launch can cover
// one patch (plain schedule) or all patches of a level substep (batched
// schedule).  Threads map to region entries with x fastest, so consecutive
// lanes touch consecutive addresses of the structure-of-arrays buffers.
//
// Precision: Real = double (FP64), float (FP32) or float with the pressure
// recovered in double, the Riemann problem solved in double at low-beta
// faces and flux/EMF registers kept in double with two-sum compensation
// (FP32 mixed).  Registers are double except in plain FP32.

#include <math.h>
#include <stdint.h>

#include <mutex>

#include <type_traits>

#include "amrx_internal.h"
#include "../../include/amrx.h"

namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Division, reciprocal and square root.  FP64 keeps the IEEE operations.
// FP32 uses the hardware reciprocal refined by one Newton step (error within
// about 1 ulp, against several instructions of scaling and fix-up for a
// correctly rounded quotient) and the hardware square root (1 ulp); FP32
// results are held to a relative L1 tolerance of 1e-5, far above that.
#ifndef AMRX_FAST_FP32
#define AMRX_FAST_FP32 1
#endif
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double qsqrt(double x) { return sqrt(x); }
#if AMRX_FAST_FP32
__device__ __forceinline__ float rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ float qdiv(float a, float b) { return a * rcp(b); }
__device__ __forceinline__ float qsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
#else
__device__ __forceinline__ float rcp(float x) { return 1.0f / x; }
__device__ __forceinline__ float qdiv(float a, float b) { return a / b; }
__device__ __forceinline__ float qsqrt(float x) { return sqrtf(x); }
#endif

// FD selects, for double, the hardware reciprocal refined by two Newton steps and a
// corrected quotient (within about 1 ulp) instead of the IEEE division sequence; used by
// the FP32_MIXED mode's double-precision Riemann solver.  The FP64 mode keeps IEEE.
template <bool FD, typename R>
__device__ __forceinline__ R rcp_t(R x) { return rcp(x); }
template <>
__device__ __forceinline__ double rcp_t<true, double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
template <bool FD, typename R>
__device__ __forceinline__ R qdiv_t(R a, R b) { return qdiv(a, b); }
template <>
__device__ __forceinline__ double qdiv_t<true, double>(double a, double b) {
  const double r = rcp_t<true>(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

template <typename R>
__device__ __forceinline__ R mc_limit(R dm, R dp) {
  // monotonised central: minmod(2 dm, 2 dp, (dm + dp)/2), zero unless dm, dp share a strict sign
  if (!(dm * dp > R(0))) return R(0);
  R a = fmin(fmin(R(2) * fabs(dm), R(2) * fabs(dp)), R(0.5) * fabs(dm + dp));
  return dm > R(0) ? a : -a;
}

template <typename R>
__device__ __forceinline__ R minmod2(R a, R b) {
  if (!(a * b > R(0))) return R(0);
  R m = fmin(fabs(a), fabs(b));
  return a > R(0) ? m : -m;
}

template <typename R>
__device__ __forceinline__ R upwind(R flux, R minus_val, R plus_val) {
  const R mean = R(0.5) * (minus_val + plus_val);
  return flux > R(0) ? minus_val : (flux < R(0) ? plus_val : mean);
}

// gas pressure from conserved variables.  MIX evaluates it again in double where the subtraction
// cancels: the float result keeps about log2(e / (e - kin - mag)) fewer bits than e, so where the
// kinetic and magnetic energies exceed 15/16 of e (low beta, fast flow) more than 4 bits would go.
template <typename R, bool MIX>
__device__ __forceinline__ R pressure(R rho, R mx, R my, R mz, R e, R bx, R by, R bz, R gm1) {
  const R kin = qdiv(R(0.5) * (mx * mx + my * my + mz * mz), rho);
  const R mag = R(0.5) * (bx * bx + by * by + bz * bz);
  const R eint = e - kin - mag;
  if (MIX && !(R(16) * eint > e)) {
    const double r = rho;
    const double kd = 0.5 * ((double)mx * mx + (double)my * my + (double)mz * mz) / r;
    const double md = 0.5 * ((double)bx * bx + (double)by * by + (double)bz * bz);
    return (R)((double)gm1 * ((double)e - kd - md));
  }
  return gm1 * eint;
}

template <typename R, bool FD = false>
__device__ __forceinline__ R fast_speed(R rho, R p, R b2, R bn2, R gamma) {
  const R ir = rcp_t<FD>(rho);
  R a2 = gamma * p * ir;
  R s = a2 + b2 * ir;
  R disc = s * s - R(4) * a2 * bn2 * ir;
  disc = disc > R(0) ? disc : R(0);
  return qsqrt(R(0.5) * (s + qsqrt(disc)));
}

// primitive w = (rho, vx, vy, vz, p, Bx, By, Bz) -> physical flux along D (global component order)
template <int D, typename R>
__device__ __forceinline__ void phys_flux(const R* w, R gm1, R* f) {
  const R rho = w[0], p = w[4];
  const R v0 = w[1], v1 = w[2], v2 = w[3];
  const R b0 = w[5], b1 = w[6], b2 = w[7];
  const R un = w[1 + D], bn = w[5 + D];
  const R bb = b0 * b0 + b1 * b1 + b2 * b2;
  const R pt = p + R(0.5) * bb;
  const R e = qdiv(p, gm1) + R(0.5) * rho * (v0 * v0 + v1 * v1 + v2 * v2) + R(0.5) * bb;
  const R vb = v0 * b0 + v1 * b1 + v2 * b2;
  f[0] = rho * un;
  f[1] = rho * v0 * un - b0 * bn;
  f[2] = rho * v1 * un - b1 * bn;
  f[3] = rho * v2 * un - b2 * bn;
  f[1 + D] += pt;
  f[4] = (e + pt) * un - bn * vb;
  f[5] = b0 * un - bn * v0;
  f[6] = b1 * un - bn * v1;
  f[7] = b2 * un - bn * v2;
  f[5 + D] = R(0);
}

// primitive state -> 8 conserved (rho, m, E, B)
template <typename R>
__device__ __forceinline__ void to_cons(const R* w, R gm1, R* u) {
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = qdiv(w[4], gm1) + R(0.5) * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) +
         R(0.5) * (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]);
  u[5] = w[5];
  u[6] = w[6];
  u[7] = w[7];
}

template <typename R, bool MIX>
__device__ __forceinline__ void to_prim(const R* u, R gm1, R* w) {
  w[0] = u[0];
  w[1] = qdiv(u[1], u[0]);
  w[2] = qdiv(u[2], u[0]);
  w[3] = qdiv(u[3], u[0]);
  w[4] = pressure<R, MIX>(u[0], u[1], u[2], u[3], u[4], u[5], u[6], u[7], gm1);
  w[5] = u[5];
  w[6] = u[6];
  w[7] = u[7];
}

// Transverse star-state velocity and field of one side (Miyoshi & Kusano 2005, their
// eqs. 44-47): with dn = rho sd (s - sm) - bn^2 and num = rho sd^2 - bn^2 (sd = s - u),
// v* = v - bn by (sm - u) / dn and by* = by num / dn; a degenerate dn keeps v and B.
// primitives of the isothermal workload: p = cs2 rho, the field components as stored (zero)
template <typename R>
__device__ __forceinline__ void to_prim_iso(const R* u, R cs2, R* w) {
  w[0] = u[0];
  w[1] = qdiv(u[1], u[0]);
  w[2] = qdiv(u[2], u[0]);
  w[3] = qdiv(u[3], u[0]);
  w[4] = cs2 * u[0];
  w[5] = u[5];
  w[6] = u[6];
  w[7] = u[7];
}

template <bool FD, typename R>
__device__ __forceinline__ void star_transverse(R r, R sd, R s, R sm, R u, R v, R z, R by, R bz, R bn, R& vs, R& zs,
                                                R& bys, R& bzs) {
  const R dn = r * sd * (s - sm) - bn * bn;
  if (fabs(dn) <= R(1e-8) * r * sd * sd) {
    vs = v; zs = z; bys = by; bzs = bz;
  } else {
    const R num = r * sd * sd - bn * bn;
    const R dsm = sm - u;
    vs = v - qdiv_t<FD>(bn * by * dsm, dn);
    zs = z - qdiv_t<FD>(bn * bz * dsm, dn);
    bys = qdiv_t<FD>(by * num, dn);
    bzs = qdiv_t<FD>(bz * num, dn);
  }
}

// HLLD flux normal to D.  Normal field bn replaces both states' normal component.
template <int D, typename R, bool FD = false>
__device__ __forceinline__ void hlld(const R* wl, const R* wr, R bn, R gamma, R* out) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const R gm1 = gamma - R(1);
  const R rl = wl[0], ul = wl[1 + D], vl = wl[1 + T1], zl = wl[1 + T2], pl = wl[4], byl = wl[5 + T1], bzl = wl[5 + T2];
  const R rr = wr[0], ur = wr[1 + D], vr = wr[1 + T1], zr = wr[1 + T2], pr = wr[4], byr = wr[5 + T1], bzr = wr[5 + T2];
  const R bn2 = bn * bn;
  const R b2l = bn2 + byl * byl + bzl * bzl;
  const R b2r = bn2 + byr * byr + bzr * bzr;
  const R cfl = fast_speed<R, FD>(rl, pl, b2l, bn2, gamma);
  const R cfr = fast_speed<R, FD>(rr, pr, b2r, bn2, gamma);
  const R cmax = fmax(cfl, cfr);
  const R sl = fmin(ul, ur) - cmax;
  const R sr = fmax(ul, ur) + cmax;
  const R ptl = pl + R(0.5) * b2l;
  const R ptr = pr + R(0.5) * b2r;
  const R el = qdiv_t<FD>(pl, gm1) + R(0.5) * rl * (ul * ul + vl * vl + zl * zl) + R(0.5) * b2l;
  const R er = qdiv_t<FD>(pr, gm1) + R(0.5) * rr * (ur * ur + vr * vr + zr * zr) + R(0.5) * b2r;
  const R vbl = ul * bn + vl * byl + zl * bzl;
  const R vbr = ur * bn + vr * byr + zr * bzr;

  R f[7];
  if (sl >= R(0)) {
    f[0] = rl * ul;
    f[1] = rl * ul * ul + ptl - bn2;
    f[2] = rl * ul * vl - bn * byl;
    f[3] = rl * ul * zl - bn * bzl;
    f[4] = (el + ptl) * ul - bn * vbl;
    f[5] = byl * ul - bn * vl;
    f[6] = bzl * ul - bn * zl;
  } else if (sr <= R(0) && !(sr >= R(0))) {
    f[0] = rr * ur;
    f[1] = rr * ur * ur + ptr - bn2;
    f[2] = rr * ur * vr - bn * byr;
    f[3] = rr * ur * zr - bn * bzr;
    f[4] = (er + ptr) * ur - bn * vbr;
    f[5] = byr * ur - bn * vr;
    f[6] = bzr * ur - bn * zr;
  } else {
    const R sdl = sl - ul, sdr = sr - ur;
    const R den = sdr * rr - sdl * rl;
    const R sm = qdiv_t<FD>(sdr * rr * ur - sdl * rl * ul - ptr + ptl, den);
    const R pts = qdiv_t<FD>(sdr * rr * ptl - sdl * rl * ptr + rl * rr * sdr * sdl * (ur - ul), den);
    // left star state
    const R rls = qdiv_t<FD>(rl * sdl, sl - sm);
    R vls, zls, byls, bzls;
    star_transverse<FD>(rl, sdl, sl, sm, ul, vl, zl, byl, bzl, bn, vls, zls, byls, bzls);
    const R vbls = sm * bn + vls * byls + zls * bzls;
    const R els = qdiv_t<FD>(sdl * el - ptl * ul + pts * sm + bn * (vbl - vbls), sl - sm);
    // right star state
    const R rrs = qdiv_t<FD>(rr * sdr, sr - sm);
    R vrs, zrs, byrs, bzrs;
    star_transverse<FD>(rr, sdr, sr, sm, ur, vr, zr, byr, bzr, bn, vrs, zrs, byrs, bzrs);
    const R vbrs = sm * bn + vrs * byrs + zrs * bzrs;
    const R ers = qdiv_t<FD>(sdr * er - ptr * ur + pts * sm + bn * (vbr - vbrs), sr - sm);

    const bool skip = bn2 <= R(1e-12) * (ptl + ptr);
    const R sql = qsqrt(rls), sqr = qsqrt(rrs);
    const R abn = fabs(bn);
    const R ssl = skip ? sm : sm - qdiv_t<FD>(abn, sql);
    const R ssr = skip ? sm : sm + qdiv_t<FD>(abn, sqr);
    const bool left = sm >= R(0);
    // star flux of the side that holds x/t = 0
    R us[7], uo[7], fo[7], s_out;
    if (left) {
      us[0] = rls; us[1] = rls * sm; us[2] = rls * vls; us[3] = rls * zls; us[4] = els; us[5] = byls; us[6] = bzls;
      uo[0] = rl; uo[1] = rl * ul; uo[2] = rl * vl; uo[3] = rl * zl; uo[4] = el; uo[5] = byl; uo[6] = bzl;
      fo[0] = rl * ul; fo[1] = rl * ul * ul + ptl - bn2; fo[2] = rl * ul * vl - bn * byl; fo[3] = rl * ul * zl - bn * bzl;
      fo[4] = (el + ptl) * ul - bn * vbl; fo[5] = byl * ul - bn * vl; fo[6] = bzl * ul - bn * zl;
      s_out = sl;
    } else {
      us[0] = rrs; us[1] = rrs * sm; us[2] = rrs * vrs; us[3] = rrs * zrs; us[4] = ers; us[5] = byrs; us[6] = bzrs;
      uo[0] = rr; uo[1] = rr * ur; uo[2] = rr * vr; uo[3] = rr * zr; uo[4] = er; uo[5] = byr; uo[6] = bzr;
      fo[0] = rr * ur; fo[1] = rr * ur * ur + ptr - bn2; fo[2] = rr * ur * vr - bn * byr; fo[3] = rr * ur * zr - bn * bzr;
      fo[4] = (er + ptr) * ur - bn * vbr; fo[5] = byr * ur - bn * vr; fo[6] = bzr * ur - bn * zr;
      s_out = sr;
    }
    for (int q = 0; q < 7; ++q) f[q] = fo[q] + s_out * (us[q] - uo[q]);
    const bool in_star = left ? (ssl >= R(0)) : !(ssr >= R(0));
    if (!skip && !in_star) {
      // double-star state of the same side
      const R sgn = bn > R(0) ? R(1) : (bn < R(0) ? R(-1) : R(0));
      const R inv = rcp_t<FD>(sql + sqr);
      const R vss = (sql * vls + sqr * vrs + (byrs - byls) * sgn) * inv;
      const R zss = (sql * zls + sqr * zrs + (bzrs - bzls) * sgn) * inv;
      const R byss = (sql * byrs + sqr * byls + sql * sqr * (vrs - vls) * sgn) * inv;
      const R bzss = (sql * bzrs + sqr * bzls + sql * sqr * (zrs - zls) * sgn) * inv;
      const R vbss = sm * bn + vss * byss + zss * bzss;
      R uss[7];
      const R rs = left ? rls : rrs;
      uss[0] = rs; uss[1] = rs * sm; uss[2] = rs * vss; uss[3] = rs * zss;
      uss[4] = left ? els - sql * (vbls - vbss) * sgn : ers + sqr * (vbrs - vbss) * sgn;
      uss[5] = byss; uss[6] = bzss;
      const R ss = left ? ssl : ssr;
      for (int q = 0; q < 7; ++q) f[q] = f[q] + ss * (uss[q] - us[q]);
    }
  }
  // a mass flux at round-off level of its scale max(rho) max(|S|) vanishes in exact arithmetic (a
  // stagnant face ahead of a flow front); it is set to zero because the edge EMFs take their upwind
  // side from its sign, which would otherwise follow the rounding (the same band in every
  // precision: a wider one for float states moves the upwind choice at genuine small mass fluxes)
  const R mscale = fmax(rl, rr) * fmax(fabs(sl), fabs(sr));
  out[0] = fabs(f[0]) <= R(1e-12) * mscale ? R(0) : f[0];
  out[1 + D] = f[1];
  out[1 + T1] = f[2];
  out[1 + T2] = f[3];
  out[4] = f[4];
  out[5 + D] = R(0);
  out[5 + T1] = f[5];
  out[5 + T2] = f[6];
}

// Isothermal HLLC flux normal to D (the isothermal workload): mass and normal momentum are the
// HLL fluxes between S_L = min(u) - c_s and S_R = max(u) + c_s, the transverse momenta carry the
// transverse velocity of the side the contact speed S_M = F_rho / rho_hll comes from (left for
// S_M >= 0); energy and field fluxes are zero.
template <int D, typename R>
__device__ __forceinline__ void hllc_iso(const R* wl, const R* wr, R cs, R* out) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const R cs2 = cs * cs;
  const R rl = wl[0], ul = wl[1 + D], rr = wr[0], ur = wr[1 + D];
  const R sl = fmin(ul, ur) - cs;
  const R sr = fmax(ul, ur) + cs;
  const R fl0 = rl * ul, fr0 = rr * ur;
  R f0, fn, ft1, ft2;
  if (sl >= R(0)) {
    f0 = fl0;
    fn = rl * ul * ul + cs2 * rl;
    ft1 = rl * wl[1 + T1] * ul;
    ft2 = rl * wl[1 + T2] * ul;
  } else if (sr <= R(0)) {
    f0 = fr0;
    fn = rr * ur * ur + cs2 * rr;
    ft1 = rr * wr[1 + T1] * ur;
    ft2 = rr * wr[1 + T2] * ur;
  } else {
    const R fln = rl * ul * ul + cs2 * rl, frn = rr * ur * ur + cs2 * rr;
    const R inv = rcp(sr - sl);
    f0 = (sr * fl0 - sl * fr0 + sl * sr * (rr - rl)) * inv;
    fn = (sr * fln - sl * frn + sl * sr * (rr * ur - rl * ul)) * inv;
    const R rho_hll = (sr * rr - sl * rl - (fr0 - fl0)) * inv;
    const bool left = qdiv(f0, rho_hll) >= R(0);
    ft1 = f0 * (left ? wl[1 + T1] : wr[1 + T1]);
    ft2 = f0 * (left ? wl[1 + T2] : wr[1 + T2]);
  }
  out[0] = f0;
  out[1 + D] = fn;
  out[1 + T1] = ft1;
  out[1 + T2] = ft2;
  out[4] = R(0);
  out[5] = out[6] = out[7] = R(0);
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* slot, double v) {
  // non-negative doubles order like their bit patterns
  if (!(v >= 0.0)) v = 1.0e308;  // NaN: report as huge
  atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void flag_phys(unsigned long long* slots) { atomicOr(&slots[SLOT_PHYS], 1ULL); }

// time step of a level: dt0 (device slot) * 2^-level, exact
__device__ __forceinline__ double level_dt(const DevCtx& c, int level) {
  return ldexp(__longlong_as_double((long long)c.slots[SLOT_DT]), -level);
}

// ---------------------------------------------------------------------------
// task lookup
// ---------------------------------------------------------------------------
struct Where {
  int task;
  int i, j, k;
};

// Workgroups are handed to the 8 XCDs round-robin; renumber them so that each
// XCD (with its own L2) works on one contiguous range of logical blocks, i.e.
// on a compact slab of the region, and stencil neighbours stay in its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// q = n / d and r = n % d for n < 2^31 and 1 <= d < 2^20, from a double reciprocal of d: the
// product is within 2^-20 of n / d, so its truncation is the quotient or one less (when n / d is
// an integer and 1/d rounded down), fixed by one comparison.
__device__ __forceinline__ void split_index(unsigned n, unsigned d, double inv, unsigned& q, int& r) {
  unsigned qq = (unsigned)((double)n * inv);
  unsigned rr = n - qq * d;
  if (rr >= d) {
    ++qq;
    rr -= d;
  }
  q = qq;
  r = (int)rr;
}

// Task of block b (0 <= b < the list's block count) of the list starting at task `first`: one lookup
// in the list's block table.
__device__ __forceinline__ int task_of_block(const DevCtx& c, int first, int b) { return c.b2t[c.tbl[first] + b]; }

// Entry of thread `tid` of block b of a launch over a task list (its task and padded (i, j, k)).
__device__ __forceinline__ bool locate_tid(const DevCtx& c, int first, int n, int b, int tid, Where& w) {
  (void)n;
  const int t = task_of_block(c, first, b);
  const Task& T = c.tasks[t];
  // a region lies inside one padded patch, whose volume the host keeps below 2^31 entries
  const unsigned ex = T.hi[0] - T.lo[0], ey = T.hi[1] - T.lo[1], ez = T.hi[2] - T.lo[2];
  const unsigned local = (unsigned)(b - c.blk[t]) * AMRX_BLOCK + (unsigned)tid;
  if (local >= ex * ey * ez) return false;
  w.task = t;
  unsigned row, k;
  split_index(local, ex, T.inv0, row, w.i);
  split_index(row, ey, T.inv1, k, w.j);
  w.i += T.lo[0];
  w.j += T.lo[1];
  w.k = T.lo[2] + (int)k;
  return true;
}

__device__ __forceinline__ bool locate(const DevCtx& c, int first, int n, int b, Where& w) {
  return locate_tid(c, first, n, b, (int)threadIdx.x, w);
}

struct Strides {
  long long s[3];
  long long v;
};
__device__ __forceinline__ Strides strides(const PatchDev& p) {
  Strides s;
  s.s[0] = 1;
  s.s[1] = p.dim[0];
  s.s[2] = (long long)p.dim[0] * p.dim[1];
  s.v = p.vol;
  return s;
}

// register precision per mode
template <typename R, bool MIX> struct RegOf { using T = double; };
template <> struct RegOf<float, false> { using T = float; };

// set (mode 0) or add (mode 1) a value into an (acc, lo) register pair
template <typename Q, bool MIX>
__device__ __forceinline__ void reg_put(Q* acc, Q* lo, long long idx, Q v, int mode) {
  if (mode == 0) {
    acc[idx] = v;
    if (MIX) lo[idx] = Q(0);
  } else if (MIX) {
    const Q a = acc[idx];
    const Q s = a + v;
    const Q bb = s - a;
    const Q err = (a - (s - bb)) + (v - bb);
    acc[idx] = s;
    lo[idx] = lo[idx] + err;
  } else {
    acc[idx] = acc[idx] + v;
  }
}
template <typename Q, bool MIX>
__device__ __forceinline__ Q reg_get(const Q* acc, const Q* lo, long long idx) {
  return MIX ? acc[idx] + lo[idx] : acc[idx];
}

// 16-byte vector access to the interleaved intermediates (records of 4 or 8 reals)
__device__ __forceinline__ void ld4(const float* p, float* o) {
  const float4 a = *(const float4*)p;
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}
__device__ __forceinline__ void ld4(const double* p, double* o) {
  const double2 a = ((const double2*)p)[0], b = ((const double2*)p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
template <typename R>
__device__ __forceinline__ void ld8(const R* p, R* o) {
  ld4(p, o);
  ld4(p + 4, o + 4);
}
__device__ __forceinline__ void st4(float* p, const float* v) { *(float4*)p = make_float4(v[0], v[1], v[2], v[3]); }
__device__ __forceinline__ void st4(double* p, const double* v) {
  ((double2*)p)[0] = make_double2(v[0], v[1]);
  ((double2*)p)[1] = make_double2(v[2], v[3]);
}
template <typename R>
__device__ __forceinline__ void st8(R* p, const R* v) {
  st4(p, v);
  st4(p + 4, v + 4);
}

// ---------------------------------------------------------------------------
// stage 1: primitives and cell EMFs at t^n   (cells of the region grown by 2)
// ---------------------------------------------------------------------------
template <typename R, bool MIX>
__device__ __forceinline__ void d_prim(const DevCtx& c, int vb, int nb, int first, int n, int cur) {
  (void)nb;
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const PatchDev& p = c.patches[c.tasks[w.task].patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* X = (R*)c.rscr + p.scr;
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  const long long v = S.v;
  const R gm1 = R(c.gamma) - R(1);
  const R rho = U[q], mx = U[v + q], my = U[2 * v + q], mz = U[3 * v + q], e = U[4 * v + q];
  const R bx = R(0.5) * (U[5 * v + q] + U[5 * v + q + 1]);
  const R by = R(0.5) * (U[6 * v + q] + U[6 * v + q + S.s[1]]);
  const R bz = R(0.5) * (U[7 * v + q] + U[7 * v + q + S.s[2]]);
  const R vx = qdiv(mx, rho), vy = qdiv(my, rho), vz = qdiv(mz, rho);
  const R pr = c.iso ? R(c.cs2) * rho : pressure<R, MIX>(rho, mx, my, mz, e, bx, by, bz, gm1);
  if (!(rho > R(0)) || !(pr > R(0)) || !isfinite(e)) flag_phys(c.slots);
  const R wv[8] = {rho, vx, vy, vz, pr, bx, by, bz};
  st8(X + SCR_W * v + 8 * q, wv);
  R* EC = X + SCR_EC * v;
  EC[q] = -(vy * bz - vz * by);
  EC[v + q] = -(vz * bx - vx * bz);
  EC[2 * v + q] = -(vx * by - vy * bx);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_prim(DevCtx c, int first, int n, int cur) {
  d_prim<R, MIX>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur);
}

// ---------------------------------------------------------------------------
// stage 2: face-normal field at t^{n+1/2} (faces of the cells of the region grown by 1)
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R ebar(const R* ec, long long q, long long sa, long long sc) {
  return R(0.25) * (ec[q] + ec[q - sa] + ec[q - sc] + ec[q - sa - sc]);
}

template <int D, typename R>
__device__ __forceinline__ R bhalf_axis(const R* U, const R* EC, const Strides& S, long long q, R half_dt_dx) {
  constexpr int A = (D + 1) % 3, C = (D + 2) % 3;
  // edge-averaged cell EMFs: component C has in-plane axes (D, A); component A has (C, D)
  const R* ecC = EC + C * S.v;
  const R* ecA = EC + A * S.v;
  const R eC0 = ebar(ecC, q, S.s[D], S.s[A]);
  const R eC1 = ebar(ecC, q + S.s[A], S.s[D], S.s[A]);
  const R eA0 = ebar(ecA, q, S.s[C], S.s[D]);
  const R eA1 = ebar(ecA, q + S.s[C], S.s[C], S.s[D]);
  const R curl = (eC1 - eC0) - (eA1 - eA0);
  return U[(5 + D) * S.v + q] - half_dt_dx * curl;
}

template <typename R, bool MIX>
__device__ __forceinline__ void d_bhalf(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level) {
  (void)nb;
  const double dt = level_dt(c, level);
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* X = (R*)c.rscr + p.scr;
  const R* EC = X + SCR_EC * S.v;
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  const R h = R(0.5 * dt / p.dx);
  // the task region is the node box [lo, hi]; the cell box is [lo, hi - 1]
  const bool ix = w.i < T.hi[0] - 1, iy = w.j < T.hi[1] - 1, iz = w.k < T.hi[2] - 1;
  R* BH = X + SCR_BH * S.v;
  if (iy && iz) BH[q] = bhalf_axis<0>(U, EC, S, q, h);
  if (ix && iz) BH[S.v + q] = bhalf_axis<1>(U, EC, S, q, h);
  if (ix && iy) BH[2 * S.v + q] = bhalf_axis<2>(U, EC, S, q, h);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_bhalf(DevCtx c, int first, int n, int cur, int level) {
  d_bhalf<R, MIX>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level);
}

// ---------------------------------------------------------------------------
// stage 3: limited slopes, conservative Hancock half step and the cell
// reference EMF at t^{n+1/2} (cells of the region grown by 1)
// ---------------------------------------------------------------------------
template <int D, typename R>
__device__ __forceinline__ void hancock_axis(const R* W, long long q, long long sd, const R* w0, R gm1, R half_dt_dx,
                                             R* du) {
  R wm[8], wp[8], f1[8], f2[8];
  ld8(W + 8 * (q - sd), wm);
  ld8(W + 8 * (q + sd), wp);
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const R s = mc_limit(w0[m] - wm[m], wp[m] - w0[m]);
    wp[m] = w0[m] + R(0.5) * s;
    wm[m] = w0[m] - R(0.5) * s;
  }
  phys_flux<D>(wp, gm1, f1);
  phys_flux<D>(wm, gm1, f2);
#pragma unroll
  for (int m = 0; m < 8; ++m) du[m] -= half_dt_dx * (f1[m] - f2[m]);
}

template <typename R, bool MIX>
__device__ __forceinline__ void d_pred(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level) {
  (void)nb;
  const double dt = level_dt(c, level);
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const PatchDev& p = c.patches[c.tasks[w.task].patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* X = (R*)c.rscr + p.scr;
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  const long long v = S.v;
  const R* W = X + SCR_W * v;
  const R gm1 = R(c.gamma) - R(1);
  const R h = R(0.5 * dt / p.dx);
  R w0[8], du[8];
  ld8(W + 8 * q, w0);
#pragma unroll
  for (int m = 0; m < 8; ++m) du[m] = R(0);
  hancock_axis<0>(W, q, S.s[0], w0, gm1, h, du);
  hancock_axis<1>(W, q, S.s[1], w0, gm1, h, du);
  hancock_axis<2>(W, q, S.s[2], w0, gm1, h, du);
  st8(X + SCR_DU * v + 8 * q, du);
  // half-step velocity and face-averaged half-step field -> reference EMF
  const R* BH = X + SCR_BH * v;
  const R rho = U[q] + du[0];
  const R vx = qdiv(U[v + q] + du[1], rho);
  const R vy = qdiv(U[2 * v + q] + du[2], rho);
  const R vz = qdiv(U[3 * v + q] + du[3], rho);
  const R bx = R(0.5) * (BH[q] + BH[q + 1]);
  const R by = R(0.5) * (BH[v + q] + BH[v + q + S.s[1]]);
  const R bz = R(0.5) * (BH[2 * v + q] + BH[2 * v + q + S.s[2]]);
  R* ER = X + SCR_ER * v;
  ER[q] = -(vy * bz - vz * by);
  ER[v + q] = -(vz * bx - vx * bz);
  ER[2 * v + q] = -(vx * by - vy * bx);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_pred(DevCtx c, int first, int n, int cur, int level) {
  d_pred<R, MIX>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level);
}

// ---------------------------------------------------------------------------
// stages 1-3 fused: one workgroup per tile of the primitive region (the update
// region grown by 2).  The primitives and cell EMFs of the tile and a one-cell
// halo are computed into LDS, the half-step face field of the tile's faces
// from them, then the Hancock increments and reference EMFs of the tile's
// cells that lie in the update region grown by 1.  Results are bit-identical
// to the three staged kernels (same operations in the same order); the cell
// EMFs never reach HBM and the primitives are read back from LDS.
// ---------------------------------------------------------------------------
// Walk over a box nx x ny x nz in steps of `step` linear entries (x fastest) without a
// division per entry: the coordinates of the start and of the step are split once and
// then added with carries.
struct Walk3 {
  int x, y, z, dx, dy, dz, nx, ny;
  __device__ __forceinline__ Walk3(int t, int step, int nx_, int ny_) : nx(nx_), ny(ny_) {
    int r = t / nx;
    x = t - r * nx;
    y = r % ny;
    z = r / ny;
    r = step / nx;
    dx = step - r * nx;
    dy = r % ny;
    dz = r / ny;
  }
  __device__ __forceinline__ void next() {
    x += dx;
    const int cx = x >= nx ? 1 : 0;
    x -= cx * nx;
    y += dy + cx;
    const int cy = y >= ny ? 1 : 0;
    y -= cy * ny;
    z += dz + cy;
  }
};

template <typename R>
__device__ __forceinline__ R ebar_l(const R* ec, int q, int sa, int sc) {
  return R(0.25) * (ec[q] + ec[q - sa] + ec[q - sc] + ec[q - sa - sc]);
}

template <int D, typename R>
__device__ __forceinline__ R bhalf_lds(R face, const R* sE, int HV, int hq, const int hs[3], R half_dt_dx) {
  constexpr int A = (D + 1) % 3, C = (D + 2) % 3;
  const R* ecC = sE + C * HV;
  const R* ecA = sE + A * HV;
  const R eC0 = ebar_l(ecC, hq, hs[D], hs[A]);
  const R eC1 = ebar_l(ecC, hq + hs[A], hs[D], hs[A]);
  const R eA0 = ebar_l(ecA, hq, hs[C], hs[D]);
  const R eA1 = ebar_l(ecA, hq + hs[C], hs[C], hs[D]);
  const R curl = (eC1 - eC0) - (eA1 - eA0);
  return face - half_dt_dx * curl;
}

template <int D, typename R>
__device__ __forceinline__ void hancock_lds(const R* sW, int HV, int hq, int sd, const R* w0, R gm1, R half_dt_dx,
                                            R* du) {
  R wm[8], wp[8], f1[8], f2[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    wm[m] = sW[m * HV + hq - sd];
    wp[m] = sW[m * HV + hq + sd];
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const R s = mc_limit(w0[m] - wm[m], wp[m] - w0[m]);
    wp[m] = w0[m] + R(0.5) * s;
    wm[m] = w0[m] - R(0.5) * s;
  }
  phys_flux<D>(wp, gm1, f1);
  phys_flux<D>(wm, gm1, f2);
#pragma unroll
  for (int m = 0; m < 8; ++m) du[m] -= half_dt_dx * (f1[m] - f2[m]);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_fused_a(DevCtx c, int first, int n, int cur, int level, int tx, int ty,
                                                         int tz) {
  extern __shared__ double smem_d[];
  R* sm = reinterpret_cast<R*>(smem_d);
  const int nthr = blockDim.x;
  const int vb = xcd_block(blockIdx.x, gridDim.x);
  (void)n;
  const int t = task_of_block(c, first, vb);
  const Task& T = c.tasks[t];
  const int tile = vb - c.blk[t];
  const int ntx = (T.hi[0] - T.lo[0] + tx - 1) / tx, nty = (T.hi[1] - T.lo[1] + ty - 1) / ty;
  const int tix = tile % ntx, tiy = (tile / ntx) % nty, tiz = tile / (ntx * nty);
  const int o[3] = {T.lo[0] + tix * tx, T.lo[1] + tiy * ty, T.lo[2] + tiz * tz};
  const int e[3] = {min(tx, T.hi[0] - o[0]), min(ty, T.hi[1] - o[1]), min(tz, T.hi[2] - o[2])};
  // region grown by 1 (the half-step region): the task region shrunk by one cell
  const int lo1[3] = {T.lo[0] + 1, T.lo[1] + 1, T.lo[2] + 1};
  const int hi1[3] = {T.hi[0] - 1, T.hi[1] - 1, T.hi[2] - 1};

  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* X = (R*)c.rscr + p.scr;
  const long long v = S.v;
  const R gm1 = R(c.gamma) - R(1);
  const double dt = level_dt(c, level);
  const R h = R(0.5 * dt / p.dx);

  const int H0 = tx + 2, H1 = ty + 2, H2 = tz + 2;
  const int HV = H0 * H1 * H2;
  const int hs[3] = {1, H0, H0 * H1};
  const int N0 = tx + 1, N1 = ty + 1;
  const int NB = N0 * N1 * (tz + 1);
  const int ns[3] = {1, N0, N0 * N1};
  R* sW = sm;            // 8 x HV primitives
  R* sE = sW + 8 * HV;   // 3 x HV cell EMFs
  R* sB = sE + 3 * HV;   // 3 x NB half-step face field (low faces of the tile's cells + one layer)

  // 1. primitives and cell EMFs of the tile and its halo (cells that exist in the padded arrays)
  Walk3 w1(threadIdx.x, nthr, H0, H1);
  for (int t = threadIdx.x; t < HV; t += nthr, w1.next()) {
    const int hx = w1.x, hy = w1.y, hz = w1.z;
    const int i = o[0] - 1 + hx, j = o[1] - 1 + hy, k = o[2] - 1 + hz;
    if (i < 0 || j < 0 || k < 0 || i >= p.dim[0] - 1 || j >= p.dim[1] - 1 || k >= p.dim[2] - 1) continue;
    const long long q = i + j * S.s[1] + k * S.s[2];
    const R rho = U[q], mx = U[v + q], my = U[2 * v + q], mz = U[3 * v + q], en = U[4 * v + q];
    const R bx = R(0.5) * (U[5 * v + q] + U[5 * v + q + 1]);
    const R by = R(0.5) * (U[6 * v + q] + U[6 * v + q + S.s[1]]);
    const R bz = R(0.5) * (U[7 * v + q] + U[7 * v + q + S.s[2]]);
    const R vx = qdiv(mx, rho), vy = qdiv(my, rho), vz = qdiv(mz, rho);
    const R pr = c.iso ? R(c.cs2) * rho : pressure<R, MIX>(rho, mx, my, mz, en, bx, by, bz, gm1);
    const R wv[8] = {rho, vx, vy, vz, pr, bx, by, bz};
#pragma unroll
    for (int m = 0; m < 8; ++m) sW[m * HV + t] = wv[m];
    sE[t] = -(vy * bz - vz * by);
    sE[HV + t] = -(vz * bx - vx * bz);
    sE[2 * HV + t] = -(vx * by - vy * bx);
    if (hx >= 1 && hx <= e[0] && hy >= 1 && hy <= e[1] && hz >= 1 && hz <= e[2]) {
      if (!(rho > R(0)) || !(pr > R(0)) || !isfinite(en)) flag_phys(c.slots);
      st8(X + SCR_W * v + 8 * q, wv);
    }
  }
  __syncthreads();

  // 2. half-step normal field on the faces of the half-step region's cells
  R* BH = X + SCR_BH * v;
  Walk3 w2(threadIdx.x, nthr, N0, N1);
  for (int t = threadIdx.x; t < NB; t += nthr, w2.next()) {
    const int fx = w2.x, fy = w2.y, fz = w2.z;
    const int i = o[0] + fx, j = o[1] + fy, k = o[2] + fz;
    // in_d: a face position along d (low faces of the tile's cells and the next one);
    // c_d: a cell of the tile along d; both restricted to the half-step region
    const bool in0 = fx <= e[0] && i >= lo1[0] && i <= hi1[0];
    const bool in1 = fy <= e[1] && j >= lo1[1] && j <= hi1[1];
    const bool in2 = fz <= e[2] && k >= lo1[2] && k <= hi1[2];
    const bool c0 = in0 && fx < e[0] && i < hi1[0];
    const bool c1 = in1 && fy < e[1] && j < hi1[1];
    const bool c2 = in2 && fz < e[2] && k < hi1[2];
    const int hq = (fx + 1) + (fy + 1) * hs[1] + (fz + 1) * hs[2];
    const long long q = i + j * S.s[1] + k * S.s[2];
    if (in0 && c1 && c2) {
      const R b = bhalf_lds<0>(U[5 * v + q], sE, HV, hq, hs, h);
      sB[t] = b;
      if (fx < e[0]) BH[q] = b;
    }
    if (c0 && in1 && c2) {
      const R b = bhalf_lds<1>(U[6 * v + q], sE, HV, hq, hs, h);
      sB[NB + t] = b;
      if (fy < e[1]) BH[v + q] = b;
    }
    if (c0 && c1 && in2) {
      const R b = bhalf_lds<2>(U[7 * v + q], sE, HV, hq, hs, h);
      sB[2 * NB + t] = b;
      if (fz < e[2]) BH[2 * v + q] = b;
    }
  }
  __syncthreads();

  // 3. Hancock increments and reference EMFs of the tile's cells in the half-step region
  const int CV = tx * ty * tz;
  Walk3 w3(threadIdx.x, nthr, tx, ty);
  for (int t = threadIdx.x; t < CV; t += nthr, w3.next()) {
    const int cx = w3.x, cy = w3.y, cz = w3.z;
    if (cx >= e[0] || cy >= e[1] || cz >= e[2]) continue;
    const int i = o[0] + cx, j = o[1] + cy, k = o[2] + cz;
    if (i < lo1[0] || i >= hi1[0] || j < lo1[1] || j >= hi1[1] || k < lo1[2] || k >= hi1[2]) continue;
    const int hq = (cx + 1) + (cy + 1) * hs[1] + (cz + 1) * hs[2];
    const long long q = i + j * S.s[1] + k * S.s[2];
    R w0[8], du[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      w0[m] = sW[m * HV + hq];
      du[m] = R(0);
    }
    hancock_lds<0>(sW, HV, hq, hs[0], w0, gm1, h, du);
    hancock_lds<1>(sW, HV, hq, hs[1], w0, gm1, h, du);
    hancock_lds<2>(sW, HV, hq, hs[2], w0, gm1, h, du);
    st8(X + SCR_DU * v + 8 * q, du);
    const int nq = cx + cy * ns[1] + cz * ns[2];
    const R rho = U[q] + du[0];
    const R vx = qdiv(U[v + q] + du[1], rho);
    const R vy = qdiv(U[2 * v + q] + du[2], rho);
    const R vz = qdiv(U[3 * v + q] + du[3], rho);
    const R bx = R(0.5) * (sB[nq] + sB[nq + 1]);
    const R by = R(0.5) * (sB[NB + nq] + sB[NB + nq + ns[1]]);
    const R bz = R(0.5) * (sB[2 * NB + nq] + sB[2 * NB + nq + ns[2]]);
    R* ER = X + SCR_ER * v;
    ER[q] = -(vy * bz - vz * by);
    ER[v + q] = -(vz * bx - vx * bz);
    ER[2 * v + q] = -(vx * by - vy * bx);
  }
}

// ---------------------------------------------------------------------------
// stage 4: HLLD fluxes through the faces normal to D, boundary registers
// ---------------------------------------------------------------------------
// PASS (FP32_MIXED only): 0 = every face in one pass, the Riemann solver in double at low-beta
// faces; 1 = float faces only, a low-beta face gets a NaN mass flux and nothing else; 2 = the faces
// pass 1 left, in double.  Split in two launches, the float kernel keeps the register footprint of
// the plain FP32 one; the arithmetic of every face is the same in both forms.
template <int D, typename R, bool MIX, bool ISO, int PASS = 0>
__device__ bool flux_face(const DevCtx& c, const PatchDev& p, const Strides& S, R* X, int i, int j, int k, int level,
                          int substep, double dt) {
  using Q = typename RegOf<R, MIX>::T;
  constexpr int A = (D + 1) % 3, C = (D + 2) % 3;
  const long long v = S.v;
  const long long sd = S.s[D];
  const long long q = i + j * S.s[1] + k * S.s[2];
  const R* W = X + SCR_W * v;
  const R* DU = X + SCR_DU * v;
  const R gamma = R(c.gamma);
  const R gm1 = gamma - R(1);
  R a[8], b[8], cc[8], wl[8], wr[8], u[8], d[8];
  ld8(W + 8 * (q - 2 * sd), a);
  ld8(W + 8 * (q - sd), b);
  ld8(W + 8 * q, cc);
  // + state of the cell on the low side
#pragma unroll
  for (int m = 0; m < 8; ++m) wl[m] = b[m] + R(0.5) * mc_limit(b[m] - a[m], cc[m] - b[m]);
  ld8(W + 8 * (q + sd), a);
  // - state of the cell on the high side
#pragma unroll
  for (int m = 0; m < 8; ++m) wr[m] = cc[m] - R(0.5) * mc_limit(cc[m] - b[m], a[m] - cc[m]);
  to_cons(wl, gm1, u);
  ld8(DU + 8 * (q - sd), d);
#pragma unroll
  for (int m = 0; m < 8; ++m) u[m] += d[m];
  if constexpr (ISO) to_prim_iso(u, R(c.cs2), wl);
  else to_prim<R, MIX>(u, gm1, wl);
  to_cons(wr, gm1, u);
  ld8(DU + 8 * q, d);
#pragma unroll
  for (int m = 0; m < 8; ++m) u[m] += d[m];
  if constexpr (ISO) to_prim_iso(u, R(c.cs2), wr);
  else to_prim<R, MIX>(u, gm1, wr);
  if (!(wl[0] > R(0)) || !(wl[4] > R(0)) || !(wr[0] > R(0)) || !(wr[4] > R(0))) flag_phys(c.slots);
  const R bn = X[(SCR_BH + D) * v + q];
  R f[8];
  // FP32_MIXED at low-beta faces (beta = 2p/B^2 < 0.1 on either side): the Riemann solver in
  // double.  With a strong field the star states approach the degenerate limit
  // rho (S - u)^2 ~ Bn^2, where float32 rounding of the wave speeds and of
  // rho (S - u)(S - S_M) - Bn^2 decides between branches.
  bool low_beta = false;
  if (MIX) {
    const R bn2 = bn * bn;
    const R b2l = bn2 + wl[5 + (D + 1) % 3] * wl[5 + (D + 1) % 3] + wl[5 + (D + 2) % 3] * wl[5 + (D + 2) % 3];
    const R b2r = bn2 + wr[5 + (D + 1) % 3] * wr[5 + (D + 1) % 3] + wr[5 + (D + 2) % 3] * wr[5 + (D + 2) % 3];
    low_beta = R(20) * fmin(wl[4], wr[4]) < fmax(b2l, b2r);
  }
  if constexpr (ISO) {
    hllc_iso<D, R>(wl, wr, R(sqrt(c.cs2)), f);
  } else if constexpr (PASS == 1) {
    if (low_beta) {
      X[(SCR_F0 + D) * v + q] = R(__builtin_nan(""));
      return true;
    }
    hlld<D, R>(wl, wr, bn, gamma, f);
  } else {
    if (PASS == 2 && !low_beta) return false;  // a non-finite flux of pass 1, not a face left to this pass
    if (low_beta) {
      double wld[8], wrd[8], fd[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        wld[m] = wl[m];
        wrd[m] = wr[m];
      }
      hlld<D, double, true>(wld, wrd, (double)bn, c.gamma, fd);
#pragma unroll
      for (int m = 0; m < 8; ++m) f[m] = (R)fd[m];
    } else {
      hlld<D, R>(wl, wr, bn, gamma, f);
    }
  }
  const R rec[4] = {f[1], f[2], f[3], f[4]};
  st4(X + (SCR_F4 + 4 * D) * v + 4 * q, rec);
  X[(SCR_F0 + D) * v + q] = f[0];
  X[(SCR_FE + 2 * D) * v + q] = -f[5 + A];     // EMF along C carried by this face
  X[(SCR_FE + 2 * D + 1) * v + q] = f[5 + C];  // EMF along A carried by this face

  // registers ---------------------------------------------------------------
  const int r[3] = {i - AMRX_G, j - AMRX_G, k - AMRX_G};
  int a1, a2;
  other_axes(D, a1, a2);
  Q* regs = (Q*)c.reg;
  const bool trans_in = r[a1] >= 0 && r[a1] < p.n[a1] && r[a2] >= 0 && r[a2] < p.n[a2];
  if (trans_in && (r[D] == 0 || r[D] == p.n[D])) {
    const int side = r[D] == 0 ? 0 : 1;
    const int mode = (level > 0 && substep > 0) ? 1 : 0;
    Q* acc = regs + p.freg;
    Q* lo = acc + p.fsize;
    Q* last = lo + p.fsize;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const long long idx = face_reg_index(p.n, D, side, m, r[a1], r[a2]);
      const Q val = (Q)f[m] * (Q)dt;
      reg_put<Q, MIX>(acc, lo, idx, val, mode);
      last[idx] = val;
    }
  }
  if (p.has_children) {
    const int* cov = c.cov + p.cov;
    const int cl = cov[q - sd], ch = cov[q];
    if ((cl >= 0) != (ch >= 0)) {
      const int child = cl >= 0 ? cl : ch;
      const PatchDev& cp = c.patches[child];
      const int side = ch >= 0 ? 0 : 1;
      const int nc[3] = {cp.n[0] / 2, cp.n[1] / 2, cp.n[2] / 2};
      const int g[3] = {i + p.lo[0] - AMRX_G, j + p.lo[1] - AMRX_G, k + p.lo[2] - AMRX_G};
      const int t1 = g[a1] - cp.lo[a1] / 2, t2 = g[a2] - cp.lo[a2] / 2;
#pragma unroll
      for (int m = 0; m < 5; ++m) regs[cp.creg + face_reg_index(nc, D, side, m, t1, t2)] = (Q)f[m] * (Q)dt;
    }
  }
  return false;
}

// ISO: the isothermal workload's faces (a separate instantiation, so the MHD kernel carries no
// branch of it); PASS 0 or 1 as in flux_face
// PASS 1 lists every wave that left a face: lbflag[0] counts the items, lbflag[1 + i] holds item i,
// block * (waves per block) + wave, appended by the wave's first lane that left one.
constexpr int kWavesPerBlock = AMRX_BLOCK / 64;

template <typename R, bool MIX, bool ISO = false, int PASS = 0>
__device__ __forceinline__ void d_flux(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level, int substep) {
  static_assert(PASS != 2, "pass 2 runs over the listed waves (d_flux_left)");
  (void)nb;
  const double dt = level_dt(c, level);
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  R* X = (R*)c.rscr + p.scr;
  (void)cur;
  bool left;
  if (T.axis == 0) left = flux_face<0, R, MIX, ISO, PASS>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else if (T.axis == 1) left = flux_face<1, R, MIX, ISO, PASS>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else left = flux_face<2, R, MIX, ISO, PASS>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  if constexpr (PASS == 1) {
    const unsigned long long m = __ballot(left);
    if (m != 0ull && (int)(threadIdx.x & 63) == __builtin_ctzll(m)) {
      const int at = atomicAdd(c.lbflag, 1);
      c.lbflag[1 + at] = vb * kWavesPerBlock + (int)(threadIdx.x >> 6);
    }
  }
}

// Pass 2 of FP32_MIXED: the entry of lane `tid` (0..255 within its block) of a listed pass-1 block
// whose mass flux pass 1 left as NaN, solved with the double Riemann solver.
template <typename R>
__device__ __forceinline__ void d_flux_left(const DevCtx& c, int vb, int tid, int first, int n, int level,
                                            int substep) {
  const double dt = level_dt(c, level);
  Where w;
  if (!locate_tid(c, first, n, vb, tid, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  R* X = (R*)c.rscr + p.scr;
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  if (!isnan(X[(SCR_F0 + T.axis) * S.v + q])) return;
  if (T.axis == 0) flux_face<0, R, true, false, 2>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else if (T.axis == 1) flux_face<1, R, true, false, 2>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else flux_face<2, R, true, false, 2>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
}

// the flux stage of either physics from a device-side scheduler (one code path per workload)
template <typename R, bool MIX>
__device__ __forceinline__ void d_flux_any(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level,
                                           int substep) {
  if (c.iso) d_flux<R, MIX, true>(c, vb, nb, first, n, cur, level, substep);
  else d_flux<R, MIX, false>(c, vb, nb, first, n, cur, level, substep);
}

// FP32_MIXED runs this kernel as pass 1 and k_flux_low_beta as pass 2 over the waves it listed
template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flux(DevCtx c, int first, int n, int cur, int level, int substep) {
  d_flux<R, MIX, false, MIX ? 1 : 0>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level, substep);
}

// each wave takes listed items in turn (a grid smaller than the list strides over it)
template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flux_low_beta(DevCtx c, int first, int n, int level, int substep) {
  const int count = c.lbflag[0];
  const int lane = (int)(threadIdx.x & 63);
#pragma unroll 1
  for (int it = (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6); it < count;
       it += (int)gridDim.x * kWavesPerBlock) {
    const int item = __builtin_amdgcn_readfirstlane(c.lbflag[1 + it]);  // one item per wave
    d_flux_left<R>(c, item / kWavesPerBlock, (item % kWavesPerBlock) * 64 + lane, first, n, level, substep);
  }
}

// FP32_MIXED in one pass (the double Riemann solver inline at low-beta faces)
template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flux_mixed_one_pass(DevCtx c, int first, int n, int cur, int level,
                                                                    int substep) {
  d_flux<R, true, false, 0>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level, substep);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flux_iso(DevCtx c, int first, int n, int cur, int level, int substep) {
  d_flux<R, MIX, true>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level, substep);
}

// ---------------------------------------------------------------------------
// stage 5: upwinded CT-contact edge EMFs along E, boundary registers
// ---------------------------------------------------------------------------
// EMF along E at the edge of padded index q (low corner of the cell q in the two other axes)
template <int E, typename R>
__device__ __forceinline__ R edge_value(const Strides& S, const R* X, long long q) {
  constexpr int A = (E + 1) % 3, C = (E + 2) % 3;
  const long long v = S.v;
  const long long sa = S.s[A], sc = S.s[C];
  const R* efa = X + (SCR_FE + 2 * A) * v;      // faces normal to A: EMF along (A+2)%3 = E
  const R* efc = X + (SCR_FE + 2 * C + 1) * v;  // faces normal to C: EMF along (C+1)%3 = E
  const R* fa0 = X + (SCR_F0 + A) * v;
  const R* fc0 = X + (SCR_F0 + C) * v;
  const R* er = X + (SCR_ER + E) * v;
  const R ea_bm = efa[q - sc], ea_b0 = efa[q];
  const R eb_am = efc[q - sa], eb_a0 = efc[q];
  const R r_mm = er[q - sa - sc], r_0m = er[q - sc], r_m0 = er[q - sa], r_00 = er[q];
  const R ma_hi = fa0[q], ma_lo = fa0[q - sc], mc_hi = fc0[q], mc_lo = fc0[q - sa];
  const R d_b_upper = upwind(ma_hi, r_m0 - eb_am, r_00 - eb_a0);
  const R d_b_lower = upwind(ma_lo, eb_am - r_mm, eb_a0 - r_0m);
  const R d_a_upper = upwind(mc_hi, r_0m - ea_bm, r_00 - ea_b0);
  const R d_a_lower = upwind(mc_lo, ea_bm - r_mm, ea_b0 - r_m0);
  return R(0.25) * (ea_bm + ea_b0 + eb_am + eb_a0) + R(0.25) * (d_b_lower - d_b_upper) +
         R(0.25) * (d_a_lower - d_a_upper);
}

// EMF x dt of the edge (i, j, k) along E into the patch's edge registers (edges on its box surface)
// and into a child's coarse edge registers (edges on a child's coarse box surface)
template <int E, typename R, bool MIX>
__device__ __forceinline__ void edge_registers(const DevCtx& c, const PatchDev& p, const Strides& S, int i, int j, int k,
                                               R emf, int level, int substep, double dt) {
  using Q = typename RegOf<R, MIX>::T;
  constexpr int A = (E + 1) % 3, C = (E + 2) % 3;
  const long long q = i + j * S.s[1] + k * S.s[2];
  const long long sa = S.s[A], sc = S.s[C];
  Q* regs = (Q*)c.reg;
  const int r[3] = {i - AMRX_G, j - AMRX_G, k - AMRX_G};
  const Q val = (Q)emf * (Q)dt;
  if (r[E] >= 0 && r[E] < p.n[E] && r[A] >= 0 && r[A] <= p.n[A] && r[C] >= 0 && r[C] <= p.n[C]) {
    const int mode = (level > 0 && substep > 0) ? 1 : 0;
    Q* acc = regs + p.ereg;
    Q* lo = acc + p.esize;
    if (r[A] == 0 || r[A] == p.n[A])
      reg_put<Q, MIX>(acc, lo, edge_reg_pa(p.n, E, r[A] == 0 ? 0 : 1, r[C], r[E]), val, mode);
    if (r[C] == 0 || r[C] == p.n[C])
      reg_put<Q, MIX>(acc, lo, edge_reg_pb(p.n, E, r[C] == 0 ? 0 : 1, r[A], r[E]), val, mode);
  }
  if (p.has_children) {
    const int* cov = c.cov + p.cov;
    const int nb[4] = {cov[q - sa - sc], cov[q - sc], cov[q - sa], cov[q]};
    const bool any = nb[0] >= 0 || nb[1] >= 0 || nb[2] >= 0 || nb[3] >= 0;
    const bool all = nb[0] >= 0 && nb[1] >= 0 && nb[2] >= 0 && nb[3] >= 0;
    if (any && !all) {
      const int owner = nb[0] >= 0 ? nb[0] : (nb[1] >= 0 ? nb[1] : (nb[2] >= 0 ? nb[2] : nb[3]));
      const PatchDev& cp = c.patches[owner];
      const int nc[3] = {cp.n[0] / 2, cp.n[1] / 2, cp.n[2] / 2};
      const int g[3] = {i + p.lo[0] - AMRX_G - cp.lo[0] / 2, j + p.lo[1] - AMRX_G - cp.lo[1] / 2,
                        k + p.lo[2] - AMRX_G - cp.lo[2] / 2};
      Q* cr = regs + cp.cereg;
      if (g[A] == 0 || g[A] == nc[A]) cr[edge_reg_pa(nc, E, g[A] == 0 ? 0 : 1, g[C], g[E])] = val;
      if (g[C] == 0 || g[C] == nc[C]) cr[edge_reg_pb(nc, E, g[C] == 0 ? 0 : 1, g[A], g[E])] = val;
    }
  }
}

template <int E, typename R, bool MIX>
__device__ void edge_emf(const DevCtx& c, const PatchDev& p, const Strides& S, R* X, int i, int j, int k, int level,
                         int substep, double dt) {
  const long long q = i + j * S.s[1] + k * S.s[2];
  const R emf = edge_value<E>(S, X, q);
  X[(SCR_E + E) * S.v + q] = emf;
  edge_registers<E, R, MIX>(c, p, S, i, j, k, emf, level, substep, dt);
}

template <typename R, bool MIX>
__device__ __forceinline__ void d_edge(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level, int substep) {
  (void)nb;
  const double dt = level_dt(c, level);
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  R* X = (R*)c.rscr + p.scr;
  (void)cur;
  if (T.axis == 0) edge_emf<0, R, MIX>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else if (T.axis == 1) edge_emf<1, R, MIX>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
  else edge_emf<2, R, MIX>(c, p, S, X, w.i, w.j, w.k, level, substep, dt);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_edge(DevCtx c, int first, int n, int cur, int level, int substep) {
  d_edge<R, MIX>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level, substep);
}

// ---------------------------------------------------------------------------
// stage 6: conservative cell update and Stokes face update into the next buffer
// ---------------------------------------------------------------------------
// Cell update (conservative flux differences) and Stokes update of the low faces of padded entry q
// (cell if ix && iy && iz; face normal to D if the two other flags hold).  Edge EMF along E at entry
// index eq + offsets is ee[E][...] with strides es (global arrays or an LDS tile).  Every operand is
// loaded before the first store: both state buffers share one arena, so a load after a store could
// not be moved ahead of it.
// Store of the next state: NT marks it non-temporal (a cache hint only; the value is the same).
template <bool NT, typename R>
__device__ __forceinline__ void store_next(R* p, R v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <typename R, typename I, bool NT = false>
__device__ __forceinline__ void update_entry(const R* U, R* N, const R* X, const Strides& S, long long q, bool ix,
                                             bool iy, bool iz, R dt_dx, const R* const ee[3], const I es[3], I eq) {
  const long long v = S.v;
  const bool cell = ix && iy && iz;
  const bool face[3] = {iy && iz, ix && iz, ix && iy};
  R u[5], f0[3][4], f1[3][4], m0[3], m1[3];
  if (cell) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const R* F4 = X + (SCR_F4 + 4 * d) * v;
      const R* F0 = X + (SCR_F0 + d) * v;
      ld4(F4 + 4 * q, f0[d]);
      ld4(F4 + 4 * (q + S.s[d]), f1[d]);
      m0[d] = F0[q];
      m1[d] = F0[q + S.s[d]];
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] = U[m * v + q];
  }
  // faces normal to D: curl of the edge EMFs along C = D+2 and A = D+1
  R bo[3], ec_hi[3], ec_lo[3], ea_hi[3], ea_lo[3];
#pragma unroll
  for (int D = 0; D < 3; ++D) {
    if (face[D]) {
      const int A = (D + 1) % 3, C = (D + 2) % 3;
      bo[D] = U[(5 + D) * v + q];
      ec_hi[D] = ee[C][eq + es[A]];
      ec_lo[D] = ee[C][eq];
      ea_hi[D] = ee[A][eq + es[C]];
      ea_lo[D] = ee[A][eq];
    }
  }
  if (cell) {
    R div[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      div[0] += m1[d] - m0[d];
#pragma unroll
      for (int m = 0; m < 4; ++m) div[1 + m] += f1[d][m] - f0[d][m];
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) store_next<NT>(N + m * v + q, u[m] - dt_dx * div[m]);
  }
#pragma unroll
  for (int D = 0; D < 3; ++D) {
    if (face[D]) {
      const R curl = (ec_hi[D] - ec_lo[D]) - (ea_hi[D] - ea_lo[D]);
      store_next<NT>(N + (5 + D) * v + q, bo[D] - dt_dx * curl);
    }
  }
}

template <typename R, bool MIX, bool NT = false>
__device__ __forceinline__ void d_update(const DevCtx& c, int vb, int nb, int first, int n, int cur, int level) {
  (void)nb;
  const double dt = level_dt(c, level);
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* N = (R*)c.state + p.st[1 - cur];
  const R* X = (const R*)c.rscr + p.scr;
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  const R dt_dx = R(dt / p.dx);
  const bool ix = w.i < T.hi[0] - 1, iy = w.j < T.hi[1] - 1, iz = w.k < T.hi[2] - 1;
  const R* EE = X + SCR_E * S.v;
  const R* const ee[3] = {EE, EE + S.v, EE + 2 * S.v};
  update_entry<R, long long, NT>(U, N, X, S, q, ix, iy, iz, dt_dx, ee, S.s, q);
}

template <typename R, bool MIX, bool NT = false>
__global__ __launch_bounds__(AMRX_BLOCK) void k_update(DevCtx c, int first, int n, int cur, int level) {
  d_update<R, MIX, NT>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur, level);
}

// ---------------------------------------------------------------------------
// stages 5-6 fused: one workgroup per tile of the update region.  The edge
// EMFs the tile's faces need (its own edges and one more layer on the high side
// of the two axes normal to each edge) are computed into LDS, then the cells
// and faces of the tile are updated from them.  Edges of the halo layer are
// computed again by the neighbouring tile with the same arithmetic, and only a
// tile's own edges write registers, so the results are bit-identical to the
// staged edge and update kernels; the edge EMFs never reach HBM.
// ---------------------------------------------------------------------------
// The tile's edges: at each entry of the tile grown by one node on the high side of every axis,
// the edges along x, y and z that the staged edge region holds there (along E the cells of the
// update region, along the other axes its nodes; along E within the tile, along the others up to
// one past it).  The three EMFs of an entry are computed together so their loads are in flight at
// once (every such entry lies inside the padded arrays; values outside the region are discarded).
template <typename R, bool MIX>
__device__ __forceinline__ void fused_b_edges(const DevCtx& c, const PatchDev& p, const Strides& S, const R* X,
                                              const Task& T, const int o[3], const int e[3], R* sE, int NE,
                                              const int ls[3], int level, int substep, double dt) {
  const int b0 = e[0] + 1, b1 = e[1] + 1, b2 = e[2] + 1;
  const int nbox = b0 * b1 * b2;
  const int nthr = blockDim.x;
  Walk3 w(threadIdx.x, nthr, b0, b1);
  for (int t = threadIdx.x; t < nbox; t += nthr, w.next()) {
    const int l[3] = {w.x, w.y, w.z};
    const int g[3] = {o[0] + w.x, o[1] + w.y, o[2] + w.z};
    bool node[3], cell[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      node[a] = g[a] < T.hi[a];
      cell[a] = l[a] < e[a] && g[a] < T.hi[a] - 1;
    }
    const bool own = l[0] < e[0] && l[1] < e[1] && l[2] < e[2];
    const long long q = g[0] + g[1] * S.s[1] + g[2] * S.s[2];
    const int lq = l[0] * ls[0] + l[1] * ls[1] + l[2] * ls[2];
    const R v0 = edge_value<0>(S, X, q);
    const R v1 = edge_value<1>(S, X, q);
    const R v2 = edge_value<2>(S, X, q);
    if (cell[0] && node[1] && node[2]) {
      sE[lq] = v0;
      if (own) edge_registers<0, R, MIX>(c, p, S, g[0], g[1], g[2], v0, level, substep, dt);
    }
    if (node[0] && cell[1] && node[2]) {
      sE[NE + lq] = v1;
      if (own) edge_registers<1, R, MIX>(c, p, S, g[0], g[1], g[2], v1, level, substep, dt);
    }
    if (node[0] && node[1] && cell[2]) {
      sE[2 * NE + lq] = v2;
      if (own) edge_registers<2, R, MIX>(c, p, S, g[0], g[1], g[2], v2, level, substep, dt);
    }
  }
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_fused_b(DevCtx c, int first, int n, int cur, int level, int substep,
                                                         int tx, int ty, int tz) {
  extern __shared__ double smem_d[];
  R* sE = reinterpret_cast<R*>(smem_d);
  const int nthr = blockDim.x;
  const int vb = xcd_block(blockIdx.x, gridDim.x);
  (void)n;
  const int t = task_of_block(c, first, vb);
  const Task& T = c.tasks[t];
  const int tile = vb - c.blk[t];
  const int ntx = (T.hi[0] - T.lo[0] + tx - 1) / tx, nty = (T.hi[1] - T.lo[1] + ty - 1) / ty;
  const int tix = tile % ntx, tiy = (tile / ntx) % nty, tiz = tile / (ntx * nty);
  const int o[3] = {T.lo[0] + tix * tx, T.lo[1] + tiy * ty, T.lo[2] + tiz * tz};
  const int e[3] = {min(tx, T.hi[0] - o[0]), min(ty, T.hi[1] - o[1]), min(tz, T.hi[2] - o[2])};
  const PatchDev& p = c.patches[T.patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  R* N = (R*)c.state + p.st[1 - cur];
  const R* X = (const R*)c.rscr + p.scr;
  const double dt = level_dt(c, level);
  const R dt_dx = R(dt / p.dx);
  const int ls[3] = {1, tx + 1, (tx + 1) * (ty + 1)};
  const int NE = ls[2] * (tz + 1);

  // 1. edge EMFs of the tile and its high-side layer
  fused_b_edges<R, MIX>(c, p, S, X, T, o, e, sE, NE, ls, level, substep, dt);
  __syncthreads();

  // 2. cells and low faces of the tile's entries
  const R* const ee[3] = {sE, sE + NE, sE + 2 * NE};
  const int CV = e[0] * e[1] * e[2];
  Walk3 w(threadIdx.x, nthr, e[0], e[1]);
  for (int k = threadIdx.x; k < CV; k += nthr, w.next()) {
    const int g[3] = {o[0] + w.x, o[1] + w.y, o[2] + w.z};
    const long long q = g[0] + g[1] * S.s[1] + g[2] * S.s[2];
    const bool ix = g[0] < T.hi[0] - 1, iy = g[1] < T.hi[1] - 1, iz = g[2] < T.hi[2] - 1;
    update_entry<R, int>(U, N, X, S, q, ix, iy, iz, dt_dx, ee, ls, w.x * ls[0] + w.y * ls[1] + w.z * ls[2]);
  }
}

// ---------------------------------------------------------------------------
// same-level ghost copy: one thread per copied entry; runs are consecutive
// along x so neighbouring lanes read and write neighbouring addresses
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void d_copy(const DevCtx& c, int vb, int nb, int first, int n, int blk_first, int nelem, int cur) {
  (void)nb;
  __shared__ int offs[AMRX_BLOCK + 1];
  // runs touched by this block: [r0, r1] (a run has >= 1 entry, so at most AMRX_BLOCK of them)
  const int r0 = c.run_blk[blk_first + vb];
  const int r1 = vb + 1 < nb ? c.run_blk[blk_first + vb + 1] : n - 1;
  const int nr = r1 - r0 + 1;
  for (int t = threadIdx.x; t < nr; t += AMRX_BLOCK) offs[t] = c.runs[first + r0 + t].off;
  __syncthreads();
  const int e = vb * AMRX_BLOCK + threadIdx.x;
  if (e >= nelem) return;
  int lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= e) lo = mid; else hi = mid - 1;
  }
  const Run& r = c.runs[first + r0 + lo];
  const int k = e - r.off;
  const PatchDev& dp = c.patches[r.dst_patch];
  const PatchDev& sp = c.patches[r.src_patch];
  R* dst = (R*)c.state + dp.st[cur];
  const R* src = (const R*)c.state + sp.st[cur];
  if (r.kind == 0) {
#pragma unroll
    for (int m = 0; m < 5; ++m) dst[m * dp.vol + r.dst_lin + k] = src[m * sp.vol + r.src_lin + k];
  } else {
    const int m = 4 + r.kind;
    dst[m * dp.vol + r.dst_lin + k] = src[m * sp.vol + r.src_lin + k];
  }
}

template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_copy(DevCtx c, int first, int n, int blk_first, int nelem, int cur) {
  d_copy<R>(c, blockIdx.x, gridDim.x, first, n, blk_first, nelem, cur);
}

// ---------------------------------------------------------------------------
// prolongation of one parent cell into a fine ghost region
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void d_prolong(const DevCtx& c, int vb, int nb, int first, int n, int cur_fine, int old_parent,
                                          int new_parent = 0, double w = 0.0) {
  (void)nb;
  const int id = vb * AMRX_BLOCK + threadIdx.x;
  if (id >= n) return;
  const Pro& pr = c.pros[first + id];
  const PatchDev& fp = c.patches[pr.patch];
  const PatchDev& mp = c.patches[fp.parent];
  const Strides FS = strides(fp), MS = strides(mp);
  const R* M = (const R*)c.state + mp.st[old_parent];
  const R* Mn = (const R*)c.state + mp.st[new_parent];
  R* F = (R*)c.state + fp.st[cur_fine];
  // parent value at offset o: the old buffer, or old + w (new - old) along the coarse time derivative
  const R wr = R(w);
  auto pv = [&](long long o) -> R {
    const R a = M[o];
    return w == 0.0 ? a : a + wr * (Mn[o] - a);
  };
  const long long P0 = pr.pidx;
  const long long f0 = 2LL * pr.c[0] + 2LL * pr.c[1] * FS.s[1] + 2LL * pr.c[2] * FS.s[2];
  // cells: conservative minmod-limited linear; child o = ox + 2 oy + 4 oz (written after the
  // positivity check at the end, which needs the children's faces)
  R cv[5][8], u0v[5];
  for (int m = 0; m < 5; ++m) {
    const long long u = m * MS.v;
    const R u0 = pv(u + P0);
    const R sx = minmod2(pv(u + P0 + MS.s[0]) - u0, u0 - pv(u + P0 - MS.s[0]));
    const R sy = minmod2(pv(u + P0 + MS.s[1]) - u0, u0 - pv(u + P0 - MS.s[1]));
    const R sz = minmod2(pv(u + P0 + MS.s[2]) - u0, u0 - pv(u + P0 - MS.s[2]));
    u0v[m] = u0;
    for (int o = 0; o < 8; ++o)
      cv[m][o] = u0 + R(0.25) * (R(2 * (o & 1) - 1) * sx + R(2 * ((o >> 1) & 1) - 1) * sy +
                                 R(2 * ((o >> 2) & 1) - 1) * sz);
  }
  // faces: outer[d][s][t2][t1] with (t1, t2) the offsets along the two other axes in increasing order
  R outer[3][2][2][2];
  for (int d = 0; d < 3; ++d) {
    int a1, a2;
    other_axes(d, a1, a2);
    const long long b = (5 + d) * MS.v;
    R* fb = F + (5 + d) * FS.v;
    for (int s = 0; s < 2; ++s) {
      const long long fbase = f0 + 2LL * s * FS.s[d];
      if (pr.flags & (1 << (2 * d + s))) {
        for (int t2 = 0; t2 < 2; ++t2)
          for (int t1 = 0; t1 < 2; ++t1) outer[d][s][t2][t1] = fb[fbase + t1 * FS.s[a1] + t2 * FS.s[a2]];
      } else {
        const long long pf = P0 + s * MS.s[d];
        const R bc = pv(b + pf);
        const R s1 = minmod2(pv(b + pf + MS.s[a1]) - bc, bc - pv(b + pf - MS.s[a1]));
        const R s2 = minmod2(pv(b + pf + MS.s[a2]) - bc, bc - pv(b + pf - MS.s[a2]));
        for (int t2 = 0; t2 < 2; ++t2)
          for (int t1 = 0; t1 < 2; ++t1) {
            const R val = bc + R(0.25) * (R(2 * t1 - 1) * s1 + R(2 * t2 - 1) * s2);
            outer[d][s][t2][t1] = val;
            fb[fbase + t1 * FS.s[a1] + t2 * FS.s[a2]] = val;
          }
      }
    }
  }
  // interior faces: mean of the aligned outer faces, then the least-norm divergence correction.
  // Cell (o0, o1, o2) divergence (times h) = sum_d [high_d - low_d].  With interior guesses g,
  // residual r = -div; phi = L^+ r for the cube graph Laplacian L (eigenvectors: Walsh functions
  // chi_S(o) = (-1)^(S.o) with eigenvalue 2|S|); correction of the interior face of axis d at
  // transverse offsets t: phi(o_d = 0, t) - phi(o_d = 1, t).
  R inner[3][2][2];
  for (int d = 0; d < 3; ++d)
    for (int t2 = 0; t2 < 2; ++t2)
      for (int t1 = 0; t1 < 2; ++t1) inner[d][t2][t1] = R(0.5) * (outer[d][0][t2][t1] + outer[d][1][t2][t1]);
  R res[8];
  for (int o = 0; o < 8; ++o) {
    const int oo[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
    R div = R(0);
    for (int d = 0; d < 3; ++d) {
      int a1, a2;
      other_axes(d, a1, a2);
      const int t1 = oo[a1], t2 = oo[a2];
      const R lowf = oo[d] == 0 ? outer[d][0][t2][t1] : inner[d][t2][t1];
      const R highf = oo[d] == 0 ? inner[d][t2][t1] : outer[d][1][t2][t1];
      div += highf - lowf;
    }
    res[o] = -div;
  }
  R phi[8];
  for (int o = 0; o < 8; ++o) phi[o] = R(0);
  for (int sm = 1; sm < 8; ++sm) {
    const int nbits = (sm & 1) + ((sm >> 1) & 1) + ((sm >> 2) & 1);
    R coef = R(0);
    for (int o = 0; o < 8; ++o) coef += (__popc(sm & o) & 1) ? -res[o] : res[o];
    coef *= R(1) / R(16 * nbits);  // (1/8) projection and 1/(2|S|)
    for (int o = 0; o < 8; ++o) phi[o] += (__popc(sm & o) & 1) ? -coef : coef;
  }
  for (int d = 0; d < 3; ++d) {
    int a1, a2;
    other_axes(d, a1, a2);
    R* fb = F + (5 + d) * FS.v;
    for (int t2 = 0; t2 < 2; ++t2)
      for (int t1 = 0; t1 < 2; ++t1) {
        int o_lo = (t1 << a1) | (t2 << a2);
        int o_hi = o_lo | (1 << d);
        const R val = inner[d][t2][t1] + (phi[o_lo] - phi[o_hi]);
        inner[d][t2][t1] = val;
        fb[f0 + FS.s[d] + t1 * FS.s[a1] + t2 * FS.s[a2]] = val;
      }
  }
  // positivity fallback: limiting rho, m and E separately does not keep the kinetic energy below
  // the total energy, so if any child has rho <= 0 or p <= 0 (its cell-centred field the mean of
  // its two faces per axis; decided in double in every precision) all 8 children take the coarse
  // cell's conserved values (first order, still conservative; the faces are kept)
  bool ok = true;
  const double gm1 = c.gamma - 1.0;
  for (int o = 0; o < 8; ++o) {
    const int oo[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
    double mag = 0.0;
    for (int d = 0; d < 3; ++d) {
      int a1, a2;
      other_axes(d, a1, a2);
      const int t1 = oo[a1], t2 = oo[a2];
      const double lowf = oo[d] == 0 ? (double)outer[d][0][t2][t1] : (double)inner[d][t2][t1];
      const double highf = oo[d] == 0 ? (double)inner[d][t2][t1] : (double)outer[d][1][t2][t1];
      const double bc = 0.5 * (lowf + highf);
      mag += bc * bc;
    }
    const double rho = cv[0][o];
    const double kin = 0.5 * ((double)cv[1][o] * cv[1][o] + (double)cv[2][o] * cv[2][o] + (double)cv[3][o] * cv[3][o]) / rho;
    // isothermal gas: p = cs2 rho, so the density and finite momenta decide
    const double prs = c.iso ? (isfinite(kin) ? c.cs2 * rho : -1.0) : gm1 * ((double)cv[4][o] - kin - 0.5 * mag);
    ok = ok && rho > 0.0 && prs > 0.0 && isfinite(prs);
  }
  for (int m = 0; m < 5; ++m)
    for (int o = 0; o < 8; ++o)
      F[m * FS.v + f0 + (o & 1) + ((o >> 1) & 1) * FS.s[1] + ((o >> 2) & 1) * FS.s[2]] = ok ? cv[m][o] : u0v[m];
}

template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_prolong(DevCtx c, int first, int n, int cur_fine, int old_parent,
                                                         int new_parent, double w) {
  d_prolong<R>(c, blockIdx.x, gridDim.x, first, n, cur_fine, old_parent, new_parent, w);
}

// ---------------------------------------------------------------------------
// restriction of a child onto its parent: node box of the child's coarse box
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void d_restrict(const DevCtx& c, int vb, int nb, int first, int n, int cur_fine, int cur_coarse) {
  (void)nb;
  Where w;
  if (!locate(c, first, n, vb, w)) return;
  const Task& T = c.tasks[w.task];
  const PatchDev& fp = c.patches[T.patch];
  const PatchDev& mp = c.patches[fp.parent];
  const Strides FS = strides(fp), MS = strides(mp);
  const R* F = (const R*)c.state + fp.st[cur_fine];
  R* M = (R*)c.state + mp.st[cur_coarse];
  const int I[3] = {w.i, w.j, w.k};
  const int nc[3] = {fp.n[0] / 2, fp.n[1] / 2, fp.n[2] / 2};
  long long pq = 0, fq = 0;
  for (int a = 0; a < 3; ++a) {
    pq += (long long)(fp.lo[a] / 2 - mp.lo[a] + AMRX_G + I[a]) * MS.s[a];
    fq += (long long)(AMRX_G + 2 * I[a]) * FS.s[a];
  }
  const bool in[3] = {I[0] < nc[0], I[1] < nc[1], I[2] < nc[2]};
  if (in[0] && in[1] && in[2]) {
    for (int m = 0; m < 5; ++m) {
      const R* u = F + m * FS.v;
      R s = R(0);
      for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
          for (int ox = 0; ox < 2; ++ox) s += u[fq + ox + oy * FS.s[1] + oz * FS.s[2]];
      M[m * MS.v + pq] = R(0.125) * s;
    }
  }
  for (int d = 0; d < 3; ++d) {
    int a1, a2;
    other_axes(d, a1, a2);
    if (!(in[a1] && in[a2])) continue;
    const R* b = F + (5 + d) * FS.v;
    R s = R(0);
    for (int t2 = 0; t2 < 2; ++t2)
      for (int t1 = 0; t1 < 2; ++t1) s += b[fq + t1 * FS.s[a1] + t2 * FS.s[a2]];
    M[(5 + d) * MS.v + pq] = R(0.25) * s;
  }
}

template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_restrict(DevCtx c, int first, int n, int cur_fine, int cur_coarse) {
  d_restrict<R>(c, xcd_block(blockIdx.x, gridDim.x), gridDim.x, first, n, cur_fine, cur_coarse);
}

// ---------------------------------------------------------------------------
// flux correction of an uncovered parent cell next to the fine region
// ---------------------------------------------------------------------------
template <typename R, bool MIX>
__device__ __forceinline__ void d_flux_corr(const DevCtx& c, int vb, int nb, int first, int n, int cur_coarse) {
  (void)nb;
  using Q = typename RegOf<R, MIX>::T;
  const int id = vb * AMRX_BLOCK + threadIdx.x;
  if (id >= n) return;
  const Corr& e = c.fcorrs[first + id];
  const PatchDev& mp = c.patches[e.patch];
  const Strides S = strides(mp);
  R* M = (R*)c.state + mp.st[cur_coarse];
  const int* cov = c.cov + mp.cov;
  const Q* regs = (const Q*)c.reg;
  const long long q = e.lin;
  const unsigned uq = (unsigned)e.lin, row = uq / (unsigned)mp.dim[0], kq = row / (unsigned)mp.dim[1];
  const int ijk[3] = {(int)(uq - row * (unsigned)mp.dim[0]), (int)(row - kq * (unsigned)mp.dim[1]), (int)kq};
  double corr[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    int a1, a2;
    other_axes(d, a1, a2);
    for (int sg = -1; sg <= 1; sg += 2) {
      const int ch = cov[q + sg * S.s[d]];
      if (ch < 0) continue;
      const PatchDev& cp = c.patches[ch];
      const int nc[3] = {cp.n[0] / 2, cp.n[1] / 2, cp.n[2] / 2};
      const int side = sg > 0 ? 0 : 1;
      int g[3];
      for (int a = 0; a < 3; ++a) g[a] = ijk[a] + mp.lo[a] - AMRX_G - cp.lo[a] / 2;
      const int t1 = g[a1], t2 = g[a2];
      const Q* acc = regs + cp.freg;
      const Q* lo = acc + cp.fsize;
      for (int m = 0; m < 5; ++m) {
        Q fine = Q(0);
        for (int u2 = 0; u2 < 2; ++u2)
          for (int u1 = 0; u1 < 2; ++u1)
            fine += reg_get<Q, MIX>(acc, lo, face_reg_index(cp.n, d, side, m, 2 * t1 + u1, 2 * t2 + u2));
        const Q coarse = regs[cp.creg + face_reg_index(nc, d, side, m, t1, t2)];
        const double delta = (double)(Q(0.25) * fine - coarse);
        corr[m] += sg > 0 ? -delta : delta;
      }
    }
  }
  for (int m = 0; m < 5; ++m) M[m * S.v + q] = (R)((double)M[m * S.v + q] + corr[m] / mp.dx);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flux_corr(DevCtx c, int first, int n, int cur_coarse) {
  d_flux_corr<R, MIX>(c, blockIdx.x, gridDim.x, first, n, cur_coarse);
}

// EMF change (new - old, times dt) at a parent edge along e at node q, zero off the coverage boundary
template <typename R, bool MIX>
__device__ double emf_delta(const DevCtx& c, const PatchDev& mp, const Strides& S, const int* cov, int e,
                            const int ijk[3]) {
  using Q = typename RegOf<R, MIX>::T;
  const int A = (e + 1) % 3, C = (e + 2) % 3;
  const long long q = ijk[0] + ijk[1] * S.s[1] + ijk[2] * S.s[2];
  const int nb[4] = {cov[q - S.s[A] - S.s[C]], cov[q - S.s[C]], cov[q - S.s[A]], cov[q]};
  const bool any = nb[0] >= 0 || nb[1] >= 0 || nb[2] >= 0 || nb[3] >= 0;
  const bool all = nb[0] >= 0 && nb[1] >= 0 && nb[2] >= 0 && nb[3] >= 0;
  if (!any || all) return 0.0;
  const int owner = nb[0] >= 0 ? nb[0] : (nb[1] >= 0 ? nb[1] : (nb[2] >= 0 ? nb[2] : nb[3]));
  const PatchDev& cp = c.patches[owner];
  const int nc[3] = {cp.n[0] / 2, cp.n[1] / 2, cp.n[2] / 2};
  int g[3];
  for (int a = 0; a < 3; ++a) g[a] = ijk[a] + mp.lo[a] - AMRX_G - cp.lo[a] / 2;
  const Q* regs = (const Q*)c.reg;
  const Q* acc = regs + cp.ereg;
  const Q* lo = acc + cp.esize;
  Q enew, eold;
  if (g[A] == 0 || g[A] == nc[A]) {
    const int s = g[A] == 0 ? 0 : 1;
    eold = regs[cp.cereg + edge_reg_pa(nc, e, s, g[C], g[e])];
    enew = Q(0.5) * (reg_get<Q, MIX>(acc, lo, edge_reg_pa(cp.n, e, s, 2 * g[C], 2 * g[e])) +
                     reg_get<Q, MIX>(acc, lo, edge_reg_pa(cp.n, e, s, 2 * g[C], 2 * g[e] + 1)));
  } else {
    const int s = g[C] == 0 ? 0 : 1;
    eold = regs[cp.cereg + edge_reg_pb(nc, e, s, g[A], g[e])];
    enew = Q(0.5) * (reg_get<Q, MIX>(acc, lo, edge_reg_pb(cp.n, e, s, 2 * g[A], 2 * g[e])) +
                     reg_get<Q, MIX>(acc, lo, edge_reg_pb(cp.n, e, s, 2 * g[A], 2 * g[e] + 1)));
  }
  return (double)(enew - eold);
}

template <typename R, bool MIX>
__device__ __forceinline__ void d_emf_corr(const DevCtx& c, int vb, int nb, int first, int n, int cur_coarse) {
  (void)nb;
  const int id = vb * AMRX_BLOCK + threadIdx.x;
  if (id >= n) return;
  const Corr& e = c.ecorrs[first + id];
  const PatchDev& mp = c.patches[e.patch];
  const Strides S = strides(mp);
  R* M = (R*)c.state + mp.st[cur_coarse];
  const int* cov = c.cov + mp.cov;
  const long long q = e.lin;
  const int d = e.axis;
  const int A = (d + 1) % 3, C = (d + 2) % 3;
  const unsigned uq = (unsigned)e.lin, row = uq / (unsigned)mp.dim[0], kq = row / (unsigned)mp.dim[1];
  const int ijk[3] = {(int)(uq - row * (unsigned)mp.dim[0]), (int)(row - kq * (unsigned)mp.dim[1]), (int)kq};
  int nA[3] = {ijk[0], ijk[1], ijk[2]};
  nA[A] += 1;
  int nC[3] = {ijk[0], ijk[1], ijk[2]};
  nC[C] += 1;
  const double curl = (emf_delta<R, MIX>(c, mp, S, cov, C, nA) - emf_delta<R, MIX>(c, mp, S, cov, C, ijk)) -
                      (emf_delta<R, MIX>(c, mp, S, cov, A, nC) - emf_delta<R, MIX>(c, mp, S, cov, A, ijk));
  R* b = M + (5 + d) * S.v;
  b[q] = (R)((double)b[q] - curl / mp.dx);
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_emf_corr(DevCtx c, int first, int n, int cur_coarse) {
  d_emf_corr<R, MIX>(c, blockIdx.x, gridDim.x, first, n, cur_coarse);
}

// Restriction of a fine level and both corrections of its parents in one launch: they write
// disjoint data (covered cells and closure faces; uncovered cells next to the coverage
// boundary; uncovered faces around its edges) and read only fine data and registers.
template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_restrict_corr(DevCtx c, int rfirst, int rn, int rnblk, int ffirst,
                                                               int fn, int efirst, int en, int cur_fine,
                                                               int cur_coarse) {
  const int b = blockIdx.x;
  const int fnblk = (fn + AMRX_BLOCK - 1) / AMRX_BLOCK;
  if (b < rnblk) {
    d_restrict<R>(c, b, rnblk, rfirst, rn, cur_fine, cur_coarse);
  } else if (b < rnblk + fnblk) {
    d_flux_corr<R, MIX>(c, b - rnblk, fnblk, ffirst, fn, cur_coarse);
  } else {
    d_emf_corr<R, MIX>(c, b - rnblk - fnblk, (en + AMRX_BLOCK - 1) / AMRX_BLOCK, efirst, en, cur_coarse);
  }
}

// ---------------------------------------------------------------------------
// same-level synchronisation of shared boundary faces
// ---------------------------------------------------------------------------
template <typename R, bool MIX>
__device__ __forceinline__ void d_sync(const DevCtx& c, int vb, int nb, int first, int n, int cur) {
  (void)nb;
  using Q = typename RegOf<R, MIX>::T;
  const int id = vb * AMRX_BLOCK + threadIdx.x;
  if (id >= n) return;
  const SyncPair& s = c.syncs[first + id];
  const PatchDev& pa = c.patches[s.a];
  const PatchDev& pb = c.patches[s.b];
  const Q* regs = (const Q*)c.reg;
  const Q* la = regs + pa.freg + 2 * pa.fsize;
  const Q* lb = regs + pb.freg + 2 * pb.fsize;
  double worst = 0.0;
  double delta[5];
  // component m of a face register sits m * (n_a2 * n_a1) entries after component 0
  int a1, a2;
  other_axes(s.axis, a1, a2);
  const long long stride_a = (long long)pa.n[a1] * pa.n[a2];
  const long long stride_b = (long long)pb.n[a1] * pb.n[a2];
  for (int m = 0; m < 5; ++m) {
    const double fa = la[s.a_reg + m * stride_a], fb = lb[s.b_reg + m * stride_b];
    delta[m] = 0.5 * (fb - fa);
    worst = fmax(worst, fabs(fb - fa));
  }
  if (!(worst == 0.0)) atomic_max_pos(&c.slots[SLOT_SYNC_F], worst);
  const R* Ua = (const R*)c.state + pa.st[cur];
  const R* Ub = (const R*)c.state + pb.st[cur];
  const double bd = fabs((double)Ua[(5 + s.axis) * pa.vol + s.a_face] - (double)Ub[(5 + s.axis) * pb.vol + s.b_face]);
  if (!(bd == 0.0)) atomic_max_pos(&c.slots[SLOT_SYNC_B], bd);
  if (worst > 0.0) {
    R* U = (R*)c.state + pa.st[cur];
    for (int m = 0; m < 5; ++m) {
      const double v = (s.a_side == 0 ? delta[m] : -delta[m]) / pa.dx;
      atomicAdd(&U[m * pa.vol + s.a_cell], (R)v);
    }
  }
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_sync(DevCtx c, int first, int n, int cur) {
  d_sync<R, MIX>(c, blockIdx.x, gridDim.x, first, n, cur);
}

// ---------------------------------------------------------------------------
// CFL signal speed: max over interior cells of sum_d (|v_d| + c_f,d) / dx
// ---------------------------------------------------------------------------
// Grid-stride over the list's blocks; one atomic per block on the level's slot.
template <typename R, bool MIX>
// Largest signal-speed sum over the cells of the blocks b0, b0 + stride, ... of a level's CFL list:
// the block maximum goes to out[b0] when out is given (reduced by a later kernel, no atomics),
// else into the level's slot with one atomic per block.
__device__ __forceinline__ void d_cfl(const DevCtx& c, int b0, int stride, int first, int n, int nblk, int cur, int level,
                                      double* out = nullptr) {
  __shared__ double red[AMRX_BLOCK / 64];
  double s = 0.0;
  (void)n;
  for (int b = b0; b < nblk; b += stride) {
    const int t = task_of_block(c, first, b);
    const Task& T = c.tasks[t];
    const unsigned ex = T.hi[0] - T.lo[0], ey = T.hi[1] - T.lo[1], ez = T.hi[2] - T.lo[2];
    const unsigned local = (unsigned)(b - c.blk[t]) * AMRX_BLOCK + threadIdx.x;
    if (local >= ex * ey * ez) continue;
    unsigned row, kk;
    int i, j;
    split_index(local, ex, T.inv0, row, i);
    split_index(row, ey, T.inv1, kk, j);
    i += T.lo[0];
    j += T.lo[1];
    const int k = T.lo[2] + (int)kk;
    const PatchDev& p = c.patches[T.patch];
    const Strides S = strides(p);
    const R* U = (const R*)c.state + p.st[cur];
    const long long q = i + j * S.s[1] + k * S.s[2];
    const long long v = S.v;
    const R gamma = R(c.gamma);
    const R rho = U[q];
    const R bx = R(0.5) * (U[5 * v + q] + U[5 * v + q + 1]);
    const R by = R(0.5) * (U[6 * v + q] + U[6 * v + q + S.s[1]]);
    const R bz = R(0.5) * (U[7 * v + q] + U[7 * v + q + S.s[2]]);
    const R pr = c.iso ? R(c.cs2) * rho
                       : pressure<R, MIX>(rho, U[v + q], U[2 * v + q], U[3 * v + q], U[4 * v + q], bx, by, bz, gamma - R(1));
    const R b2 = bx * bx + by * by + bz * bz;
    const R vx = qdiv(U[v + q], rho), vy = qdiv(U[2 * v + q], rho), vz = qdiv(U[3 * v + q], rho);
    const R inv = R(1.0 / p.dx);
    R tot;
    if (c.iso) {
      const R cs = R(sqrt(c.cs2));
      tot = (fabs(vx) + cs) * inv + (fabs(vy) + cs) * inv + (fabs(vz) + cs) * inv;
    } else {
      tot = (fabs(vx) + fast_speed(rho, pr, b2, bx * bx, gamma)) * inv +
            (fabs(vy) + fast_speed(rho, pr, b2, by * by, gamma)) * inv +
            (fabs(vz) + fast_speed(rho, pr, b2, bz * bz, gamma)) * inv;
    }
    double sv = (double)tot;
    if (!(rho > R(0)) || !(pr > R(0)) || !isfinite(sv)) flag_phys(c.slots);
    if (!isfinite(sv)) sv = 1.0e308;
    s = fmax(s, sv);
  }
  for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < AMRX_BLOCK / 64; ++w) m = fmax(m, red[w]);
    if (out) out[b0] = m;
    else if (m > 0.0) atomic_max_pos(&c.slots[SLOT_SMAX + level], m);
  }
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_cfl(DevCtx c, int first, int n, int nblk, int cur, int level) {
  d_cfl<R, MIX>(c, blockIdx.x, gridDim.x, first, n, nblk, cur, level);
}

// All levels' CFL reductions in one launch: block ranges [grid0[l], grid0[l + 1]) serve level l.
template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_cfl_all(DevCtx c, CflLevels L) {
  int l = 0;
  while (l + 1 < L.nlev && L.grid0[l + 1] <= (int)blockIdx.x) ++l;
  const int stride = L.grid0[l + 1] - L.grid0[l];
  d_cfl<R, MIX>(c, blockIdx.x - L.grid0[l], stride, L.first[l], L.n[l], L.nblk[l], L.cur[l], l,
                c.partials + L.grid0[l]);
}

// dt0 = min over levels of 2^l C / (largest signal-speed sum of level l), from the per-block
// maxima the CFL launch left in the partials; also records each level's maximum in its slot.
__global__ __launch_bounds__(AMRX_BLOCK) void k_dt_from_partials(DevCtx c, CflLevels L, double cfl) {
  __shared__ double red[AMRX_BLOCK / 64];
  double best = 1e300;
  for (int l = 0; l < L.nlev; ++l) {
    double m = 0.0;
    for (int i = L.grid0[l] + threadIdx.x; i < L.grid0[l + 1]; i += AMRX_BLOCK) m = fmax(m, c.partials[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int w = 1; w < AMRX_BLOCK / 64; ++w) mm = fmax(mm, red[w]);
      c.slots[SLOT_SMAX + l] = (unsigned long long)__double_as_longlong(mm);
      if (mm > 0.0) best = fmin(best, ldexp(cfl, l) / mm);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) c.slots[SLOT_DT] = (unsigned long long)__double_as_longlong(best);
}

// ---------------------------------------------------------------------------
// conservation sums over leaf cells with compensated (two-sum) accumulation
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

struct Curs {
  int c[AMRX_MAXLEV];
};

template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_cons(DevCtx c, int first, int n, Curs curs) {
  __shared__ double sh_s[8][AMRX_BLOCK];
  __shared__ double sh_e[8][AMRX_BLOCK];
  Where w;
  double x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (locate(c, first, n, blockIdx.x, w)) {
    const PatchDev& p = c.patches[c.tasks[w.task].patch];
    const Strides S = strides(p);
    const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
    const bool leaf = !p.has_children || c.cov[p.cov + q] < 0;
    if (leaf) {
      const R* U = (const R*)c.state + p.st[curs.c[p.level]];
      const long long v = S.v;
      const double dv = p.dx * p.dx * p.dx;
      for (int m = 0; m < 5; ++m) x[m] = (double)U[m * v + q] * dv;
      x[5] = (double)(R(0.5) * (U[5 * v + q] + U[5 * v + q + 1])) * dv;
      x[6] = (double)(R(0.5) * (U[6 * v + q] + U[6 * v + q + S.s[1]])) * dv;
      x[7] = (double)(R(0.5) * (U[7 * v + q] + U[7 * v + q + S.s[2]])) * dv;
    }
  }
  for (int m = 0; m < 8; ++m) {
    sh_s[m][threadIdx.x] = x[m];
    sh_e[m][threadIdx.x] = 0.0;
  }
  __syncthreads();
  for (int half = AMRX_BLOCK / 2; half > 0; half >>= 1) {
    if (threadIdx.x < half) {
      for (int m = 0; m < 8; ++m) {
        double s, e;
        two_sum(sh_s[m][threadIdx.x], sh_s[m][threadIdx.x + half], s, e);
        sh_s[m][threadIdx.x] = s;
        sh_e[m][threadIdx.x] += sh_e[m][threadIdx.x + half] + e;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) {
    c.partials[(long long)blockIdx.x * 16 + threadIdx.x] = sh_s[threadIdx.x][0];
    c.partials[(long long)blockIdx.x * 16 + 8 + threadIdx.x] = sh_e[threadIdx.x][0];
  }
}

__global__ __launch_bounds__(AMRX_BLOCK) void k_cons_final(DevCtx c, int nblk) {
  __shared__ double sh_s[8][AMRX_BLOCK];
  __shared__ double sh_e[8][AMRX_BLOCK];
  double s[8], e[8];
  for (int m = 0; m < 8; ++m) {
    s[m] = 0.0;
    e[m] = 0.0;
  }
  for (int b = threadIdx.x; b < nblk; b += AMRX_BLOCK) {
    for (int m = 0; m < 8; ++m) {
      double t, err;
      two_sum(s[m], c.partials[(long long)b * 16 + m], t, err);
      s[m] = t;
      e[m] += err + c.partials[(long long)b * 16 + 8 + m];
    }
  }
  for (int m = 0; m < 8; ++m) {
    sh_s[m][threadIdx.x] = s[m];
    sh_e[m][threadIdx.x] = e[m];
  }
  __syncthreads();
  for (int half = AMRX_BLOCK / 2; half > 0; half >>= 1) {
    if (threadIdx.x < half) {
      for (int m = 0; m < 8; ++m) {
        double t, err;
        two_sum(sh_s[m][threadIdx.x], sh_s[m][threadIdx.x + half], t, err);
        sh_s[m][threadIdx.x] = t;
        sh_e[m][threadIdx.x] += sh_e[m][threadIdx.x + half] + err;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) {
    double t, err;
    two_sum(sh_s[threadIdx.x][0], sh_e[threadIdx.x][0], t, err);
    c.partials[(long long)nblk * 16 + threadIdx.x] = t;
    c.partials[(long long)nblk * 16 + 8 + threadIdx.x] = err;
  }
}

__global__ void k_clear_slots(DevCtx c) {
  const int t = threadIdx.x;
  if (t < NSLOT) c.slots[t] = 0ULL;
}

__global__ void k_clear_acc(DevCtx c) {
  const int t = threadIdx.x;
  if (t < NSLOT_ALL - NSLOT) c.slots[NSLOT + t] = 0ULL;
}

// after a root step: latch its unphysical-state flag, add its dt to the time advanced, count it
__global__ void k_step_acc(DevCtx c) {
  if (threadIdx.x == 0) {
    unsigned long long* s = c.slots;
    s[ACC_PHYS] |= s[SLOT_PHYS];
    const double t = __longlong_as_double((long long)s[ACC_TIME]) + __longlong_as_double((long long)s[SLOT_DT]);
    s[ACC_TIME] = (unsigned long long)__double_as_longlong(t);
    s[ACC_STEPS] += 1ULL;
  }
}

__global__ void k_set_dt(DevCtx c, double dt0) {
  if (threadIdx.x == 0) c.slots[SLOT_DT] = (unsigned long long)__double_as_longlong(dt0);
}

// dt0 = min over levels of 2^l * cfl / (max signal speed sum of level l)
__global__ void k_dt_from_cfl(DevCtx c, int nlev, double cfl) {
  if (threadIdx.x != 0) return;
  double best = 1e300;
  for (int l = 0; l < nlev; ++l) {
    const double smax = __longlong_as_double((long long)c.slots[SLOT_SMAX + l]);
    if (smax > 0.0) best = fmin(best, ldexp(cfl, l) / smax);
  }
  c.slots[SLOT_DT] = (unsigned long long)__double_as_longlong(best);
}

__device__ __forceinline__ void dt_from_cfl(const DevCtx& c, int nlev, double cfl) {
  double best = 1e300;
  for (int l = 0; l < nlev; ++l) {
    const double smax = __longlong_as_double((long long)c.slots[SLOT_SMAX + l]);
    if (smax > 0.0) best = fmin(best, ldexp(cfl, l) / smax);
  }
  c.slots[SLOT_DT] = (unsigned long long)__double_as_longlong(best);
}

// ---------------------------------------------------------------------------
// persistent fine-first scheduler
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool node_ready(const Sched& sc, const Node& nd) {
  for (int k = 0; k < nd.npred; ++k) {
    const int p = sc.preds[nd.pred_first + k];
    // relaxed (coherent, no cache invalidation); the claimer acquires once after a successful claim
    if (__hip_atomic_load(&sc.done[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < sc.nodes[p].nblk) return false;
  }
  return true;
}

// Claim the first ready item of the finest queue that has one.  Non-blocking: a
// workgroup never holds an item while waiting, so progress needs no co-residency.
// Returns -1 once every queue is exhausted, or after ~10 s without any ready item
// (then SLOT_SCHED is raised so the host reports the failure).  Idle polling
// sleeps ~3 us between rounds and touches only coherent counters.
__device__ int claim_item(const Sched& sc, unsigned long long* slots) {
  const unsigned long long t0 = wall_clock64();
  for (unsigned spin = 0;; ++spin) {
    bool pending = false;
    for (int q = sc.nq - 1; q >= 0; --q) {
      const Queue Q = sc.queues[q];
      int h = __hip_atomic_load(&sc.heads[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (h < Q.len) {
        pending = true;
        const Item& it = sc.items[Q.first + h];
        if (!node_ready(sc, sc.nodes[it.node])) break;
        int expected = h;
        if (__hip_atomic_compare_exchange_strong(&sc.heads[q], &expected, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
          return Q.first + h;
        h = expected;
      }
    }
    if (!pending) return -1;
    // wall_clock64 ticks at 100 MHz; the iteration cap (>= 3 us per round) bounds the wait even without a clock
    if (wall_clock64() - t0 > 1000000000ULL || spin > 4000000u) {
      atomicOr(&slots[SLOT_SCHED], 1ULL);
      return -1;
    }
    __builtin_amdgcn_s_sleep(127);
  }
}

template <typename R, bool MIX>
__device__ __forceinline__ void run_node(const DevCtx& c, const Node& nd, int b, int nlev, double cfl) {
  switch (nd.op) {
    case OP_CFL: d_cfl<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.nblk, nd.cur, nd.level); break;
    case OP_DT:
      if (threadIdx.x == 0) dt_from_cfl(c, nlev, cfl);
      break;
    case OP_COPY: d_copy<R>(c, b, nd.nblk, nd.first, nd.n, nd.blk_first, nd.nelem, nd.cur); break;
    case OP_PROLONG: d_prolong<R>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.aux); break;
    case OP_PRIM: d_prim<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur); break;
    case OP_BHALF: d_bhalf<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.level); break;
    case OP_PRED: d_pred<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.level); break;
    case OP_FLUX: d_flux_any<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.level, nd.substep); break;
    case OP_EDGE: d_edge<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.level, nd.substep); break;
    case OP_UPDATE: d_update<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.level); break;
    case OP_RESTRICT: d_restrict<R>(c, b, nd.nblk, nd.first, nd.n, nd.cur, nd.aux); break;
    case OP_FCORR: d_flux_corr<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.aux); break;
    case OP_ECORR: d_emf_corr<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.aux); break;
    case OP_SYNC: d_sync<R, MIX>(c, b, nd.nblk, nd.first, nd.n, nd.cur); break;
    default: break;
  }
}

template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_persistent(DevCtx c, Sched sc, int nlev, double cfl) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) {
      const int got = claim_item(sc, c.slots);
      // acquire once per claimed item: the data of its completed predecessors; the
      // barrier below orders the other waves of this workgroup after it
      if (got >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_item = got;
    }
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it < 0) return;
    const Item I = sc.items[it];
    const Node nd = sc.nodes[I.node];
    for (int b = I.b0; b < I.b1; ++b) {
      run_node<R, MIX>(c, nd, b, nlev, cfl);
      __syncthreads();  // every wave's stores of this workgroup are done (workgroup scope)
    }
    // release by one thread: the workgroup's writes become visible device-wide before the count
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&sc.done[I.node], I.b1 - I.b0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// regridding: refinement flags of a level's interior cells, and element runs
// copied between the state arenas of two hierarchies
// ---------------------------------------------------------------------------
// flag of an interior cell: the density jump to a face neighbour inside the patch exceeds
// eps times the smaller density, evaluated in the state's precision; one byte per padded cell
// at (first state offset of the patch) / 16 + padded index
template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_flag(DevCtx c, int first, int n, int cur, double eps,
                                                      unsigned char* flags) {
  Where w;
  if (!locate(c, first, n, xcd_block(blockIdx.x, gridDim.x), w)) return;
  const PatchDev& p = c.patches[c.tasks[w.task].patch];
  const Strides S = strides(p);
  const R* U = (const R*)c.state + p.st[cur];
  const long long q = w.i + w.j * S.s[1] + w.k * S.s[2];
  const R e = R(eps);
  const R rc = U[q];
  const int g[3] = {w.i, w.j, w.k};
  bool f = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (g[d] > AMRX_G) {
      const R rn = U[q - S.s[d]];
      f = f || fabs(rn - rc) > e * fmin(rn, rc);
    }
    if (g[d] < AMRX_G + p.n[d] - 1) {
      const R rn = U[q + S.s[d]];
      f = f || fabs(rn - rc) > e * fmin(rn, rc);
    }
  }
  flags[p.st[0] / 16 + q] = f ? 1 : 0;
}

// one thread per element of a list of runs (src offset, dst offset, length; offsets in reals
// of the two arenas); off[r] = first element of run r (prefix), r found by binary search
template <typename R>
__global__ __launch_bounds__(AMRX_BLOCK) void k_xcopy(const R* src, R* dst, const XRun* runs, int nrun, long long nelem) {
  const long long e = (long long)blockIdx.x * AMRX_BLOCK + threadIdx.x;
  if (e >= nelem) return;
  int lo = 0, hi = nrun - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (runs[mid].off <= e) lo = mid; else hi = mid - 1;
  }
  const XRun& r = runs[lo];
  const long long k = e - r.off;
  dst[r.dst + k] = src[r.src + k];
}

// ---------------------------------------------------------------------------
// layered fine-first schedule: the dependency graph of one root step cut into
// layers of mutually independent batched launches (a node's layer is one more
// than its latest predecessor's).  One launch per layer with a persistent grid;
// workgroups claim the layer's items (block ranges of its nodes, finer levels'
// items first) from an atomic counter and leave once it passes the end: no
// workgroup ever waits for another, so every launch drains.
// ---------------------------------------------------------------------------
template <typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_layer(DevCtx c, const Node* nodes, const Item* items, int first, int n,
                                                       int* counter, int nlev, double cfl) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    // the claimed index is the same in every lane: keep it (and all node parameters derived from it)
    // in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n) return;
    const Item I = items[first + it];
    const Node nd = nodes[I.node];
    for (int b = I.b0; b < I.b1; ++b) {
      run_node<R, MIX>(c, nd, b, nlev, cfl);
      __syncthreads();
    }
  }
}

__global__ void k_clear_ints(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// paired launches: two independent batched launches (one level's advance stage
// and the next finer level's ghost fill or advance stage of its first substep,
// which reads only the coarse level's pre-advance buffer) in one grid, so that
// their blocks share the GPU (e.g. arithmetic-bound fluxes beside
// memory-bound stages).  Block ranges [0, pa) and [pa, pa + pb) serve a and b.
// ---------------------------------------------------------------------------
template <int OP, typename R, bool MIX>
__device__ __forceinline__ void run_op(const DevCtx& c, const Node& nd, int vb) {
  if constexpr (OP == OP_COPY) d_copy<R>(c, vb, nd.nblk, nd.first, nd.n, nd.blk_first, nd.nelem, nd.cur);
  else if constexpr (OP == OP_PROLONG) d_prolong<R>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.aux);
  else if constexpr (OP == OP_PRIM) d_prim<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur);
  else if constexpr (OP == OP_BHALF) d_bhalf<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.level);
  else if constexpr (OP == OP_PRED) d_pred<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.level);
  else if constexpr (OP == OP_FLUX) d_flux_any<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.level, nd.substep);
  else if constexpr (OP == OP_EDGE) d_edge<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.level, nd.substep);
  else if constexpr (OP == OP_UPDATE) d_update<R, MIX>(c, vb, nd.nblk, nd.first, nd.n, nd.cur, nd.level);
}

template <int OP>
__device__ __forceinline__ int pair_block(int local, int padded) {
  // ghost copies and prolongation index their lists directly; stage kernels use the XCD remap
  return (OP == OP_COPY || OP == OP_PROLONG) ? local : xcd_block(local, padded);
}

template <int OA, int OB, typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_pair(DevCtx c, Node a, Node b, int pa, int pb) {
  // groups of 8 consecutive blocks (one per XCD) alternate between a and b in proportion to
  // their sizes, so both run side by side through the whole launch; a block keeps its XCD
  const long long ga = pa >> 3, gt = (pa + pb) >> 3;
  const long long g = blockIdx.x >> 3;
  const int lane = blockIdx.x & 7;
  const long long ka = g * ga / gt, ka1 = (g + 1) * ga / gt;  // a-groups before group g, and through it
  if (ka1 > ka) {
    const int vb = pair_block<OA>((int)(ka * 8 + lane), pa);
    if (vb < a.nblk) run_op<OA, R, MIX>(c, a, vb);
  } else {
    const int vb = pair_block<OB>((int)((g - ka) * 8 + lane), pb);
    if (vb < b.nblk) run_op<OB, R, MIX>(c, b, vb);
  }
}

// A layer whose launches all run one stage or ghost-fill operation: the same claim loop with only
// that operation's code (the register footprint of the generic kernel covers every operation).
template <int OP, typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_layer_op(DevCtx c, const Node* nodes, const Item* items, int first,
                                                          int n, int* counter) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n) return;
    const Item I = items[first + it];
    const Node nd = nodes[I.node];
    for (int b = I.b0; b < I.b1; ++b) {
      run_op<OP, R, MIX>(c, nd, b);
      // only the ghost copy shares LDS between the threads of a block
      if (OP == OP_COPY) __syncthreads();
    }
  }
}

// A layer whose launches run two stage or ghost-fill operations (typically a coarse level's stage
// beside a finer level's next one): the claim loop with only those two operations' code.
template <int OA, int OB, typename R, bool MIX>
__global__ __launch_bounds__(AMRX_BLOCK) void k_layer2(DevCtx c, const Node* nodes, const Item* items, int first, int n,
                                                        int* counter) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n) return;
    const Item I = items[first + it];
    const Node nd = nodes[I.node];
    for (int b = I.b0; b < I.b1; ++b) {
      if (nd.op == OA) run_op<OA, R, MIX>(c, nd, b);
      else run_op<OB, R, MIX>(c, nd, b);
      if (OA == OP_COPY || OB == OP_COPY) __syncthreads();
    }
  }
}

template <int OA, int OB>
hipError_t launch_layer2_t(const DevCtx& c, const Node* nodes, const Item* items, int first, int n, int* counter, int g) {
  if (c.precision == 0) k_layer2<OA, OB, double, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  else if (c.precision == 1) k_layer2<OA, OB, float, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  else k_layer2<OA, OB, float, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  return hipGetLastError();
}

// operation pairs with a specialised layer kernel, as (lower op, higher op)
#define LAYER2_CASES(X)                                                                               \
  X(OP_PRIM, OP_BHALF) X(OP_BHALF, OP_PRED) X(OP_PRED, OP_FLUX) X(OP_FLUX, OP_EDGE) X(OP_EDGE, OP_UPDATE) \
  X(OP_COPY, OP_PROLONG) X(OP_COPY, OP_PRIM) X(OP_PROLONG, OP_PRIM)

template <int OP>
hipError_t launch_layer_op_t(const DevCtx& c, const Node* nodes, const Item* items, int first, int n, int* counter,
                             int g) {
  if (c.precision == 0) k_layer_op<OP, double, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  else if (c.precision == 1) k_layer_op<OP, float, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  else k_layer_op<OP, float, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter);
  return hipGetLastError();
}

__global__ void k_clear_sched(Sched sc, int nnodes) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nnodes; i += gridDim.x * blockDim.x) sc.done[i] = 0;
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < sc.nq; q += blockDim.x) sc.heads[q] = 0;
}

inline unsigned grid_of(long long n, int per) { return (unsigned)((n + per - 1) / per); }


#define DISPATCH(KERNEL, GRID, ...)                                                              \
  do {                                                                                           \
    if (c.precision == 0) KERNEL<double, false><<<GRID, AMRX_BLOCK, 0, c.stream>>>(__VA_ARGS__); \
    else if (c.precision == 1) KERNEL<float, false><<<GRID, AMRX_BLOCK, 0, c.stream>>>(__VA_ARGS__); \
    else KERNEL<float, true><<<GRID, AMRX_BLOCK, 0, c.stream>>>(__VA_ARGS__);                    \
  } while (0)

#define DISPATCH_R(KERNEL, GRID, ...)                                                     \
  do {                                                                                    \
    if (c.precision == 0) KERNEL<double><<<GRID, AMRX_BLOCK, 0, c.stream>>>(__VA_ARGS__); \
    else KERNEL<float><<<GRID, AMRX_BLOCK, 0, c.stream>>>(__VA_ARGS__);                   \
  } while (0)

}  // namespace

hipError_t launch_stage(const DevCtx& c, int stage, int task_first, int ntask, int blk_first, int nblk, int cur,
                        int level, int substep) {
  (void)blk_first;
  if (ntask == 0 || nblk == 0) return hipSuccess;
  const dim3 g(nblk);
  switch (stage) {
    case STAGE_PRIM: DISPATCH(k_prim, g, c, task_first, ntask, cur); break;
    case STAGE_BHALF: DISPATCH(k_bhalf, g, c, task_first, ntask, cur, level); break;
    case STAGE_PRED: DISPATCH(k_pred, g, c, task_first, ntask, cur, level); break;
    case STAGE_FLUX:
      if (c.iso) {
        DISPATCH(k_flux_iso, g, c, task_first, ntask, cur, level, substep);
      } else {
        return launch_flux(c, task_first, ntask, nblk, cur, level, substep, true);
      }
      break;
    case STAGE_EDGE: DISPATCH(k_edge, g, c, task_first, ntask, cur, level, substep); break;
    case STAGE_UPDATE: DISPATCH(k_update, g, c, task_first, ntask, cur, level); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_update(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, bool nt) {
  if (ntask == 0 || nblk == 0) return hipSuccess;
  const dim3 g(nblk);
  if (!nt) DISPATCH(k_update, g, c, task_first, ntask, cur, level);
  else if (c.precision == 0) k_update<double, false, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, task_first, ntask, cur, level);
  else if (c.precision == 1) k_update<float, false, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, task_first, ntask, cur, level);
  else k_update<float, true, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, task_first, ntask, cur, level);
  return hipGetLastError();
}

hipError_t launch_flux(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int substep,
                       bool split) {
  if (ntask == 0 || nblk == 0) return hipSuccess;
  const dim3 g(nblk);
  if (c.iso) {
    DISPATCH(k_flux_iso, g, c, task_first, ntask, cur, level, substep);
  } else if (c.precision == 2 && !split) {
    k_flux_mixed_one_pass<float><<<g, AMRX_BLOCK, 0, c.stream>>>(c, task_first, ntask, cur, level, substep);
  } else {
    if (c.precision == 2) {
      const hipError_t e = launch_clear_ints(c, c.lbflag, 1);  // the list of waves pass 1 appends to
      if (e != hipSuccess) return e;
    }
    DISPATCH(k_flux, g, c, task_first, ntask, cur, level, substep);
    if (c.precision == 2) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      k_flux_low_beta<float><<<dim3(std::min(nblk, 1024)), AMRX_BLOCK, 0, c.stream>>>(c, task_first, ntask, level,
                                                                                     substep);
    }
  }
  return hipGetLastError();
}

int fused_a_threads(int tx, int ty, int tz) { return tx * ty * tz <= 128 ? 128 : AMRX_BLOCK; }

size_t fused_a_lds_bytes(int precision, int tx, int ty, int tz) {
  const size_t hv = (size_t)(tx + 2) * (ty + 2) * (tz + 2);
  const size_t nb = (size_t)(tx + 1) * (ty + 1) * (tz + 1);
  return (11 * hv + 3 * nb) * (precision == 0 ? sizeof(double) : sizeof(float));
}

hipError_t launch_fused_a(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int tx, int ty,
                          int tz) {
  if (ntask == 0 || nblk == 0) return hipSuccess;
  const size_t lds = fused_a_lds_bytes(c.precision, tx, ty, tz);
  if (lds > AMRX_FUSED_LDS_MAX) return hipErrorInvalidValue;
  const int nthr = fused_a_threads(tx, ty, tz);
  const dim3 g(nblk);
  if (c.precision == 0)
    k_fused_a<double, false><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, tx, ty, tz);
  else if (c.precision == 1)
    k_fused_a<float, false><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, tx, ty, tz);
  else
    k_fused_a<float, true><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, tx, ty, tz);
  return hipGetLastError();
}

size_t fused_b_lds_bytes(int precision, int tx, int ty, int tz) {
  return (size_t)3 * (tx + 1) * (ty + 1) * (tz + 1) * (precision == 0 ? sizeof(double) : sizeof(float));
}

hipError_t launch_fused_b(const DevCtx& c, int task_first, int ntask, int nblk, int cur, int level, int substep, int tx,
                          int ty, int tz) {
  if (ntask == 0 || nblk == 0) return hipSuccess;
  const size_t lds = fused_b_lds_bytes(c.precision, tx, ty, tz);
  if (lds > AMRX_FUSED_LDS_MAX) return hipErrorInvalidValue;
  const int nthr = fused_a_threads(tx, ty, tz);
  const dim3 g(nblk);
  if (c.precision == 0)
    k_fused_b<double, false><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, substep, tx, ty, tz);
  else if (c.precision == 1)
    k_fused_b<float, false><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, substep, tx, ty, tz);
  else
    k_fused_b<float, true><<<g, nthr, lds, c.stream>>>(c, task_first, ntask, cur, level, substep, tx, ty, tz);
  return hipGetLastError();
}

hipError_t launch_copy(const DevCtx& c, int run_first, int nrun, int blk_first, int nblk, int nelem, int cur) {
  if (nrun == 0 || nblk == 0) return hipSuccess;
  DISPATCH_R(k_copy, dim3(nblk), c, run_first, nrun, blk_first, nelem, cur);
  return hipGetLastError();
}

hipError_t launch_prolong(const DevCtx& c, int first, int n, int cur_fine, int old_parent, int new_parent, double w) {
  if (n == 0) return hipSuccess;
  DISPATCH_R(k_prolong, dim3(grid_of(n, AMRX_BLOCK)), c, first, n, cur_fine, old_parent, new_parent, w);
  return hipGetLastError();
}

hipError_t launch_restrict(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk, int cur_fine,
                           int cur_coarse) {
  (void)blk_first;
  if (ntask == 0 || nblk == 0) return hipSuccess;
  DISPATCH_R(k_restrict, dim3(nblk), c, task_first, ntask, cur_fine, cur_coarse);
  return hipGetLastError();
}

hipError_t launch_flux_corr(const DevCtx& c, int first, int n, int cur_coarse) {
  if (n == 0) return hipSuccess;
  DISPATCH(k_flux_corr, dim3(grid_of(n, AMRX_BLOCK)), c, first, n, cur_coarse);
  return hipGetLastError();
}

hipError_t launch_emf_corr(const DevCtx& c, int first, int n, int cur_coarse) {
  if (n == 0) return hipSuccess;
  DISPATCH(k_emf_corr, dim3(grid_of(n, AMRX_BLOCK)), c, first, n, cur_coarse);
  return hipGetLastError();
}

hipError_t launch_sync(const DevCtx& c, int first, int n, int cur) {
  if (n == 0) return hipSuccess;
  DISPATCH(k_sync, dim3(grid_of(n, AMRX_BLOCK)), c, first, n, cur);
  return hipGetLastError();
}

template <int OA, int OB>
hipError_t launch_pair_t(const DevCtx& c, const Node& a, const Node& b) {
  // pad each range to a multiple of the 8 XCDs so that both remaps see whole rounds
  const int pa = (a.nblk + 7) & ~7, pb = (b.nblk + 7) & ~7;
  if (pa + pb == 0) return hipSuccess;
  const dim3 g(pa + pb);
  if (c.precision == 0)
    k_pair<OA, OB, double, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, a, b, pa, pb);
  else if (c.precision == 1)
    k_pair<OA, OB, float, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, a, b, pa, pb);
  else
    k_pair<OA, OB, float, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, a, b, pa, pb);
  return hipGetLastError();
}

#define PAIR_CASES(X)                                                                                \
  X(OP_PRIM, OP_COPY) X(OP_BHALF, OP_PROLONG) X(OP_PRED, OP_PRIM) X(OP_FLUX, OP_BHALF) X(OP_EDGE, OP_PRED) \
  X(OP_UPDATE, OP_FLUX)

bool pair_supported(int op_a, int op_b) {
#define PAIR_TEST(A, B) if (op_a == A && op_b == B) return true;
  PAIR_CASES(PAIR_TEST)
#undef PAIR_TEST
  return false;
}

hipError_t launch_pair(const DevCtx& c, const Node& a, const Node& b) {
#define PAIR_LAUNCH(A, B) \
  if (a.op == A && b.op == B) return launch_pair_t<A, B>(c, a, b);
  PAIR_CASES(PAIR_LAUNCH)
#undef PAIR_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_cfl_all(const DevCtx& c, const CflLevels& L, double cfl) {
  const int g = L.grid0[L.nlev];
  if (g > 0) DISPATCH(k_cfl_all, dim3(g), c, L);
  k_dt_from_partials<<<1, AMRX_BLOCK, 0, c.stream>>>(c, L, cfl);
  return hipGetLastError();
}

hipError_t launch_restrict_corr(const DevCtx& c, int rfirst, int rn, int rnblk, int ffirst, int fn, int efirst, int en,
                                int cur_fine, int cur_coarse) {
  const int g = (rn > 0 ? rnblk : 0) + (fn + AMRX_BLOCK - 1) / AMRX_BLOCK + (en + AMRX_BLOCK - 1) / AMRX_BLOCK;
  if (g == 0) return hipSuccess;
  DISPATCH(k_restrict_corr, dim3(g), c, rfirst, rn, rn > 0 ? rnblk : 0, ffirst, fn, efirst, en, cur_fine, cur_coarse);
  return hipGetLastError();
}

hipError_t launch_cfl(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk, int cur, int level) {
  (void)blk_first;
  if (ntask == 0 || nblk == 0) return hipSuccess;
  DISPATCH(k_cfl, dim3(cfl_grid(nblk)), c, task_first, ntask, nblk, cur, level);
  return hipGetLastError();
}

hipError_t launch_conservation(const DevCtx& c, int task_first, int ntask, int blk_first, int nblk,
                               const int* cur_of_level) {
  (void)blk_first;
  Curs cs;
  for (int l = 0; l < AMRX_MAXLEV; ++l) cs.c[l] = cur_of_level[l];
  if (ntask > 0 && nblk > 0) DISPATCH_R(k_cons, dim3(nblk), c, task_first, ntask, cs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_cons_final<<<1, AMRX_BLOCK, 0, c.stream>>>(c, nblk);
  return hipGetLastError();
}

hipError_t launch_clear_slots(const DevCtx& c) {
  k_clear_slots<<<1, 64, 0, c.stream>>>(c);
  return hipGetLastError();
}

hipError_t launch_clear_acc(const DevCtx& c) {
  k_clear_acc<<<1, 64, 0, c.stream>>>(c);
  return hipGetLastError();
}

hipError_t launch_step_acc(const DevCtx& c) {
  k_step_acc<<<1, 64, 0, c.stream>>>(c);
  return hipGetLastError();
}

hipError_t launch_persistent(const DevCtx& c, const Sched& sc, int nnodes, int nworkgroups, int nlev, double cfl) {
  const unsigned gc = grid_of(nnodes, AMRX_BLOCK);
  k_clear_sched<<<gc < 64 ? gc : 64, AMRX_BLOCK, 0, c.stream>>>(sc, nnodes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g(nworkgroups);
  if (c.precision == 0) k_persistent<double, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, sc, nlev, cfl);
  else if (c.precision == 1) k_persistent<float, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, sc, nlev, cfl);
  else k_persistent<float, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, sc, nlev, cfl);
  return hipGetLastError();
}

hipError_t launch_flag(const DevCtx& c, int first, int n, int nblk, int cur, double eps, unsigned char* flags) {
  if (n == 0 || nblk == 0) return hipSuccess;
  if (c.precision == 0) k_flag<double><<<nblk, AMRX_BLOCK, 0, c.stream>>>(c, first, n, cur, eps, flags);
  else k_flag<float><<<nblk, AMRX_BLOCK, 0, c.stream>>>(c, first, n, cur, eps, flags);
  return hipGetLastError();
}

hipError_t launch_xcopy(int precision, hipStream_t s, const void* src, void* dst, const XRun* runs, int nrun,
                        long long nelem) {
  if (nrun == 0 || nelem == 0) return hipSuccess;
  const unsigned g = (unsigned)((nelem + AMRX_BLOCK - 1) / AMRX_BLOCK);
  if (precision == 0) k_xcopy<double><<<g, AMRX_BLOCK, 0, s>>>((const double*)src, (double*)dst, runs, nrun, nelem);
  else k_xcopy<float><<<g, AMRX_BLOCK, 0, s>>>((const float*)src, (float*)dst, runs, nrun, nelem);
  return hipGetLastError();
}

bool layer2_supported(int oa, int ob) {
#define X(A, B) if (oa == A && ob == B) return true;
  LAYER2_CASES(X)
#undef X
  return false;
}

hipError_t launch_layer(const DevCtx& c, const Node* nodes, const Item* items, int first, int n, int* counter,
                        int nworkgroups, int nlev, double cfl, int op) {
  if (n <= 0) return hipSuccess;
  const int gi = nworkgroups;
  switch (op) {
    case OP_COPY: return launch_layer_op_t<OP_COPY>(c, nodes, items, first, n, counter, gi);
    case OP_PROLONG: return launch_layer_op_t<OP_PROLONG>(c, nodes, items, first, n, counter, gi);
    case OP_PRIM: return launch_layer_op_t<OP_PRIM>(c, nodes, items, first, n, counter, gi);
    case OP_BHALF: return launch_layer_op_t<OP_BHALF>(c, nodes, items, first, n, counter, gi);
    case OP_PRED: return launch_layer_op_t<OP_PRED>(c, nodes, items, first, n, counter, gi);
    case OP_FLUX: return launch_layer_op_t<OP_FLUX>(c, nodes, items, first, n, counter, gi);
    case OP_EDGE: return launch_layer_op_t<OP_EDGE>(c, nodes, items, first, n, counter, gi);
    case OP_UPDATE: return launch_layer_op_t<OP_UPDATE>(c, nodes, items, first, n, counter, gi);
    default: break;
  }
  if (op >= 64) {  // a pair: 64 * (lower op + 1) + higher op
    const int oa = op / 64 - 1, ob = op % 64;
#define X(A, B) if (oa == A && ob == B) return launch_layer2_t<A, B>(c, nodes, items, first, n, counter, gi);
    LAYER2_CASES(X)
#undef X
    return hipErrorInvalidValue;
  }
  const dim3 g(nworkgroups);
  if (c.precision == 0) k_layer<double, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter, nlev, cfl);
  else if (c.precision == 1) k_layer<float, false><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter, nlev, cfl);
  else k_layer<float, true><<<g, AMRX_BLOCK, 0, c.stream>>>(c, nodes, items, first, n, counter, nlev, cfl);
  return hipGetLastError();
}

hipError_t launch_clear_ints(const DevCtx& c, int* p, int n) {
  if (n <= 0) return hipSuccess;
  k_clear_ints<<<grid_of(n, AMRX_BLOCK) < 64 ? grid_of(n, AMRX_BLOCK) : 64, AMRX_BLOCK, 0, c.stream>>>(p, n);
  return hipGetLastError();
}

int layer_blocks_per_cu(int precision) {
  int nb = 0;
  hipError_t e;
  if (precision == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_layer<double, false>, AMRX_BLOCK, 0);
  else if (precision == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_layer<float, false>, AMRX_BLOCK, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_layer<float, true>, AMRX_BLOCK, 0);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

int persistent_blocks_per_cu(int precision) {
  int nb = 0;
  hipError_t e;
  if (precision == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<double, false>, AMRX_BLOCK, 0);
  else if (precision == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<float, false>, AMRX_BLOCK, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<float, true>, AMRX_BLOCK, 0);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_set_dt(const DevCtx& c, double dt0) {

  k_set_dt<<<1, 64, 0, c.stream>>>(c, dt0);
  return hipGetLastError();
}

hipError_t launch_dt_from_cfl(const DevCtx& c, int nlev, double cfl) {
  k_dt_from_cfl<<<1, 64, 0, c.stream>>>(c, nlev, cfl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// static workspace of the entry points that allocate nothing
// ---------------------------------------------------------------------------
// One copy per device, held until the process ends.  Host code never passes the symbol itself (in
// host code it names a host-side stand-in): the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[AMRX_STATIC_WORK_BYTES];

void* static_work_ptr(int dev, hipError_t* err) {
  static std::mutex mu;
  static void* addr[AMRX_MAX_DEVICES] = {};
  *err = hipSuccess;
  if (dev < 0 || dev >= AMRX_MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int prev = -1;
    if ((*err = hipGetDevice(&prev)) != hipSuccess) return nullptr;
    if (prev != dev && (*err = hipSetDevice(dev)) != hipSuccess) return nullptr;
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != dev) {
      const hipError_t e2 = hipSetDevice(prev);
      if (*err == hipSuccess) *err = e2;
    }
    if (*err != hipSuccess) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}
