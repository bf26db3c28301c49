// mhd_math.hpp -- device-side pointwise physics of the ideal-MHD update
// (Stone, Tomida, White & Felker 2020, Sec. 3): fast magnetosonic speed,
// face-frame physical flux, HLLE and HLLD Riemann solvers (Sec. 3.2.2),
// van Leer PLM and Colella-Sekora PPM reconstruction (Sec. 3.2.1), and the
// upwind CT corner-EMF average of Gardiner & Stone (2005) (Sec. 3.1).
//
// All functions are branch-light straight-line FP64 code meant to be inlined
// into the stencil kernels; every lane of a wavefront follows the same
// instruction stream and regions of the Riemann fan are chosen with selects.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

#include "common.hpp"

namespace athmhd {

// Primitive state in the frame of a face: normal direction n, transverse t1, t2
// (cyclic), normal field supplied separately.
struct FaceState {
  double rho, vn, vt1, vt2, p, bt1, bt2;
};

// Flux in the same frame: mass, normal/t1/t2 momentum, energy, B_t1, B_t2.
struct FaceFlux {
  double rho, mn, mt1, mt2, e, bt1, bt2;
};

struct Gas {
  double gamma, gm1, igm1;  // gamma, gamma-1, 1/(gamma-1)
};

__device__ __forceinline__ double sqr(double x) { return x * x; }

// Reciprocal: hardware estimate (v_rcp_f64, relative error below 5e-8 on
// gfx950) refined by one second-order step: with e = 1 - x r0 (exact in an
// FMA), 1/x = r0 / (1 - e) = r0 (1 + e + e^2 + ...); keeping e^2 leaves an
// error of order e^3 < 1e-22, so the result is within about an ulp.  x must
// be finite and non-zero.
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// a / b through the refined reciprocal plus one residual correction.
__device__ __forceinline__ double fdiv(double a, double b) {
  const double r = frcp(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// 1/sqrt(x), x > 0: hardware estimate (v_rsq_f64, relative error below 6e-8)
// refined by one second-order step: with h = 1 - x r0^2,
// 1/sqrt(x) = r0 (1 - h)^(-1/2) = r0 (1 + h/2 + 3h^2/8 + ...).
__device__ __forceinline__ double frsq(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double h = fma(-(x * r), r, 1.0);
  return fma(r, h * fma(0.375, h, 0.5), r);
}

// sqrt(x), x >= 0: one Goldschmidt step from the reciprocal square root
// estimate (g -> sqrt(x), h -> 1/(2 sqrt(x)), relative error ~1e-14 after
// it), finished by a Newton step on the residual x - g^2, which squares the
// error again.
__device__ __forceinline__ double fsqrt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}

// cons -> prim of one cell: u = (rho, M1, M2, M3, E), b = cell-centred field;
// w = (rho, v1, v2, v3, P).  Returns bit 0 set for a non-physical cell (rho <= 0,
// P <= 0 or not finite; with floors on, only a non-finite input) and bit 1 set
// when a floor acted (rho_W = max(rho, d), v = M / rho_W, P = max(P, p)).
// Contraction into multiply-adds is off so that every place that converts a
// cell gets the same bits.
__device__ __forceinline__ int cell_prim(const double* u, const double* b, double gm1, const Floors& fl,
                                         double* w) {
#pragma clang fp contract(off)
  double rho = u[0];
  int flags = 0;
  const bool finite_in = rho == rho && u[4] == u[4] && fabs(rho) < 1.0e300 && fabs(u[4]) < 1.0e300;
  if (fl.on() && finite_in && !(rho >= fl.d)) {
    rho = fl.d;
    flags |= 2;
  }
  const double ir = frcp(rho);
  const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
  const double ke = v1 * v1 + v2 * v2 + v3 * v3;
  const double me = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  double p = gm1 * ((u[4] - 0.5 * rho * ke) - 0.5 * me);
  if (fl.on() && finite_in && !(p >= fl.p)) {
    p = fl.p;
    flags |= 2;
  }
  if (!(rho > 0.0) || !(p > 0.0) || !(p < 1.0e300)) flags |= 1;
  w[0] = rho;
  w[1] = v1;
  w[2] = v2;
  w[3] = v3;
  w[4] = p;
  return flags;
}

// Fast magnetosonic speed along the normal:
//   c_f^2 = ((a^2 + B^2/rho) + sqrt((a^2 + B^2/rho)^2 - 4 a^2 B_n^2/rho)) / 2
__device__ __forceinline__ double fast_speed(double irho, double p, double bnsq, double btsq, double gamma) {
  double asq = gamma * p * irho;
  double s = asq + (bnsq + btsq) * irho;
  double disc = fmax(s * s - 4.0 * asq * bnsq * irho, 0.0);
  return fsqrt(0.5 * (s + fsqrt(disc)));
}

// CFL limit of one cell (Sec. 2.1.7, Sec. 3.2.3): d = min over directions of
// dx_d / (|v_d| + c_f,d) from its conserved state u and cell-centred field b.
// Returns false (d untouched) for a non-physical cell or a limit that is not
// positive and finite.  Every CFL reduction calls this, so a fused and a
// separate reduction of the same state agree.
__device__ __forceinline__ bool cfl_cell(const double* u, const double* b, double gamma, const Floors& fl,
                                         double dx1, double dx2, double dx3, double& d) {
  double w[5];
  if (cell_prim(u, b, gamma - 1.0, fl, w) & 1) return false;
  const double ir = frcp(w[0]), v1 = w[1], v2 = w[2], v3 = w[3], p = w[4];
  const double bs1 = b[0] * b[0], bs2 = b[1] * b[1], bs3 = b[2] * b[2];
  const double c1 = fast_speed(ir, p, bs1, bs2 + bs3, gamma);
  const double c2 = fast_speed(ir, p, bs2, bs3 + bs1, gamma);
  const double c3 = fast_speed(ir, p, bs3, bs1 + bs2, gamma);
  const double dd = fmin(dx1 * frcp(fabs(v1) + c1), fmin(dx2 * frcp(fabs(v2) + c2), dx3 * frcp(fabs(v3) + c3)));
  if (!(dd > 0.0) || !(dd < DBL_MAX)) return false;
  d = dd;
  return true;
}

// HLLE with Davis wave-speed bounds.
__device__ __forceinline__ void hlle(const FaceState& L, const FaceState& R, double bn, const Gas& g, FaceFlux& F,
                                     double& smax) {
  const double bnsq = bn * bn;
  const double irl = frcp(L.rho), irr = frcp(R.rho);
  const double btl = L.bt1 * L.bt1 + L.bt2 * L.bt2, btr = R.bt1 * R.bt1 + R.bt2 * R.bt2;
  const double cfl = fast_speed(irl, L.p, bnsq, btl, g.gamma);
  const double cfr = fast_speed(irr, R.p, bnsq, btr, g.gamma);
  const double sl = fmin(L.vn - cfl, R.vn - cfr);
  const double sr = fmax(L.vn + cfl, R.vn + cfr);
  smax = fmax(fabs(sl), fabs(sr));
  const double bp = fmax(sr, 0.0), bm = fmin(sl, 0.0);
  const double idb = frcp(bp - bm);
  const double wl = bp * idb, wr = -bm * idb, wd = bp * bm * idb;
  // left and right conserved states and physical fluxes
  const double pml = 0.5 * (bnsq + btl), pmr = 0.5 * (bnsq + btr);
  const double ptl = L.p + pml, ptr = R.p + pmr;
  const double el = L.p * g.igm1 + 0.5 * L.rho * (L.vn * L.vn + L.vt1 * L.vt1 + L.vt2 * L.vt2) + pml;
  const double er = R.p * g.igm1 + 0.5 * R.rho * (R.vn * R.vn + R.vt1 * R.vt1 + R.vt2 * R.vt2) + pmr;
  const double mnl = L.rho * L.vn, mnr = R.rho * R.vn;
  const double vbl = L.vn * bn + L.vt1 * L.bt1 + L.vt2 * L.bt2;
  const double vbr = R.vn * bn + R.vt1 * R.bt1 + R.vt2 * R.bt2;
  F.rho = wl * mnl + wr * mnr + wd * (R.rho - L.rho);
  F.mn = wl * (mnl * L.vn + ptl - bnsq) + wr * (mnr * R.vn + ptr - bnsq) + wd * (mnr - mnl);
  F.mt1 = wl * (mnl * L.vt1 - bn * L.bt1) + wr * (mnr * R.vt1 - bn * R.bt1) + wd * (R.rho * R.vt1 - L.rho * L.vt1);
  F.mt2 = wl * (mnl * L.vt2 - bn * L.bt2) + wr * (mnr * R.vt2 - bn * R.bt2) + wd * (R.rho * R.vt2 - L.rho * L.vt2);
  F.e = wl * ((el + ptl) * L.vn - bn * vbl) + wr * ((er + ptr) * R.vn - bn * vbr) + wd * (er - el);
  F.bt1 = wl * (L.bt1 * L.vn - bn * L.vt1) + wr * (R.bt1 * R.vn - bn * R.vt1) + wd * (R.bt1 - L.bt1);
  F.bt2 = wl * (L.bt2 * L.vn - bn * L.vt2) + wr * (R.bt2 * R.vn - bn * R.vt2) + wd * (R.bt2 - L.bt2);
}

// HLLD (Miyoshi & Kusano 2005): outer fast waves, contact S_M, rotational
// waves S*_L, S*_R.  Degenerate star states (|rho (S-u)(S-S_M) - Bn^2| or
// Bn^2/2 below 1e-8 of the star total pressure) fall back to the unmodified
// transverse state / the single-star state.
__device__ __forceinline__ void hlld(const FaceState& L, const FaceState& R, double bn, const Gas& g, FaceFlux& F,
                                     double& smax) {
  constexpr double kSmall = 1.0e-8;
  const double bnsq = bn * bn;
  const double irl = frcp(L.rho), irr = frcp(R.rho);
  const double btl = L.bt1 * L.bt1 + L.bt2 * L.bt2, btr = R.bt1 * R.bt1 + R.bt2 * R.bt2;
  const double ptl = L.p + 0.5 * (bnsq + btl), ptr = R.p + 0.5 * (bnsq + btr);

  const double cfl = fast_speed(irl, L.p, bnsq, btl, g.gamma);
  const double cfr = fast_speed(irr, R.p, bnsq, btr, g.gamma);
  const double cmax = fmax(cfl, cfr);
  const double sl = fmin(L.vn, R.vn) - cmax;
  const double sr = fmax(L.vn, R.vn) + cmax;
  smax = fmax(fabs(sl), fabs(sr));

  // contact speed and total pressure of the star region
  const double ml = (sl - L.vn) * L.rho;  // < 0
  const double mr = (sr - R.vn) * R.rho;  // > 0
  const double iden = frcp(mr - ml);
  const double sm = (mr * R.vn - ml * L.vn - ptr + ptl) * iden;
  const double pts = (mr * ptl - ml * ptr + ml * mr * (R.vn - L.vn)) * iden;

  // single-star densities and rotational speeds
  const double isl = frcp(sl - sm), isr = frcp(sr - sm);
  const double rsl = ml * isl, rsr = mr * isr;  // rho*_L, rho*_R
  // sqrt(rho*) and 1/sqrt(rho*) from one refined reciprocal square root
  const double irql = frsq(rsl), irqr = frsq(rsr);
  const double sqrl = rsl * irql, sqrr = rsr * irqr;
  const double ssl = sm - fabs(bn) * irql;
  const double ssr = sm + fabs(bn) * irqr;

  // region of the fan that contains x/t = 0, and which side's states it uses
  const bool useL = (sl > 0.0) || (!(sr < 0.0) && (ssl >= 0.0 || (!(ssr <= 0.0) && sm >= 0.0)));
  const bool star = !(sl > 0.0) && !(sr < 0.0);
  const bool dstar = !(0.5 * bnsq < kSmall * pts);
  const bool dbl = star && !(ssl >= 0.0) && !(ssr <= 0.0) && dstar;

  // transverse velocity and field of the single-star states (both sides are
  // needed by the double-star state)
  // (degenerate: the correction factors c1 = 0, c2 = 1 leave the transverse
  // state unchanged)
  double vt1sl, vt2sl, bt1sl, bt2sl, vt1sr, vt2sr, bt1sr, bt2sr;
  {
    const double d = ml * (sl - sm) - bnsq;
    const bool degen = fabs(d) < kSmall * pts;
    const double id = frcp(degen ? 1.0 : d);
    const double c1 = degen ? 0.0 : bn * (sm - L.vn) * id;
    const double c2 = degen ? 1.0 : (ml * (sl - L.vn) - bnsq) * id;
    vt1sl = L.vt1 - L.bt1 * c1;
    vt2sl = L.vt2 - L.bt2 * c1;
    bt1sl = L.bt1 * c2;
    bt2sl = L.bt2 * c2;
  }
  {
    const double d = mr * (sr - sm) - bnsq;
    const bool degen = fabs(d) < kSmall * pts;
    const double id = frcp(degen ? 1.0 : d);
    const double c1 = degen ? 0.0 : bn * (sm - R.vn) * id;
    const double c2 = degen ? 1.0 : (mr * (sr - R.vn) - bnsq) * id;
    vt1sr = R.vt1 - R.bt1 * c1;
    vt2sr = R.vt2 - R.bt2 * c1;
    bt1sr = R.bt1 * c2;
    bt2sr = R.bt2 * c2;
  }

  // double-star state (shared velocity and field)
  const double sgn = bn > 0.0 ? 1.0 : (bn < 0.0 ? -1.0 : 0.0);
  const double isum = frcp(sqrl + sqrr);
  const double vt1ss = (sqrl * vt1sl + sqrr * vt1sr + (bt1sr - bt1sl) * sgn) * isum;
  const double vt2ss = (sqrl * vt2sl + sqrr * vt2sr + (bt2sr - bt2sl) * sgn) * isum;
  const double bt1ss = (sqrl * bt1sr + sqrr * bt1sl + sqrl * sqrr * (vt1sr - vt1sl) * sgn) * isum;
  const double bt2ss = (sqrl * bt2sr + sqrr * bt2sl + sqrl * sqrr * (vt2sr - vt2sl) * sgn) * isum;
  const double vbss = sm * bn + vt1ss * bt1ss + vt2ss * bt2ss;

  // chosen side: its state, energy and physical flux, then its star and
  // double-star energies
  const double rho = useL ? L.rho : R.rho;
  const double vn = useL ? L.vn : R.vn;
  const double vt1 = useL ? L.vt1 : R.vt1;
  const double vt2 = useL ? L.vt2 : R.vt2;
  const double p = useL ? L.p : R.p;
  const double bt1 = useL ? L.bt1 : R.bt1;
  const double bt2 = useL ? L.bt2 : R.bt2;
  const double pt = useL ? ptl : ptr;
  const double s = useL ? sl : sr;
  const double is = useL ? isl : isr;
  const double ss = useL ? ssl : ssr;
  const double rs = useL ? rsl : rsr;
  const double sq = useL ? sqrl : sqrr;
  const double vt1s = useL ? vt1sl : vt1sr, vt2s = useL ? vt2sl : vt2sr;
  const double bt1s = useL ? bt1sl : bt1sr, bt2s = useL ? bt2sl : bt2sr;
  const double en = p * g.igm1 + 0.5 * rho * (vn * vn + vt1 * vt1 + vt2 * vt2) + 0.5 * (bnsq + bt1 * bt1 + bt2 * bt2);
  const double vb = vn * bn + vt1 * bt1 + vt2 * bt2;
  const double vbs = sm * bn + vt1s * bt1s + vt2s * bt2s;
  const double es = ((s - vn) * en - pt * vn + pts * sm + bn * (vb - vbs)) * is;
  const double ess = useL ? es - sq * (vbs - vbss) * sgn : es + sq * (vbs - vbss) * sgn;

  const double mn = rho * vn;
  F.rho = mn;
  F.mn = mn * vn + pt - bnsq;
  F.mt1 = mn * vt1 - bn * bt1;
  F.mt2 = mn * vt2 - bn * bt2;
  F.e = (en + pt) * vn - bn * vb;
  F.bt1 = bt1 * vn - bn * vt1;
  F.bt2 = bt2 * vn - bn * vt2;
  if (star) {
    // F + S (U* - U)
    F.rho += s * (rs - rho);
    F.mn += s * (rs * sm - mn);
    F.mt1 += s * (rs * vt1s - rho * vt1);
    F.mt2 += s * (rs * vt2s - rho * vt2);
    F.e += s * (es - en);
    F.bt1 += s * (bt1s - bt1);
    F.bt2 += s * (bt2s - bt2);
  }
  if (dbl) {
    // + S* (U** - U*)
    F.mt1 += ss * (rs * vt1ss - rs * vt1s);
    F.mt2 += ss * (rs * vt2ss - rs * vt2s);
    F.e += ss * (ess - es);
    F.bt1 += ss * (bt1ss - bt1s);
    F.bt2 += ss * (bt2ss - bt2s);
  }
}

// Roe's linearised solver (Sec. 3.2.2) with the Roe matrix of our own
// derivation: s = sqrt(rho), s-weighted velocity and total enthalpy
// H = (E + P_T) / rho, the transverse field averaged with swapped weights
// (s_R B_L + s_L B_R) / (s_L + s_R), and X = |dB_t|^2 / (2 (s_L + s_R)^2).
// With these every jump of U and of the flux is linear in the primitive jumps
// dW = (d rho, du_n, du_t1, du_t2, dP, dB_t1, dB_t2), and the matrix has seven
// waves: u, u -+ b_n (Alfven), u -+ c_f, u -+ c_s, for the sound speed
// a^2 = (gamma-1)(H - v^2/2 - B^2/rho) - (gamma-2) X.  The flux is
// (F_L + F_R)/2 - M D / 2, where dW is split into the waves' right
// eigenvectors (closed form in the frame of the averaged transverse field,
// normalised with alpha_f, alpha_s as for characteristic reconstruction),
// D = sum |lambda_k| a_k R_k, and M maps primitive onto conserved jumps at the
// averaged state.  The entropy wave carries dP = -X d rho.  No entropy fix.
// smax (for the CT weight) is the larger |u_n| + c_f of the two states.
__device__ __forceinline__ void roe(const FaceState& L, const FaceState& R, double bn, const Gas& g, FaceFlux& F,
                                    double& smax) {
  const double bnsq = bn * bn;
  const double irl = frcp(L.rho), irr = frcp(R.rho);
  const double btl = L.bt1 * L.bt1 + L.bt2 * L.bt2, btr = R.bt1 * R.bt1 + R.bt2 * R.bt2;
  smax = fmax(fabs(L.vn) + fast_speed(irl, L.p, bnsq, btl, g.gamma), fabs(R.vn) + fast_speed(irr, R.p, bnsq, btr, g.gamma));

  // physical fluxes of the two states
  const double pml = 0.5 * (bnsq + btl), pmr = 0.5 * (bnsq + btr);
  const double ptl = L.p + pml, ptr = R.p + pmr;
  const double el = L.p * g.igm1 + 0.5 * L.rho * (L.vn * L.vn + L.vt1 * L.vt1 + L.vt2 * L.vt2) + pml;
  const double er = R.p * g.igm1 + 0.5 * R.rho * (R.vn * R.vn + R.vt1 * R.vt1 + R.vt2 * R.vt2) + pmr;
  const double mnl = L.rho * L.vn, mnr = R.rho * R.vn;
  const double vbl = L.vn * bn + L.vt1 * L.bt1 + L.vt2 * L.bt2;
  const double vbr = R.vn * bn + R.vt1 * R.bt1 + R.vt2 * R.bt2;

  // averaged state
  const double sl = L.rho * frsq(L.rho), sr = R.rho * frsq(R.rho);
  const double iD = frcp(sl + sr);
  const double wl = sl * iD, wr = sr * iD;
  const double rho = sl * sr, irho = frcp(rho);
  const double S = fsqrt(rho), iS = frcp(S);
  const double u = wl * L.vn + wr * R.vn, v1 = wl * L.vt1 + wr * R.vt1, v2 = wl * L.vt2 + wr * R.vt2;
  const double H = wl * ((el + ptl) * irl) + wr * ((er + ptr) * irr);
  const double b1 = wr * L.bt1 + wl * R.bt1, b2 = wr * L.bt2 + wl * R.bt2;
  const double db1 = R.bt1 - L.bt1, db2 = R.bt2 - L.bt2;
  const double X = 0.5 * (db1 * db1 + db2 * db2) * iD * iD;
  const double vsq = u * u + v1 * v1 + v2 * v2;
  const double btsum = b1 * b1 + b2 * b2;
  const double ah2 = g.gm1 * (H - 0.5 * vsq - (bnsq + btsum) * irho - X);  // a^2 - X
  const double a2 = ah2 + X;
  const double bx2 = bnsq * irho, bt2 = btsum * irho, b2sum = bx2 + bt2;
  const double dab = a2 - b2sum;
  const double disc = fsqrt(dab * dab + 4.0 * a2 * bt2);
  const double cf2 = 0.5 * (a2 + b2sum + disc);
  const double cs2 = a2 * bx2 * frcp(cf2);
  const double cf = fsqrt(cf2), cs = fsqrt(cs2), ca = fabs(bn) * iS, a = fsqrt(a2);
  // alpha_f^2 = (a^2 - c_s^2) / (c_f^2 - c_s^2), alpha_s^2 = (c_f^2 - a^2) / (c_f^2 - c_s^2),
  // each numerator in a form without cancellation; (1, 0) when c_f = c_s
  const bool split = disc > 0.0;
  const double idisc = frcp(split ? disc : 1.0);
  const double t4 = 2.0 * a2 * bt2;
  const double cfa = dab <= 0.0 ? 0.5 * (disc - dab) : t4 * frcp(split ? disc + dab : 1.0);
  const double acs = dab >= 0.0 ? 0.5 * (disc + dab) : t4 * frcp(split ? disc - dab : 1.0);
  const double af = split ? fsqrt(acs * idisc) : 1.0;
  const double as = split ? fsqrt(cfa * idisc) : 0.0;
  // direction of the averaged transverse field ((1, 1)/sqrt2 when it vanishes)
  const bool hasbt = btsum > 0.0;
  const double ib = frsq(hasbt ? btsum : 2.0);
  const double be1 = hasbt ? b1 * ib : ib, be2 = hasbt ? b2 * ib : ib;
  const double sg = bn >= 0.0 ? 1.0 : -1.0;

  // primitive jumps, transverse parts along and across the field direction
  const double drho = R.rho - L.rho, du = R.vn - L.vn, dp = R.p - L.p;
  const double dv1 = R.vt1 - L.vt1, dv2 = R.vt2 - L.vt2;
  const double dvpar = be1 * dv1 + be2 * dv2, dvper = be1 * dv2 - be2 * dv1;
  const double dbpar = be1 * db1 + be2 * db2, dbper = be1 * db2 - be2 * db1;

  // wave strengths
  const double aAp = 0.5 * (dvper - sg * dbper * iS), aAm = 0.5 * (dvper + sg * dbper * iS);
  const double iQ = frcp(cf2 * af * af + cs2 * as * as);
  const double dF = (af * cf * du - sg * as * cs * dvpar) * iQ;
  const double dS = (as * cs * du + sg * af * cf * dvpar) * iQ;
  const double P = (dp + X * drho) * frcp(rho * a2);
  const double Qp = dbpar * frcp(S * a);
  const double sF = af * P + as * Qp, sS = as * P - af * Qp;
  const double aE = drho - rho * P;

  // |lambda| a for every wave
  const double wE = fabs(u) * aE;
  const double wAp = fabs(u + ca) * aAp, wAm = fabs(u - ca) * aAm;
  const double wFp = fabs(u + cf) * 0.5 * (sF + dF), wFm = fabs(u - cf) * 0.5 * (sF - dF);
  const double wSp = fabs(u + cs) * 0.5 * (sS + dS), wSm = fabs(u - cs) * 0.5 * (sS - dS);

  // D = sum |lambda| a R in primitive jumps
  const double fs = wFp + wFm, fd = wFp - wFm, ss = wSp + wSm, sd = wSp - wSm;
  const double Drho = wE + rho * (af * fs + as * ss);
  const double Du = cf * af * fd + cs * as * sd;
  const double Dvpar = sg * (af * cf * sd - as * cs * fd);
  const double Dvper = wAp + wAm;
  const double Dp = rho * ah2 * (af * fs + as * ss) - X * wE;
  const double Dbpar = S * a * (as * fs - af * ss);
  const double Dbper = -sg * S * (wAp - wAm);
  const double Dv1 = be1 * Dvpar - be2 * Dvper, Dv2 = be2 * Dvpar + be1 * Dvper;
  const double Db1 = be1 * Dbpar - be2 * Dbper, Db2 = be2 * Dbpar + be1 * Dbper;

  // conserved form of D at the averaged state, and the flux
  const double Umn = rho * Du + u * Drho;
  const double Um1 = rho * Dv1 + v1 * Drho, Um2 = rho * Dv2 + v2 * Drho;
  const double UE = Dp * g.igm1 + rho * (u * Du + v1 * Dv1 + v2 * Dv2) + (0.5 * vsq + X) * Drho + b1 * Db1 + b2 * Db2;
  F.rho = 0.5 * (mnl + mnr - Drho);
  F.mn = 0.5 * (mnl * L.vn + ptl - bnsq + mnr * R.vn + ptr - bnsq - Umn);
  F.mt1 = 0.5 * (mnl * L.vt1 - bn * L.bt1 + mnr * R.vt1 - bn * R.bt1 - Um1);
  F.mt2 = 0.5 * (mnl * L.vt2 - bn * L.bt2 + mnr * R.vt2 - bn * R.bt2 - Um2);
  F.e = 0.5 * ((el + ptl) * L.vn - bn * vbl + (er + ptr) * R.vn - bn * vbr - UE);
  F.bt1 = 0.5 * (L.bt1 * L.vn - bn * L.vt1 + R.bt1 * R.vn - bn * R.vt1 - Db1);
  F.bt2 = 0.5 * (L.bt2 * L.vn - bn * L.vt2 + R.bt2 * R.vn - bn * R.vt2 - Db2);
}

// Riemann solver of a kernel's compile-time choice: 0 HLLE, 1 HLLD, 2 Roe.
template <int RS>
__device__ __forceinline__ void riemann_flux(const FaceState& L, const FaceState& R, double bn, const Gas& g,
                                             FaceFlux& F, double& smax) {
  if (RS == 1) hlld(L, R, bn, g, F, smax);
  else if (RS == 2) roe(L, R, bn, g, F, smax);
  else hlle(L, R, bn, g, F, smax);
}

// van Leer (1974) slope: harmonic mean of the one-sided differences when they
// share a sign, else zero.
__device__ __forceinline__ double vl_slope(double qm, double q0, double qp) {
  const double dm = q0 - qm, dp = qp - q0;
  const double pr = dm * dp;
  return pr > 0.0 ? 2.0 * pr * frcp(dm + dp) : 0.0;
}

// Colella & Sekora (2008) extremum-preserving PPM on a uniform grid.
__device__ __forceinline__ double cs_lim3(double a, double b, double c) {
  constexpr double C = 1.25;
  const bool pos = a > 0.0 && b > 0.0 && c > 0.0;
  const bool neg = a < 0.0 && b < 0.0 && c < 0.0;
  const double m = fmin(fabs(a), fmin(C * fabs(b), C * fabs(c)));
  return pos ? m : (neg ? -m : 0.0);
}

// limited face value between q0 (=q_{c-1}) and q1 (=q_c); qm1 = q_{c-2}, q2 = q_{c+1}
__device__ __forceinline__ double ppm_face(double qm1, double q0, double q1, double q2) {
  double qf = (7.0 / 12.0) * (q0 + q1) - (1.0 / 12.0) * (qm1 + q2);
  if ((qf - q0) * (q1 - qf) < 0.0) {
    const double d2 = 3.0 * (q0 - 2.0 * qf + q1);
    const double d2l = qm1 - 2.0 * q0 + q1;
    const double d2r = q0 - 2.0 * q1 + q2;
    qf = 0.5 * (q0 + q1) - cs_lim3(d2, d2l, d2r) * (1.0 / 6.0);
  }
  return qf;
}

// limited parabola of cell c from q_{c-2..c+2} and its two raw face values;
// returns the left (qm) and right (qp) edge values
__device__ __forceinline__ void ppm_cell(double qa, double qb, double qc, double qd, double qe, double& qm,
                                         double& qp) {
  constexpr double C = 1.25;
  // qa..qe = q_{c-2}, q_{c-1}, q_c, q_{c+1}, q_{c+2}
  if ((qp - qc) * (qc - qm) <= 0.0 || (qb - qc) * (qc - qd) <= 0.0) {
    const double d2 = 6.0 * (qm + qp) - 12.0 * qc;
    const double d2c = qb - 2.0 * qc + qd;
    const double d2l = qa - 2.0 * qb + qc;
    const double d2r = qc - 2.0 * qd + qe;
    const bool pos = d2 > 0.0 && d2c > 0.0 && d2l > 0.0 && d2r > 0.0;
    const bool neg = d2 < 0.0 && d2c < 0.0 && d2l < 0.0 && d2r < 0.0;
    const double m = fmin(fabs(d2), fmin(C * fabs(d2l), fmin(C * fabs(d2r), C * fabs(d2c))));
    const double lim = pos ? m : (neg ? -m : 0.0);
    if (d2 != 0.0) {
      // lim and d2 share their sign and |lim| <= |d2|, so r is in [0, 1].  A
      // tiny d2 (denormal, as in the decaying precursor ahead of a blast wave)
      // has no finite reciprocal: scale both by a power of two first (exact).
      double num = lim, den = d2;
      if (fabs(den) < 0x1p-900) {
        num *= 0x1p900;
        den *= 0x1p900;
      }
      const double r = num * frcp(den);
      qm = qc + (qm - qc) * r;
      qp = qc + (qp - qc) * r;
    } else {
      qm = qc;
      qp = qc;
    }
  } else {
    const double dqm = qm - qc, dqp = qp - qc;
    if (fabs(dqp) >= 2.0 * fabs(dqm)) qp = qc - 2.0 * dqm;
    if (fabs(dqm) >= 2.0 * fabs(qp - qc)) qm = qc - 2.0 * (qp - qc);
  }
}

// Reconstruct the two edge values of cell c from a line of cells centred on
// it (Sec. 3.2.1): s[LA + o] = q_{c+o}, o in [-LA, LA], with LA = 0, 1, 2 for
// DC, PLM, PPM; returns (left edge, right edge).
template <int RECON>
__device__ __forceinline__ void cell_edges(const double* s, double& left, double& right) {
  if (RECON == 0) {
    left = s[0];
    right = s[0];
  } else if (RECON == 1) {
    const double d = vl_slope(s[0], s[1], s[2]);
    left = s[1] - 0.5 * d;
    right = s[1] + 0.5 * d;
  } else {
    double qm = ppm_face(s[0], s[1], s[2], s[3]);
    double qp = ppm_face(s[1], s[2], s[3], s[4]);
    ppm_cell(s[0], s[1], s[2], s[3], s[4], qm, qp);
    left = qm;
    right = qp;
  }
}

// Upwind CT corner EMF (Gardiner & Stone 2005) at the edge shared by four
// cells.  Notation for component e with transverse directions a, b:
//   ea0 = face-a EMF at (c), ea1 = at (c - b)   [faces normal to a]
//   eb0 = face-b EMF at (c), eb1 = at (c - a)   [faces normal to b]
//   c00 = cell EMF at c, ca = at c - a, cb = at c - b, cab = at c - a - b
//   wa0, wa1 = upwind weights of the a-faces (c), (c - b); wb0, wb1 of the
//   b-faces (c), (c - a); weight 1 selects the cell on the low side.
__device__ __forceinline__ double corner_emf(double ea0, double ea1, double eb0, double eb1, double c00, double ca,
                                             double cb, double cab, double wa0, double wa1, double wb0,
                                             double wb1) {
  const double avg = 0.25 * (ea0 + ea1 + eb0 + eb1);
  const double dbp = wa0 * (ca - eb1) + (1.0 - wa0) * (c00 - eb0);
  const double dbm = wa1 * (eb1 - cab) + (1.0 - wa1) * (eb0 - cb);
  const double dap = wb0 * (cb - ea1) + (1.0 - wb0) * (c00 - ea0);
  const double dam = wb1 * (ea1 - cab) + (1.0 - wb1) * (ea0 - ca);
  return avg + 0.25 * (dbm - dbp) + 0.25 * (dam - dap);
}

// Floors on a reconstructed face state; returns 1 if one acted.
__device__ __forceinline__ int floor_state(FaceState& s, const Floors& fl) {
  int acted = 0;
  if (!(s.rho >= fl.d)) { s.rho = fl.d; acted = 1; }
  if (!(s.p >= fl.p)) { s.p = fl.p; acted = 1; }
  return acted;
}

// upwind weight of a face from its mass flux
__device__ __forceinline__ double ct_weight(double frho, double rhobar, double smax, double eps) {
  if (eps > 0.0) {
    const double r = 0.5 + 0.5 * frho * frcp(rhobar * eps * smax);
    return fmin(1.0, fmax(0.0, r));
  }
  return frho > 0.0 ? 1.0 : (frho < 0.0 ? 0.0 : 0.5);
}

}  // namespace athmhd
