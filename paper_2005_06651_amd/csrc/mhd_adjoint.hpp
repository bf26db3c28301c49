// mhd_adjoint.hpp -- reverse-mode derivatives (vector-Jacobian products) of the
// pointwise physics in mhd_math.hpp: van Leer PLM edges, cons->prim, the fast
// magnetosonic speed, HLLD with the CT upwind weight, and the corner-EMF
// average.  Each *_vjp function recomputes the forward values it needs and
// then runs the reverse sweep, accumulating adjoints (`x_b += dy/dx * y_b`)
// in the opposite order of the forward statements.  Selects (regions of the
// Riemann fan, limiter branches, degenerate-state guards, min / max) route an
// adjoint to the operand the forward pass took.
#pragma once

#include "mhd_math.hpp"

namespace athmhd {

// ---- van Leer slope: d = 2 dm dp / (dm + dp) if dm dp > 0, else 0 ----------
// adjoint of d w.r.t. (qm, q0, qp)
__device__ __forceinline__ void vl_slope_vjp(double qm, double q0, double qp, double d_b, double& qm_b, double& q0_b,
                                             double& qp_b) {
  const double dm = q0 - qm, dp = qp - q0;
  if (!(dm * dp > 0.0)) return;
  const double isum = frcp(dm + dp);
  const double ddm = 2.0 * dp * dp * isum * isum;  // dd/ddm
  const double ddp = 2.0 * dm * dm * isum * isum;  // dd/ddp
  const double dm_b = d_b * ddm, dp_b = d_b * ddp;
  qm_b -= dm_b;
  q0_b += dm_b - dp_b;
  qp_b += dp_b;
}

// ---- fast magnetosonic speed (see fast_speed) -------------------------------
__device__ __forceinline__ void fast_speed_vjp(double irho, double p, double bnsq, double btsq, double gamma,
                                               double cf_b, double& irho_b, double& p_b, double& bnsq_b,
                                               double& btsq_b) {
  const double asq = gamma * p * irho;
  const double s = asq + (bnsq + btsq) * irho;
  const double disc_raw = s * s - 4.0 * asq * bnsq * irho;
  const double disc = fmax(disc_raw, 0.0);
  const double r = fsqrt(disc);
  const double cf = fsqrt(0.5 * (s + r));
  const double cf2_b = cf_b * 0.5 * frcp(cf);
  double s_b = 0.5 * cf2_b;
  const double r_b = 0.5 * cf2_b;
  const double disc_b = disc_raw > 0.0 ? r_b * 0.5 * frcp(r) : 0.0;
  s_b += 2.0 * s * disc_b;
  double asq_b = -4.0 * bnsq * irho * disc_b;
  bnsq_b += -4.0 * asq * irho * disc_b;
  irho_b += -4.0 * asq * bnsq * disc_b;
  asq_b += s_b;
  bnsq_b += s_b * irho;
  btsq_b += s_b * irho;
  irho_b += s_b * (bnsq + btsq);
  p_b += asq_b * gamma * irho;
  irho_b += asq_b * gamma * p;
}

// ---- adjoint of the CT upwind weight (see ct_weight) -------------------------
// w = clamp(1/2 + F_rho / (2 eps rho_bar c_max), 0, 1) for eps > 0; piecewise
// constant (zero derivative) for eps = 0.  Accumulates into the adjoints of
// F_rho, rho_bar and c_max.
__device__ __forceinline__ void ct_weight_vjp(double frho, double rhobar, double smax, double eps, double w_b,
                                              double& frho_b, double& rhobar_b, double& smax_b) {
  if (!(eps > 0.0)) return;
  const double den = rhobar * eps * smax;
  const double iden = frcp(den);
  const double r = 0.5 + 0.5 * frho * iden;
  if (!(r > 0.0 && r < 1.0)) return;
  frho_b += w_b * 0.5 * iden;
  const double t = -w_b * 0.5 * frho * iden * iden;
  rhobar_b += t * eps * smax;
  smax_b += t * rhobar * eps;
}

// ---- one side of a two-state flux: conserved state u and physical flux f ----
// u = (rho, rho vn, rho vt1, rho vt2, E, bt1, bt2) and the normal-frame ideal-MHD
// flux f of the same state; accumulates the adjoints of the primitive state
// and of bn and bn^2 from u_b and f_b.
__device__ __forceinline__ void side_vjp(const FaceState& S, double bn, const Gas& g, const double* u_b,
                                         const double* f_b, FaceState& Sb, double& bn_b, double& bnsq_b) {
  const double bnsq = bn * bn;
  const double btsq = S.bt1 * S.bt1 + S.bt2 * S.bt2;
  const double pm = 0.5 * (bnsq + btsq);
  const double pt = S.p + pm;
  const double e = S.p * g.igm1 + 0.5 * S.rho * (S.vn * S.vn + S.vt1 * S.vt1 + S.vt2 * S.vt2) + pm;
  const double mn = S.rho * S.vn;
  const double vb = S.vn * bn + S.vt1 * S.bt1 + S.vt2 * S.bt2;
  double rho_b = u_b[0], mn_b = u_b[1], e_b = u_b[4];
  double vn_b = 0, vt1_b = 0, vt2_b = 0, bt1_b = u_b[5], bt2_b = u_b[6], pt_b = 0, vb_b = 0, pm_b = 0, p_b = 0;
  rho_b += u_b[2] * S.vt1 + u_b[3] * S.vt2;
  vt1_b += u_b[2] * S.rho;
  vt2_b += u_b[3] * S.rho;
  mn_b += f_b[0] + f_b[1] * S.vn + f_b[2] * S.vt1 + f_b[3] * S.vt2;
  vn_b += f_b[1] * mn;
  pt_b += f_b[1];
  bnsq_b -= f_b[1];
  vt1_b += f_b[2] * mn;
  vt2_b += f_b[3] * mn;
  bn_b -= f_b[2] * S.bt1 + f_b[3] * S.bt2;
  bt1_b -= f_b[2] * bn;
  bt2_b -= f_b[3] * bn;
  e_b += f_b[4] * S.vn;
  pt_b += f_b[4] * S.vn;
  vn_b += f_b[4] * (e + pt);
  bn_b -= f_b[4] * vb;
  vb_b -= f_b[4] * bn;
  bt1_b += f_b[5] * S.vn;
  bt2_b += f_b[6] * S.vn;
  vn_b += f_b[5] * S.bt1 + f_b[6] * S.bt2;
  bn_b -= f_b[5] * S.vt1 + f_b[6] * S.vt2;
  vt1_b -= f_b[5] * bn;
  vt2_b -= f_b[6] * bn;
  vn_b += vb_b * bn;
  bn_b += vb_b * S.vn;
  vt1_b += vb_b * S.bt1;
  bt1_b += vb_b * S.vt1;
  vt2_b += vb_b * S.bt2;
  bt2_b += vb_b * S.vt2;
  rho_b += mn_b * S.vn;
  vn_b += mn_b * S.rho;
  p_b += e_b * g.igm1;
  rho_b += e_b * 0.5 * (S.vn * S.vn + S.vt1 * S.vt1 + S.vt2 * S.vt2);
  vn_b += e_b * S.rho * S.vn;
  vt1_b += e_b * S.rho * S.vt1;
  vt2_b += e_b * S.rho * S.vt2;
  pm_b += e_b + pt_b;
  p_b += pt_b;
  bnsq_b += 0.5 * pm_b;
  bt1_b += S.bt1 * pm_b;
  bt2_b += S.bt2 * pm_b;
  Sb.rho += rho_b;
  Sb.vn += vn_b;
  Sb.vt1 += vt1_b;
  Sb.vt2 += vt2_b;
  Sb.p += p_b;
  Sb.bt1 += bt1_b;
  Sb.bt2 += bt2_b;
}

// ---- HLLE (see hlle) with the CT upwind weight ------------------------------
__device__ __forceinline__ void hlle_vjp(const FaceState& L, const FaceState& R, double bn, const Gas& g,
                                         double ct_eps, const FaceFlux& Fb, double w_b, FaceState& Lb,
                                         FaceState& Rb, double& bn_b) {
  // forward
  const double bnsq = bn * bn;
  const double irl = frcp(L.rho), irr = frcp(R.rho);
  const double btl = L.bt1 * L.bt1 + L.bt2 * L.bt2, btr = R.bt1 * R.bt1 + R.bt2 * R.bt2;
  const double cfl = fast_speed(irl, L.p, bnsq, btl, g.gamma);
  const double cfr = fast_speed(irr, R.p, bnsq, btr, g.gamma);
  const bool slL = L.vn - cfl <= R.vn - cfr;
  const double sl = slL ? L.vn - cfl : R.vn - cfr;
  const bool srL = L.vn + cfl >= R.vn + cfr;
  const double sr = srL ? L.vn + cfl : R.vn + cfr;
  const bool smaxL = fabs(sl) >= fabs(sr);
  const double smax = smaxL ? fabs(sl) : fabs(sr);
  const double bp = fmax(sr, 0.0), bm = fmin(sl, 0.0);
  const double idb = frcp(bp - bm);
  const double wl = bp * idb, wr = -bm * idb, wd = bp * bm * idb;
  double u[2][7], f[2][7];
  {
    const FaceState* S[2] = {&L, &R};
    for (int s = 0; s < 2; ++s) {
      const FaceState& q = *S[s];
      const double pm = 0.5 * (bnsq + q.bt1 * q.bt1 + q.bt2 * q.bt2);
      const double pt = q.p + pm;
      const double e = q.p * g.igm1 + 0.5 * q.rho * (q.vn * q.vn + q.vt1 * q.vt1 + q.vt2 * q.vt2) + pm;
      const double mn = q.rho * q.vn;
      const double vb = q.vn * bn + q.vt1 * q.bt1 + q.vt2 * q.bt2;
      u[s][0] = q.rho; u[s][1] = mn; u[s][2] = q.rho * q.vt1; u[s][3] = q.rho * q.vt2; u[s][4] = e;
      u[s][5] = q.bt1; u[s][6] = q.bt2;
      f[s][0] = mn; f[s][1] = mn * q.vn + pt - bnsq; f[s][2] = mn * q.vt1 - bn * q.bt1;
      f[s][3] = mn * q.vt2 - bn * q.bt2; f[s][4] = (e + pt) * q.vn - bn * vb;
      f[s][5] = q.bt1 * q.vn - bn * q.vt1; f[s][6] = q.bt2 * q.vn - bn * q.vt2;
    }
  }
  const double frho = wl * f[0][0] + wr * f[1][0] + wd * (u[1][0] - u[0][0]);
  // reverse
  double fb[7] = {Fb.rho, Fb.mn, Fb.mt1, Fb.mt2, Fb.e, Fb.bt1, Fb.bt2};
  double rhobar_b = 0.0, smax_b = 0.0;
  ct_weight_vjp(frho, 0.5 * (L.rho + R.rho), smax, ct_eps, w_b, fb[0], rhobar_b, smax_b);
  double wl_b = 0, wr_b = 0, wd_b = 0;
  double fl_b[7], fr_b[7], ul_b[7], ur_b[7];
  for (int v = 0; v < 7; ++v) {
    wl_b += fb[v] * f[0][v];
    wr_b += fb[v] * f[1][v];
    wd_b += fb[v] * (u[1][v] - u[0][v]);
    fl_b[v] = wl * fb[v];
    fr_b[v] = wr * fb[v];
    ur_b[v] = wd * fb[v];
    ul_b[v] = -wd * fb[v];
  }
  double bnsq_b = 0.0;
  side_vjp(L, bn, g, ul_b, fl_b, Lb, bn_b, bnsq_b);
  side_vjp(R, bn, g, ur_b, fr_b, Rb, bn_b, bnsq_b);
  double bp_b = wl_b * idb + wd_b * bm * idb;
  double bm_b = -wr_b * idb + wd_b * bp * idb;
  const double idb_b = wl_b * bp - wr_b * bm + wd_b * bp * bm;
  const double t = -idb * idb * idb_b;
  bp_b += t;
  bm_b -= t;
  double sl_b = sl < 0.0 ? bm_b : 0.0;
  double sr_b = sr > 0.0 ? bp_b : 0.0;
  if (smaxL) sl_b += smax_b * (sl >= 0.0 ? 1.0 : -1.0);
  else sr_b += smax_b * (sr >= 0.0 ? 1.0 : -1.0);
  double cfl_b = 0.0, cfr_b = 0.0;
  if (slL) { Lb.vn += sl_b; cfl_b -= sl_b; } else { Rb.vn += sl_b; cfr_b -= sl_b; }
  if (srL) { Lb.vn += sr_b; cfl_b += sr_b; } else { Rb.vn += sr_b; cfr_b += sr_b; }
  double irl_b = 0.0, irr_b = 0.0, btl_b = 0.0, btr_b = 0.0;
  fast_speed_vjp(irl, L.p, bnsq, btl, g.gamma, cfl_b, irl_b, Lb.p, bnsq_b, btl_b);
  fast_speed_vjp(irr, R.p, bnsq, btr, g.gamma, cfr_b, irr_b, Rb.p, bnsq_b, btr_b);
  Lb.bt1 += 2.0 * L.bt1 * btl_b;
  Lb.bt2 += 2.0 * L.bt2 * btl_b;
  Rb.bt1 += 2.0 * R.bt1 * btr_b;
  Rb.bt2 += 2.0 * R.bt2 * btr_b;
  Lb.rho += -irl * irl * irl_b + 0.5 * rhobar_b;
  Rb.rho += -irr * irr * irr_b + 0.5 * rhobar_b;
  bn_b += 2.0 * bn * bnsq_b;
}

// ---- HLLD (see hlld) with the CT upwind weight ------------------------------
// Given the adjoint of the flux F_b and of the CT weight w_b (the weight is
// clamp(1/2 + F_rho / (2 eps rho_bar c_max), 0, 1) for eps > 0 and piecewise
// constant otherwise), accumulate the adjoints of the two states and of the
// normal field.
__device__ __forceinline__ void hlld_vjp(const FaceState& L, const FaceState& R, double bn, const Gas& g,
                                         double ct_eps, const FaceFlux& Fb_in, double w_b, FaceState& Lb,
                                         FaceState& Rb, double& bn_b) {
  constexpr double kSmall = 1.0e-8;
  // ------------------------------ forward ----------------------------------
  const double bnsq = bn * bn;
  const double irl = frcp(L.rho), irr = frcp(R.rho);
  const double btl = L.bt1 * L.bt1 + L.bt2 * L.bt2, btr = R.bt1 * R.bt1 + R.bt2 * R.bt2;
  const double ptl = L.p + 0.5 * (bnsq + btl), ptr = R.p + 0.5 * (bnsq + btr);
  const double cfl = fast_speed(irl, L.p, bnsq, btl, g.gamma);
  const double cfr = fast_speed(irr, R.p, bnsq, btr, g.gamma);
  const bool cmaxL = cfl >= cfr;
  const double cmax = cmaxL ? cfl : cfr;
  const bool minL = L.vn <= R.vn;
  const double sl = (minL ? L.vn : R.vn) - cmax;
  const bool maxL = L.vn >= R.vn;
  const double sr = (maxL ? L.vn : R.vn) + cmax;
  const bool smaxL = fabs(sl) >= fabs(sr);
  const double smax = smaxL ? fabs(sl) : fabs(sr);
  const double ml = (sl - L.vn) * L.rho;
  const double mr = (sr - R.vn) * R.rho;
  const double iden = frcp(mr - ml);
  const double Q = mr * R.vn - ml * L.vn - ptr + ptl;
  const double sm = Q * iden;
  const double P = mr * ptl - ml * ptr + ml * mr * (R.vn - L.vn);
  const double pts = P * iden;
  const double isl = frcp(sl - sm), isr = frcp(sr - sm);
  const double rsl = ml * isl, rsr = mr * isr;
  const double irql = frsq(rsl), irqr = frsq(rsr);
  const double sqrl = rsl * irql, sqrr = rsr * irqr;
  const double abn = fabs(bn);
  const double ssl = sm - abn * irql;
  const double ssr = sm + abn * irqr;
  const bool useL = (sl > 0.0) || (!(sr < 0.0) && (ssl >= 0.0 || (!(ssr <= 0.0) && sm >= 0.0)));
  const bool star = !(sl > 0.0) && !(sr < 0.0);
  const bool dstar = !(0.5 * bnsq < kSmall * pts);
  const bool dbl = star && !(ssl >= 0.0) && !(ssr <= 0.0) && dstar;
  // single-star transverse states
  const double dL = ml * (sl - sm) - bnsq;
  const bool degL = fabs(dL) < kSmall * pts;
  const double idL = frcp(degL ? 1.0 : dL);
  const double c1L = bn * (sm - L.vn) * idL;
  const double c2L = (ml * (sl - L.vn) - bnsq) * idL;
  const double vt1sl = degL ? L.vt1 : L.vt1 - L.bt1 * c1L;
  const double vt2sl = degL ? L.vt2 : L.vt2 - L.bt2 * c1L;
  const double bt1sl = degL ? L.bt1 : L.bt1 * c2L;
  const double bt2sl = degL ? L.bt2 : L.bt2 * c2L;
  const double dR = mr * (sr - sm) - bnsq;
  const bool degR = fabs(dR) < kSmall * pts;
  const double idR = frcp(degR ? 1.0 : dR);
  const double c1R = bn * (sm - R.vn) * idR;
  const double c2R = (mr * (sr - R.vn) - bnsq) * idR;
  const double vt1sr = degR ? R.vt1 : R.vt1 - R.bt1 * c1R;
  const double vt2sr = degR ? R.vt2 : R.vt2 - R.bt2 * c1R;
  const double bt1sr = degR ? R.bt1 : R.bt1 * c2R;
  const double bt2sr = degR ? R.bt2 : R.bt2 * c2R;
  // double-star state
  const double sgn = bn > 0.0 ? 1.0 : (bn < 0.0 ? -1.0 : 0.0);
  const double isum = frcp(sqrl + sqrr);
  const double A1 = sqrl * vt1sl + sqrr * vt1sr + (bt1sr - bt1sl) * sgn;
  const double A2 = sqrl * vt2sl + sqrr * vt2sr + (bt2sr - bt2sl) * sgn;
  const double C1 = sqrl * bt1sr + sqrr * bt1sl + sqrl * sqrr * (vt1sr - vt1sl) * sgn;
  const double C2 = sqrl * bt2sr + sqrr * bt2sl + sqrl * sqrr * (vt2sr - vt2sl) * sgn;
  const double vt1ss = A1 * isum, vt2ss = A2 * isum, bt1ss = C1 * isum, bt2ss = C2 * isum;
  const double vbss = sm * bn + vt1ss * bt1ss + vt2ss * bt2ss;
  // chosen side
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
  const double N = (s - vn) * en - pt * vn + pts * sm + bn * (vb - vbs);
  const double es = N * is;
  const double side = useL ? -1.0 : 1.0;
  const double ess = es + side * sq * (vbs - vbss) * sgn;
  const double mn = rho * vn;
  double Frho = mn;
  if (star) Frho += s * (rs - rho);

  // ------------------------------ reverse ----------------------------------
  FaceFlux Fb = Fb_in;
  double rhobar_b = 0.0, smax_b = 0.0;
  ct_weight_vjp(Frho, 0.5 * (L.rho + R.rho), smax, ct_eps, w_b, Fb.rho, rhobar_b, smax_b);
  // flux
  double mn_b = 0, vn_b = 0, pt_b = 0, bnsq_b = 0, vt1_b = 0, vt2_b = 0, bt1_b = 0, bt2_b = 0, en_b = 0, vb_b = 0;
  double rho_b = 0, p_b = 0, s_b = 0, rs_b = 0, sm_b = 0, vt1s_b = 0, vt2s_b = 0, es_b = 0, bt1s_b = 0, bt2s_b = 0;
  double ss_b = 0, vt1ss_b = 0, vt2ss_b = 0, ess_b = 0, bt1ss_b = 0, bt2ss_b = 0, sq_b = 0, vbs_b = 0, vbss_b = 0;
  double is_b = 0, pts_b = 0;
  mn_b += Fb.rho + Fb.mn * vn + Fb.mt1 * vt1 + Fb.mt2 * vt2;
  vn_b += Fb.mn * mn + Fb.e * (en + pt) + Fb.bt1 * bt1 + Fb.bt2 * bt2;
  pt_b += Fb.mn + Fb.e * vn;
  bnsq_b -= Fb.mn;
  vt1_b += Fb.mt1 * mn - Fb.bt1 * bn;
  vt2_b += Fb.mt2 * mn - Fb.bt2 * bn;
  bt1_b += -Fb.mt1 * bn + Fb.bt1 * vn;
  bt2_b += -Fb.mt2 * bn + Fb.bt2 * vn;
  bn_b += -Fb.mt1 * bt1 - Fb.mt2 * bt2 - Fb.e * vb - Fb.bt1 * vt1 - Fb.bt2 * vt2;
  en_b += Fb.e * vn;
  vb_b -= Fb.e * bn;
  if (star) {
    s_b += Fb.rho * (rs - rho) + Fb.mn * (rs * sm - mn) + Fb.mt1 * (rs * vt1s - rho * vt1) +
           Fb.mt2 * (rs * vt2s - rho * vt2) + Fb.e * (es - en) + Fb.bt1 * (bt1s - bt1) + Fb.bt2 * (bt2s - bt2);
    rs_b += s * (Fb.rho + Fb.mn * sm + Fb.mt1 * vt1s + Fb.mt2 * vt2s);
    rho_b -= s * (Fb.rho + Fb.mt1 * vt1 + Fb.mt2 * vt2);
    sm_b += s * Fb.mn * rs;
    mn_b -= s * Fb.mn;
    vt1s_b += s * Fb.mt1 * rs;
    vt2s_b += s * Fb.mt2 * rs;
    vt1_b -= s * Fb.mt1 * rho;
    vt2_b -= s * Fb.mt2 * rho;
    es_b += s * Fb.e;
    en_b -= s * Fb.e;
    bt1s_b += s * Fb.bt1;
    bt1_b -= s * Fb.bt1;
    bt2s_b += s * Fb.bt2;
    bt2_b -= s * Fb.bt2;
  }
  if (dbl) {
    ss_b += Fb.mt1 * (rs * vt1ss - rs * vt1s) + Fb.mt2 * (rs * vt2ss - rs * vt2s) + Fb.e * (ess - es) +
            Fb.bt1 * (bt1ss - bt1s) + Fb.bt2 * (bt2ss - bt2s);
    rs_b += ss * (Fb.mt1 * (vt1ss - vt1s) + Fb.mt2 * (vt2ss - vt2s));
    vt1ss_b += ss * Fb.mt1 * rs;
    vt1s_b -= ss * Fb.mt1 * rs;
    vt2ss_b += ss * Fb.mt2 * rs;
    vt2s_b -= ss * Fb.mt2 * rs;
    ess_b += ss * Fb.e;
    es_b -= ss * Fb.e;
    bt1ss_b += ss * Fb.bt1;
    bt1s_b -= ss * Fb.bt1;
    bt2ss_b += ss * Fb.bt2;
    bt2s_b -= ss * Fb.bt2;
  }
  // mn = rho vn
  rho_b += mn_b * vn;
  vn_b += mn_b * rho;
  // ess = es + side sq (vbs - vbss) sgn
  es_b += ess_b;
  sq_b += ess_b * side * (vbs - vbss) * sgn;
  vbs_b += ess_b * side * sq * sgn;
  vbss_b -= ess_b * side * sq * sgn;
  // es = N is
  const double N_b = es_b * is;
  is_b += es_b * N;
  s_b += N_b * en;
  vn_b += -N_b * en - N_b * pt;
  en_b += N_b * (s - vn);
  pt_b -= N_b * vn;
  pts_b += N_b * sm;
  sm_b += N_b * pts;
  bn_b += N_b * (vb - vbs);
  vb_b += N_b * bn;
  vbs_b -= N_b * bn;
  // vbs = sm bn + vt1s bt1s + vt2s bt2s
  sm_b += vbs_b * bn;
  bn_b += vbs_b * sm;
  vt1s_b += vbs_b * bt1s;
  bt1s_b += vbs_b * vt1s;
  vt2s_b += vbs_b * bt2s;
  bt2s_b += vbs_b * vt2s;
  // vb = vn bn + vt1 bt1 + vt2 bt2
  vn_b += vb_b * bn;
  bn_b += vb_b * vn;
  vt1_b += vb_b * bt1;
  bt1_b += vb_b * vt1;
  vt2_b += vb_b * bt2;
  bt2_b += vb_b * vt2;
  // en
  p_b += en_b * g.igm1;
  rho_b += en_b * 0.5 * (vn * vn + vt1 * vt1 + vt2 * vt2);
  vn_b += en_b * rho * vn;
  vt1_b += en_b * rho * vt1;
  vt2_b += en_b * rho * vt2;
  bnsq_b += 0.5 * en_b;
  bt1_b += en_b * bt1;
  bt2_b += en_b * bt2;
  // chosen-side selections -> the two sides
  double sl_b = 0, sr_b = 0, ptl_b = 0, ptr_b = 0, isl_b = 0, isr_b = 0, ssl_b = 0, ssr_b = 0, rsl_b = 0, rsr_b = 0;
  double sqrl_b = 0, sqrr_b = 0, vt1sl_b = 0, vt1sr_b = 0, vt2sl_b = 0, vt2sr_b = 0;
  double bt1sl_b = 0, bt1sr_b = 0, bt2sl_b = 0, bt2sr_b = 0;
  FaceState& C_b = useL ? Lb : Rb;
  C_b.rho += rho_b;
  C_b.vn += vn_b;
  C_b.vt1 += vt1_b;
  C_b.vt2 += vt2_b;
  C_b.p += p_b;
  C_b.bt1 += bt1_b;
  C_b.bt2 += bt2_b;
  if (useL) {
    ptl_b += pt_b; sl_b += s_b; isl_b += is_b; ssl_b += ss_b; rsl_b += rs_b; sqrl_b += sq_b;
    vt1sl_b += vt1s_b; vt2sl_b += vt2s_b; bt1sl_b += bt1s_b; bt2sl_b += bt2s_b;
  } else {
    ptr_b += pt_b; sr_b += s_b; isr_b += is_b; ssr_b += ss_b; rsr_b += rs_b; sqrr_b += sq_b;
    vt1sr_b += vt1s_b; vt2sr_b += vt2s_b; bt1sr_b += bt1s_b; bt2sr_b += bt2s_b;
  }
  // vbss = sm bn + vt1ss bt1ss + vt2ss bt2ss
  sm_b += vbss_b * bn;
  bn_b += vbss_b * sm;
  vt1ss_b += vbss_b * bt1ss;
  bt1ss_b += vbss_b * vt1ss;
  vt2ss_b += vbss_b * bt2ss;
  bt2ss_b += vbss_b * vt2ss;
  // double-star averages
  double isum_b = 0.0;
  {
    const double A1_b = vt1ss_b * isum;
    isum_b += vt1ss_b * A1;
    sqrl_b += A1_b * vt1sl; vt1sl_b += A1_b * sqrl; sqrr_b += A1_b * vt1sr; vt1sr_b += A1_b * sqrr;
    bt1sr_b += A1_b * sgn; bt1sl_b -= A1_b * sgn;
    const double A2_b = vt2ss_b * isum;
    isum_b += vt2ss_b * A2;
    sqrl_b += A2_b * vt2sl; vt2sl_b += A2_b * sqrl; sqrr_b += A2_b * vt2sr; vt2sr_b += A2_b * sqrr;
    bt2sr_b += A2_b * sgn; bt2sl_b -= A2_b * sgn;
    const double C1_b = bt1ss_b * isum;
    isum_b += bt1ss_b * C1;
    sqrl_b += C1_b * (bt1sr + sqrr * (vt1sr - vt1sl) * sgn);
    sqrr_b += C1_b * (bt1sl + sqrl * (vt1sr - vt1sl) * sgn);
    bt1sr_b += C1_b * sqrl; bt1sl_b += C1_b * sqrr;
    vt1sr_b += C1_b * sqrl * sqrr * sgn; vt1sl_b -= C1_b * sqrl * sqrr * sgn;
    const double C2_b = bt2ss_b * isum;
    isum_b += bt2ss_b * C2;
    sqrl_b += C2_b * (bt2sr + sqrr * (vt2sr - vt2sl) * sgn);
    sqrr_b += C2_b * (bt2sl + sqrl * (vt2sr - vt2sl) * sgn);
    bt2sr_b += C2_b * sqrl; bt2sl_b += C2_b * sqrr;
    vt2sr_b += C2_b * sqrl * sqrr * sgn; vt2sl_b -= C2_b * sqrl * sqrr * sgn;
    const double sum_b = -isum * isum * isum_b;
    sqrl_b += sum_b;
    sqrr_b += sum_b;
  }
  // single-star transverse states
  double ml_b = 0, mr_b = 0;
  {
    if (degL) {
      Lb.vt1 += vt1sl_b; Lb.vt2 += vt2sl_b; Lb.bt1 += bt1sl_b; Lb.bt2 += bt2sl_b;
    } else {
      Lb.vt1 += vt1sl_b; Lb.bt1 -= vt1sl_b * c1L;
      Lb.vt2 += vt2sl_b; Lb.bt2 -= vt2sl_b * c1L;
      const double c1_b = -vt1sl_b * L.bt1 - vt2sl_b * L.bt2;
      Lb.bt1 += bt1sl_b * c2L; Lb.bt2 += bt2sl_b * c2L;
      const double c2_b = bt1sl_b * L.bt1 + bt2sl_b * L.bt2;
      bn_b += c1_b * (sm - L.vn) * idL;
      sm_b += c1_b * bn * idL;
      Lb.vn -= c1_b * bn * idL;
      const double id_b = c1_b * bn * (sm - L.vn) + c2_b * (ml * (sl - L.vn) - bnsq);
      ml_b += c2_b * (sl - L.vn) * idL;
      sl_b += c2_b * ml * idL;
      Lb.vn -= c2_b * ml * idL;
      bnsq_b -= c2_b * idL;
      const double d_b = -idL * idL * id_b;
      ml_b += d_b * (sl - sm);
      sl_b += d_b * ml;
      sm_b -= d_b * ml;
      bnsq_b -= d_b;
    }
    if (degR) {
      Rb.vt1 += vt1sr_b; Rb.vt2 += vt2sr_b; Rb.bt1 += bt1sr_b; Rb.bt2 += bt2sr_b;
    } else {
      Rb.vt1 += vt1sr_b; Rb.bt1 -= vt1sr_b * c1R;
      Rb.vt2 += vt2sr_b; Rb.bt2 -= vt2sr_b * c1R;
      const double c1_b = -vt1sr_b * R.bt1 - vt2sr_b * R.bt2;
      Rb.bt1 += bt1sr_b * c2R; Rb.bt2 += bt2sr_b * c2R;
      const double c2_b = bt1sr_b * R.bt1 + bt2sr_b * R.bt2;
      bn_b += c1_b * (sm - R.vn) * idR;
      sm_b += c1_b * bn * idR;
      Rb.vn -= c1_b * bn * idR;
      const double id_b = c1_b * bn * (sm - R.vn) + c2_b * (mr * (sr - R.vn) - bnsq);
      mr_b += c2_b * (sr - R.vn) * idR;
      sr_b += c2_b * mr * idR;
      Rb.vn -= c2_b * mr * idR;
      bnsq_b -= c2_b * idR;
      const double d_b = -idR * idR * id_b;
      mr_b += d_b * (sr - sm);
      sr_b += d_b * mr;
      sm_b -= d_b * mr;
      bnsq_b -= d_b;
    }
  }
  // rotational speeds ssl = sm - |bn| irql, ssr = sm + |bn| irqr
  double irql_b = -ssl_b * abn, irqr_b = ssr_b * abn;
  sm_b += ssl_b + ssr_b;
  bn_b += (-ssl_b * irql + ssr_b * irqr) * sgn;
  // sqrl = rsl irql; irql = rsl^(-1/2)
  rsl_b += sqrl_b * irql;
  irql_b += sqrl_b * rsl;
  rsr_b += sqrr_b * irqr;
  irqr_b += sqrr_b * rsr;
  rsl_b += -0.5 * irql_b * irql * irql * irql;
  rsr_b += -0.5 * irqr_b * irqr * irqr * irqr;
  // rs = m is
  ml_b += rsl_b * isl;
  isl_b += rsl_b * ml;
  mr_b += rsr_b * isr;
  isr_b += rsr_b * mr;
  // is = 1 / (s - sm)
  {
    const double tl = -isl * isl * isl_b;
    sl_b += tl;
    sm_b -= tl;
    const double tr = -isr * isr * isr_b;
    sr_b += tr;
    sm_b -= tr;
  }
  // pts = P iden, sm = Q iden
  double iden_b = 0.0;
  {
    const double P_b = pts_b * iden;
    iden_b += pts_b * P;
    mr_b += P_b * (ptl + ml * (R.vn - L.vn));
    ptl_b += P_b * mr;
    ml_b += P_b * (-ptr + mr * (R.vn - L.vn));
    ptr_b -= P_b * ml;
    Rb.vn += P_b * ml * mr;
    Lb.vn -= P_b * ml * mr;
    const double Q_b = sm_b * iden;
    iden_b += sm_b * Q;
    mr_b += Q_b * R.vn;
    Rb.vn += Q_b * mr;
    ml_b -= Q_b * L.vn;
    Lb.vn -= Q_b * ml;
    ptr_b -= Q_b;
    ptl_b += Q_b;
    const double t = -iden * iden * iden_b;
    mr_b += t;
    ml_b -= t;
  }
  // ml = (sl - L.vn) L.rho, mr = (sr - R.vn) R.rho
  sl_b += ml_b * L.rho;
  Lb.vn -= ml_b * L.rho;
  Lb.rho += ml_b * (sl - L.vn);
  sr_b += mr_b * R.rho;
  Rb.vn -= mr_b * R.rho;
  Rb.rho += mr_b * (sr - R.vn);
  // smax = max(|sl|, |sr|)
  if (smaxL) sl_b += smax_b * (sl >= 0.0 ? 1.0 : -1.0);
  else sr_b += smax_b * (sr >= 0.0 ? 1.0 : -1.0);
  // sl = min(vnL, vnR) - cmax, sr = max(vnL, vnR) + cmax
  double cmax_b = -sl_b + sr_b;
  if (minL) Lb.vn += sl_b;
  else Rb.vn += sl_b;
  if (maxL) Lb.vn += sr_b;
  else Rb.vn += sr_b;
  double cfl_b = cmaxL ? cmax_b : 0.0, cfr_b = cmaxL ? 0.0 : cmax_b;
  // total pressures
  Lb.p += ptl_b;
  Rb.p += ptr_b;
  bnsq_b += 0.5 * (ptl_b + ptr_b);
  double btl_b = 0.5 * ptl_b, btr_b = 0.5 * ptr_b;
  // fast speeds
  double irl_b = 0.0, irr_b = 0.0;
  fast_speed_vjp(irl, L.p, bnsq, btl, g.gamma, cfl_b, irl_b, Lb.p, bnsq_b, btl_b);
  fast_speed_vjp(irr, R.p, bnsq, btr, g.gamma, cfr_b, irr_b, Rb.p, bnsq_b, btr_b);
  Lb.bt1 += 2.0 * L.bt1 * btl_b;
  Lb.bt2 += 2.0 * L.bt2 * btl_b;
  Rb.bt1 += 2.0 * R.bt1 * btr_b;
  Rb.bt2 += 2.0 * R.bt2 * btr_b;
  Lb.rho += -irl * irl * irl_b + 0.5 * rhobar_b;
  Rb.rho += -irr * irr * irr_b + 0.5 * rhobar_b;
  bn_b += 2.0 * bn * bnsq_b;
}

// ---- corner EMF (see corner_emf): partial derivatives ----------------------
// out[0..11] = dE/d(ea0, ea1, eb0, eb1, c00, ca, cb, cab, wa0, wa1, wb0, wb1)
__device__ __forceinline__ void corner_emf_grad(double ea0, double ea1, double eb0, double eb1, double c00,
                                                double ca, double cb, double cab, double wa0, double wa1,
                                                double wb0, double wb1, double* out) {
  out[0] = 0.25 * (1.0 + (1.0 - wb0) + (1.0 - wb1));
  out[1] = 0.25 * (1.0 + wb0 + wb1);
  out[2] = 0.25 * (1.0 + (1.0 - wa0) + (1.0 - wa1));
  out[3] = 0.25 * (1.0 + wa0 + wa1);
  out[4] = -0.25 * ((1.0 - wa0) + (1.0 - wb0));
  out[5] = -0.25 * (wa0 + (1.0 - wb1));
  out[6] = -0.25 * ((1.0 - wa1) + wb0);
  out[7] = -0.25 * (wa1 + wb1);
  out[8] = -0.25 * ((ca - eb1) - (c00 - eb0));
  out[9] = 0.25 * ((eb1 - cab) - (eb0 - cb));
  out[10] = -0.25 * ((cb - ea1) - (c00 - ea0));
  out[11] = 0.25 * ((ea1 - cab) - (ea0 - ca));
}

}  // namespace athmhd
