// kernels_unfused.hip -- one stage of the MHD update as a pipeline of simple
// kernels that exchange data through HBM: primitives, face fluxes per
// direction, corner EMFs, update.  It is the straightforward reading of the
// method (Sec. 3.2: reconstruct -> Riemann solve -> CT -> integrate) and the
// reference point for the fused kernel.
#include "common.hpp"
#include "kernels.hpp"
#include "mhd_math.hpp"

namespace athmhd {

namespace {

constexpr int kThreads = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// cons -> prim on every stored cell; 8 output arrays (rho, v1..3, P, B1..3 cc)
__global__ void __launch_bounds__(kThreads) k_prim(Geo g, double gamma, Floors fl, const double* __restrict__ cons,
                                                  const double* __restrict__ bface, double* __restrict__ w,
                                                  int* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= g.cvar) return;
  const int i = (int)(t % g.N1);
  const int r = (int)(t / g.N1);
  const int j = r % g.N2, k = r / g.N2;
  const double* u = cons + blockIdx.y * g.cblock;
  const double* fb = bface + blockIdx.y * g.fblock;
  double* wb = w + blockIdx.y * 8 * g.cvar;
  const double b1 = 0.5 * (fb[g.f(i, j, k)] + fb[g.f(i + 1, j, k)]);
  const double b2 = 0.5 * (fb[g.fvar + g.f(i, j, k)] + fb[g.fvar + g.f(i, j + 1, k)]);
  const double b3 = 0.5 * (fb[2 * g.fvar + g.f(i, j, k)] + fb[2 * g.fvar + g.f(i, j, k + 1)]);
  const double uc[5] = {u[t], u[g.cvar + t], u[2 * g.cvar + t], u[3 * g.cvar + t], u[4 * g.cvar + t]};
  const double bc[3] = {b1, b2, b3};
  double wc[5];
  const int flags = cell_prim(uc, bc, gamma - 1.0, fl, wc);
#pragma unroll
  for (int v = 0; v < 5; ++v) wb[v * g.cvar + t] = wc[v];
  wb[5 * g.cvar + t] = b1;
  wb[6 * g.cvar + t] = b2;
  wb[7 * g.cvar + t] = b3;
  // ghost cells are periodic images of active ones: count active cells only
  const bool act = i >= g.ng && i < g.ng + g.n1 && j >= g.ng && j < g.ng + g.n2 && k >= g.ng && k < g.ng + g.n3;
  if (act && (flags & 1)) atomicAdd(bad, 1);
  if (act && (flags & 2)) add_floor_count(bad, 1ull);
}

template <int RECON>
__device__ __forceinline__ void recon_pair(const double* __restrict__ q, int s, double& ql, double& qr) {
  // q points at cell c (the face is c-1/2), s is the stride along the direction
  if (RECON == 0) {
    ql = q[-s];
    qr = q[0];
  } else if (RECON == 1) {
    const double a = q[-2 * s], b = q[-s], c = q[0], d = q[s];
    ql = b + 0.5 * vl_slope(a, b, c);
    qr = c - 0.5 * vl_slope(b, c, d);
  } else {
    const double a = q[-3 * s], b = q[-2 * s], c = q[-s], d = q[0], e = q[s], f = q[2 * s];
    const double f0 = ppm_face(a, b, c, d);  // face between b and c
    const double f1 = ppm_face(b, c, d, e);  // face between c and d (this face)
    const double f2 = ppm_face(c, d, e, f);  // face between d and e
    double lm = f0, lp = f1;
    ppm_cell(a, b, c, d, e, lm, lp);  // cell c-1
    double rm = f1, rp = f2;
    ppm_cell(b, c, d, e, f, rm, rp);  // cell c
    ql = lp;
    qr = rm;
  }
}

// ---- characteristic reconstruction (Sec. 3.2.1: C = L W) -------------------
// Face frame, primitives w = (rho, vn, vt1, vt2, P, Bt1, Bt2), normal field bn.
// Columns of R are the right eigenvectors of W_t + A W_x = 0 for the waves
// vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf, normalised after
// Roe & Balsara (1996) (alpha_f, alpha_s from the fast and slow speeds, beta
// along the transverse field, 1/sqrt2 each where it vanishes, alpha_f = 1 and
// alpha_s = 0 where cf = cs), so they stay independent where speeds coincide.
__device__ void char_right(const double* w, double bn, double gamma, double R[7][7]) {
  const double rho = w[0], p = w[4], t1 = w[5], t2 = w[6];
  const double a2 = gamma * p / rho, ca2 = bn * bn / rho, bt2 = t1 * t1 + t2 * t2;
  const double sum = a2 + ca2 + bt2 / rho;
  const double disc = fmax(sum * sum - 4.0 * a2 * ca2, 0.0);
  const double cf2 = 0.5 * (sum + sqrt(disc));
  const double cs2 = cf2 > 0.0 ? a2 * ca2 / cf2 : 0.0;
  double af = 1.0, as = 0.0;
  if (cf2 - cs2 > 0.0) {
    af = sqrt(fmin(1.0, fmax(0.0, (a2 - cs2) / (cf2 - cs2))));
    as = sqrt(fmin(1.0, fmax(0.0, (cf2 - a2) / (cf2 - cs2))));
  }
  double e1 = 0.70710678118654752440, e2 = 0.70710678118654752440;
  if (bt2 > 0.0) {
    const double bt = sqrt(bt2);
    e1 = t1 / bt;
    e2 = t2 / bt;
  }
  const double sg = bn >= 0.0 ? 1.0 : -1.0;
  const double a = sqrt(a2), cf = sqrt(cf2), cs = sqrt(cs2), sr = sqrt(rho), gp = gamma * p;
#pragma unroll
  for (int r = 0; r < 7; ++r)
#pragma unroll
    for (int c = 0; c < 7; ++c) R[r][c] = 0.0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double m = side == 0 ? -1.0 : 1.0;  // left- or right-going
    const int f = side == 0 ? 0 : 6, al = side == 0 ? 1 : 5, sl = side == 0 ? 2 : 4;
    R[0][f] = rho * af;  // fast
    R[1][f] = m * cf * af;
    R[2][f] = -m * as * cs * e1 * sg;
    R[3][f] = -m * as * cs * e2 * sg;
    R[4][f] = gp * af;
    R[5][f] = as * sr * a * e1;
    R[6][f] = as * sr * a * e2;
    R[2][al] = m * e2;  // Alfven
    R[3][al] = -m * e1;
    R[5][al] = -e2 * sg * sr;
    R[6][al] = e1 * sg * sr;
    R[0][sl] = rho * as;  // slow
    R[1][sl] = m * cs * as;
    R[2][sl] = m * af * cf * e1 * sg;
    R[3][sl] = m * af * cf * e2 * sg;
    R[4][sl] = gp * as;
    R[5][sl] = -af * sr * a * e1;
    R[6][sl] = -af * sr * a * e2;
  }
  R[0][3] = 1.0;  // entropy
}

// Projection onto the characteristic variables of the state w0: solves
// R x = B for NR right-hand sides (rows of B, replaced by the solutions) by
// Gaussian elimination with partial pivoting.  Rows are exchanged by selects
// so that every index is a compile-time constant and the system stays in
// registers.
template <int NR>
__device__ __forceinline__ void char_project(const double* w0, double bn, double gamma, double (&B)[NR][7]) {
  double M[7][7 + NR];
  {
    double R[7][7];
    char_right(w0, bn, gamma, R);
#pragma unroll
    for (int r = 0; r < 7; ++r) {
#pragma unroll
      for (int c = 0; c < 7; ++c) M[r][c] = R[r][c];
#pragma unroll
      for (int n = 0; n < NR; ++n) M[r][7 + n] = B[n][r];
    }
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    // the largest entry of column c (rows c..6) to row c
#pragma unroll
    for (int r = c + 1; r < 7; ++r) {
      const bool sw = fabs(M[r][c]) > fabs(M[c][c]);
#pragma unroll
      for (int k = c; k < 7 + NR; ++k) {
        const double a = M[c][k], b = M[r][k];
        M[c][k] = sw ? b : a;
        M[r][k] = sw ? a : b;
      }
    }
    const double inv = 1.0 / M[c][c];
#pragma unroll
    for (int r = c + 1; r < 7; ++r) {
      const double f = M[r][c] * inv;
#pragma unroll
      for (int k = c + 1; k < 7 + NR; ++k) M[r][k] -= f * M[c][k];
    }
  }
#pragma unroll
  for (int c = 6; c >= 0; --c) {
    const double inv = 1.0 / M[c][c];
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      double v = M[c][7 + n];
#pragma unroll
      for (int k = c + 1; k < 7; ++k) v -= M[c][k] * B[n][k];
      B[n][c] = v * inv;
    }
  }
}

// w0 + R d for the characteristic offset d
__device__ __forceinline__ void char_back(const double* w0, double bn, double gamma, const double* d, double* out) {
  double R[7][7];
  char_right(w0, bn, gamma, R);
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) v += R[j][k] * d[k];
    out[j] = w0[j] + v;
  }
}

// PLM edges of cell w0 on characteristic variables: the one-sided differences
// projected with L, van Leer-limited per wave family, projected back with R.
__device__ void char_plm(const double* wm, const double* w0, const double* wp, double bn, double gamma,
                         double* left, double* right) {
  double B[2][7];
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    B[0][r] = w0[r] - wm[r];
    B[1][r] = wp[r] - w0[r];
  }
  char_project<2>(w0, bn, gamma, B);
  double dl[7], dr[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double pr = B[0][k] * B[1][k];
    const double dc = pr > 0.0 ? 2.0 * pr / (B[0][k] + B[1][k]) : 0.0;
    dl[k] = -0.5 * dc;
    dr[k] = 0.5 * dc;
  }
  char_back(w0, bn, gamma, dl, left);
  char_back(w0, bn, gamma, dr, right);
}

// PPM edges of the middle cell of the stencil st[0..4] on characteristic
// variables: the differences from the middle cell projected with L, the
// limited parabola per wave family, the edge offsets projected back with R.
__device__ void char_ppm(const double (&st)[5][7], double bn, double gamma, double* left, double* right) {
  double B[4][7];
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    B[0][r] = st[0][r] - st[2][r];
    B[1][r] = st[1][r] - st[2][r];
    B[2][r] = st[3][r] - st[2][r];
    B[3][r] = st[4][r] - st[2][r];
  }
  char_project<4>(st[2], bn, gamma, B);
  double cl[7], cr[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double q[5] = {B[0][k], B[1][k], 0.0, B[2][k], B[3][k]};
    cell_edges<2>(q, cl[k], cr[k]);
  }
  char_back(st[2], bn, gamma, cl, left);
  char_back(st[2], bn, gamma, cr, right);
}

// Fluxes through the faces normal to D: normal index [ng, ng+n_D], transverse
// indices [ng-1, ng+n_t] (one extra ring for the corner EMFs).  CHAR: PLM or
// PPM on characteristic variables.
template <int D, int RECON, int RS, bool CHAR>
__global__ void __launch_bounds__(kThreads) k_flux(Geo g, Gas gas, double ct_eps, Floors fl,
                                                  const double* __restrict__ w, const double* __restrict__ bface,
                                                  double* __restrict__ fo, int* __restrict__ bad) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int e1 = D == 0 ? g.n1 + 1 : g.n1 + 2;
  const int e2 = D == 1 ? g.n2 + 1 : g.n2 + 2;
  const int e3 = D == 2 ? g.n3 + 1 : g.n3 + 2;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)e1 * e2 * e3) return;
  const int i = (int)(t % e1) + (D == 0 ? g.ng : g.ng - 1);
  const int r = (int)(t / e1);
  const int j = r % e2 + (D == 1 ? g.ng : g.ng - 1);
  const int k = r / e2 + (D == 2 ? g.ng : g.ng - 1);
  const double* wb = w + blockIdx.y * 8 * g.cvar;
  const double* fb = bface + blockIdx.y * g.fblock;
  double* ob = fo + blockIdx.y * 8 * g.fvar;
  const int s = D == 0 ? 1 : (D == 1 ? g.N1 : g.N1 * g.N2);
  const int q = g.c(i, j, k);
  FaceState L, R;
  if (CHAR && RECON == 1) {
    // cells c-2 .. c+1 in the face frame; right edge of c-1, left edge of c
    const int vi[7] = {0, 1 + D, 1 + T1, 1 + T2, 4, 5 + T1, 5 + T2};
    double w[4][7];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int n = 0; n < 7; ++n) w[o][n] = wb[vi[n] * g.cvar + q + (o - 2) * s];
    const double bnm = wb[(5 + D) * g.cvar + q - s], bn0 = wb[(5 + D) * g.cvar + q];
    double lm[7], rm[7], l0[7], r0[7];
    char_plm(w[0], w[1], w[2], bnm, gas.gamma, lm, rm);
    char_plm(w[1], w[2], w[3], bn0, gas.gamma, l0, r0);
    L = FaceState{rm[0], rm[1], rm[2], rm[3], rm[4], rm[5], rm[6]};
    R = FaceState{l0[0], l0[1], l0[2], l0[3], l0[4], l0[5], l0[6]};
  } else if (CHAR && RECON == 2) {
    // cells c-3 .. c+2; right edge of c-1 (stencil c-3 .. c+1), left edge of c
    const int vi[7] = {0, 1 + D, 1 + T1, 1 + T2, 4, 5 + T1, 5 + T2};
    double lm[7], rm[7], l0[7], r0[7];
    {
      double st[5][7];
#pragma unroll
      for (int o = 0; o < 5; ++o)
#pragma unroll
        for (int n = 0; n < 7; ++n) st[o][n] = wb[vi[n] * g.cvar + q + (o - 3) * s];
      char_ppm(st, wb[(5 + D) * g.cvar + q - s], gas.gamma, lm, rm);
    }
    {
      double st[5][7];
#pragma unroll
      for (int o = 0; o < 5; ++o)
#pragma unroll
        for (int n = 0; n < 7; ++n) st[o][n] = wb[vi[n] * g.cvar + q + (o - 2) * s];
      char_ppm(st, wb[(5 + D) * g.cvar + q], gas.gamma, l0, r0);
    }
    L = FaceState{rm[0], rm[1], rm[2], rm[3], rm[4], rm[5], rm[6]};
    R = FaceState{l0[0], l0[1], l0[2], l0[3], l0[4], l0[5], l0[6]};
  } else {
    recon_pair<RECON>(wb + q, s, L.rho, R.rho);
    recon_pair<RECON>(wb + (1 + D) * g.cvar + q, s, L.vn, R.vn);
    recon_pair<RECON>(wb + (1 + T1) * g.cvar + q, s, L.vt1, R.vt1);
    recon_pair<RECON>(wb + (1 + T2) * g.cvar + q, s, L.vt2, R.vt2);
    recon_pair<RECON>(wb + 4 * g.cvar + q, s, L.p, R.p);
    recon_pair<RECON>(wb + (5 + T1) * g.cvar + q, s, L.bt1, R.bt1);
    recon_pair<RECON>(wb + (5 + T2) * g.cvar + q, s, L.bt2, R.bt2);
  }
  const int fi = g.f(i, j, k);
  const double bn = fb[D * g.fvar + fi];
  if (fl.on()) {
    const int n = floor_state(L, fl) + floor_state(R, fl);
    if (n) add_floor_count(bad, (unsigned long long)n);
  }
  FaceFlux F;
  double smax;
  riemann_flux<RS>(L, R, bn, gas, F, smax);
  ob[fi] = F.rho;
  ob[(1 + D) * g.fvar + fi] = F.mn;
  ob[(1 + T1) * g.fvar + fi] = F.mt1;
  ob[(1 + T2) * g.fvar + fi] = F.mt2;
  ob[4 * g.fvar + fi] = F.e;
  // E = -v x B: flux of B_t1 along D is -E_t2, flux of B_t2 is +E_t1
  ob[5 * g.fvar + fi] = F.bt2;   // EMF component T1
  ob[6 * g.fvar + fi] = -F.bt1;  // EMF component T2
  ob[7 * g.fvar + fi] = ct_weight(F.rho, 0.5 * (L.rho + R.rho), smax, ct_eps);
}

// Corner EMFs on every edge that bounds an active face.
__global__ void __launch_bounds__(kThreads) k_corner(Geo g, const double* __restrict__ w,
                                                    const double* __restrict__ f0, const double* __restrict__ f1,
                                                    const double* __restrict__ f2, double* __restrict__ edge) {
  const int e1 = g.n1 + 1, e2 = g.n2 + 1, e3 = g.n3 + 1;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)e1 * e2 * e3) return;
  const int i = (int)(t % e1) + g.ng;
  const int r = (int)(t / e1);
  const int j = r % e2 + g.ng, k = r / e2 + g.ng;
  const int b = blockIdx.y;
  const double* wb = w + b * 8 * g.cvar;
  const double* fd[3] = {f0 + b * 8 * g.fvar, f1 + b * 8 * g.fvar, f2 + b * 8 * g.fvar};
  double* eb = edge + b * 3 * g.fvar;
  const int idx[3] = {i, j, k};
  const int last[3] = {g.ng + g.n1 - 1, g.ng + g.n2 - 1, g.ng + g.n3 - 1};
  const int cstr[3] = {1, g.N1, g.N1 * g.N2};
  const int fstr[3] = {1, g.F1, g.F1 * g.F2};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    if (idx[e] > last[e]) continue;
    const int a = (e + 1) % 3, bb = (e + 2) % 3;
    const int fc = g.f(i, j, k), qc = g.c(i, j, k);
    const int fa = fstr[a], fbs = fstr[bb];
    const int ca = cstr[a], cb = cstr[bb];
    const double* Fa = fd[a];
    const double* Fb = fd[bb];
    // face-a EMF of component e is slot 6 (component T2 of a), face-b is slot 5
    const double ea0 = Fa[6 * g.fvar + fc], ea1 = Fa[6 * g.fvar + fc - fbs];
    const double eb0 = Fb[5 * g.fvar + fc], eb1 = Fb[5 * g.fvar + fc - fa];
    const double wa0 = Fa[7 * g.fvar + fc], wa1 = Fa[7 * g.fvar + fc - fbs];
    const double wb0 = Fb[7 * g.fvar + fc], wb1 = Fb[7 * g.fvar + fc - fa];
    // cell EMF component e: -(v_a B_b - v_b B_a)
    auto ecell = [&](int q) {
      return -(wb[(1 + a) * g.cvar + q] * wb[(5 + bb) * g.cvar + q] - wb[(1 + bb) * g.cvar + q] * wb[(5 + a) * g.cvar + q]);
    };
    const double c00 = ecell(qc), cA = ecell(qc - ca), cB = ecell(qc - cb), cAB = ecell(qc - ca - cb);
    eb[e * g.fvar + fc] = corner_emf(ea0, ea1, eb0, eb1, c00, cA, cB, cAB, wa0, wa1, wb0, wb1);
  }
}

// out = g0 x + g1 un + bdt L(x) on the active cells and their lower faces;
// bdt = beta * (*dt_dev) when dt_dev is not NULL (a step replayed from a
// graph reads its dt on the device), else cf.bdt.  b1_lo: the first x1 index
// whose B1 face is written (ng, or ng + 1 for a block whose lower x1 boundary
// faces another block owns).
__global__ void __launch_bounds__(kThreads) k_update(Geo g, StageCoef cf, const double* dt_dev, double beta, int b1_lo,
                                                    const double* __restrict__ xc,
                                                    const double* __restrict__ xb, const double* unc,
                                                    const double* unb, const double* __restrict__ f0,
                                                    const double* __restrict__ f1, const double* __restrict__ f2,
                                                    const double* __restrict__ edge, double* outc, double* outb) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int64_t)g.n1 * g.n2 * g.n3) return;
  const int i = g.ng + (int)(t % g.n1);
  const int r = (int)(t / g.n1);
  const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
  const int b = blockIdx.y;
  const int q = g.c(i, j, k), fc = g.f(i, j, k);
  const int s2 = g.F1, s3 = g.F1 * g.F2;
  const double bdt = dt_dev ? beta * *dt_dev : cf.bdt;
  const double* F0 = f0 + b * 8 * g.fvar;
  const double* F1 = f1 + b * 8 * g.fvar;
  const double* F2 = f2 + b * 8 * g.fvar;
  const double i1 = 1.0 / g.dx1, i2 = 1.0 / g.dx2, i3 = 1.0 / g.dx3;
  const double* x = xc + b * g.cblock;
  const double* un = unc + b * g.cblock;
  double* o = outc + b * g.cblock;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const int64_t fv = v * g.fvar + fc;
    const double div = (F0[fv + 1] - F0[fv]) * i1 + (F1[fv + s2] - F1[fv]) * i2 + (F2[fv + s3] - F2[fv]) * i3;
    const int64_t cv = v * g.cvar + q;
    o[cv] = cf.g0 * x[cv] + cf.g1 * un[cv] - bdt * div;
  }
  const double* E = edge + b * 3 * g.fvar;
  const double* xbb = xb + b * g.fblock;
  const double* unbb = unb + b * g.fblock;
  double* ob = outb + b * g.fblock;
  const double* E1 = E;
  const double* E2 = E + g.fvar;
  const double* E3 = E + 2 * g.fvar;
  // dB1 = -[(E3(j+1) - E3(j))/dx2 - (E2(k+1) - E2(k))/dx3]
  const double c1 = (E3[fc + s2] - E3[fc]) * i2 - (E2[fc + s3] - E2[fc]) * i3;
  // dB2 = -[(E1(k+1) - E1(k))/dx3 - (E3(i+1) - E3(i))/dx1]
  const double c2 = (E1[fc + s3] - E1[fc]) * i3 - (E3[fc + 1] - E3[fc]) * i1;
  // dB3 = -[(E2(i+1) - E2(i))/dx1 - (E1(j+1) - E1(j))/dx2]
  const double c3 = (E2[fc + 1] - E2[fc]) * i1 - (E1[fc + s2] - E1[fc]) * i2;
  if (i >= b1_lo) ob[fc] = cf.g0 * xbb[fc] + cf.g1 * unbb[fc] - bdt * c1;
  ob[g.fvar + fc] = cf.g0 * xbb[g.fvar + fc] + cf.g1 * unbb[g.fvar + fc] - bdt * c2;
  ob[2 * g.fvar + fc] = cf.g0 * xbb[2 * g.fvar + fc] + cf.g1 * unbb[2 * g.fvar + fc] - bdt * c3;
}

template <int D, int RECON, bool CHAR>
hipError_t flux_rs(const Geo& g, const Gas& gas, int rs, double ct_eps, const Floors& fl, const double* w,
                   const double* xb, double* fo, int* bad, int nb, hipStream_t s) {
  const int64_t n = (int64_t)(D == 0 ? g.n1 + 1 : g.n1 + 2) * (D == 1 ? g.n2 + 1 : g.n2 + 2) *
                    (D == 2 ? g.n3 + 1 : g.n3 + 2);
  if (rs == 1)
    hipLaunchKernelGGL((k_flux<D, RECON, 1, CHAR>), dim3(grid_for(n), nb), dim3(kThreads), 0, s, g, gas, ct_eps, fl,
                       w, xb, fo, bad);
  else if (rs == 2)
    hipLaunchKernelGGL((k_flux<D, RECON, 2, CHAR>), dim3(grid_for(n), nb), dim3(kThreads), 0, s, g, gas, ct_eps, fl,
                       w, xb, fo, bad);
  else
    hipLaunchKernelGGL((k_flux<D, RECON, 0, CHAR>), dim3(grid_for(n), nb), dim3(kThreads), 0, s, g, gas, ct_eps, fl,
                       w, xb, fo, bad);
  return hipGetLastError();
}

template <int D>
hipError_t flux_dir(const Geo& g, const Gas& gas, int recon, bool charac, int rs, double ct_eps, const Floors& fl,
                    const double* w, const double* xb, double* fo, int* bad, int nb, hipStream_t s) {
  if (recon == 0) return flux_rs<D, 0, false>(g, gas, rs, ct_eps, fl, w, xb, fo, bad, nb, s);
  if (recon == 1 && charac) return flux_rs<D, 1, true>(g, gas, rs, ct_eps, fl, w, xb, fo, bad, nb, s);
  if (recon == 1) return flux_rs<D, 1, false>(g, gas, rs, ct_eps, fl, w, xb, fo, bad, nb, s);
  if (charac) return flux_rs<D, 2, true>(g, gas, rs, ct_eps, fl, w, xb, fo, bad, nb, s);
  return flux_rs<D, 2, false>(g, gas, rs, ct_eps, fl, w, xb, fo, bad, nb, s);
}

}  // namespace

hipError_t launch_fluxes_unfused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                                 const double* xb, int nb, UnfusedScratch& scr, const Floors& fl, int* bad,
                                 bool charac, hipStream_t s) {
  Gas gas{gamma, gamma - 1.0, 1.0 / (gamma - 1.0)};
  hipLaunchKernelGGL(k_prim, dim3(grid_for(g.cvar), nb), dim3(kThreads), 0, s, g, gamma, fl, xc, xb, scr.w, bad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int d = 0; d < 3; ++d) {
    e = d == 0   ? flux_dir<0>(g, gas, recon, charac, rs, ct_eps, fl, scr.w, xb, scr.face[0], bad, nb, s)
        : d == 1 ? flux_dir<1>(g, gas, recon, charac, rs, ct_eps, fl, scr.w, xb, scr.face[1], bad, nb, s)
                 : flux_dir<2>(g, gas, recon, charac, rs, ct_eps, fl, scr.w, xb, scr.face[2], bad, nb, s);
    if (e != hipSuccess) return e;
  }
  const int64_t ne = (int64_t)(g.n1 + 1) * (g.n2 + 1) * (g.n3 + 1);
  hipLaunchKernelGGL(k_corner, dim3(grid_for(ne), nb), dim3(kThreads), 0, s, g, scr.w, scr.face[0], scr.face[1],
                     scr.face[2], scr.edge);
  return hipGetLastError();
}

hipError_t launch_update_unfused(const Geo& g, const double* xc, const double* xb, const double* unc,
                                 const double* unb, double* outc, double* outb, StageCoef coef, const double* dt_dev,
                                 double beta, int nb, const UnfusedScratch& scr, hipStream_t s, bool keep_x1_lower) {
  const int64_t na = (int64_t)g.n1 * g.n2 * g.n3;
  const int b1_lo = keep_x1_lower ? g.ng + 1 : g.ng;
  hipLaunchKernelGGL(k_update, dim3(grid_for(na), nb), dim3(kThreads), 0, s, g, coef, dt_dev, beta, b1_lo, xc, xb,
                     unc, unb, scr.face[0], scr.face[1], scr.face[2], scr.edge, outc, outb);
  return hipGetLastError();
}

hipError_t launch_stage_unfused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                                const double* xb, const double* unc, const double* unb, double* outc,
                                double* outb, StageCoef coef, const double* dt_dev, double beta, int nb,
                                UnfusedScratch& scr, const Floors& fl, int* bad, bool charac, hipStream_t s) {
  hipError_t e = launch_fluxes_unfused(g, gamma, recon, rs, ct_eps, xc, xb, nb, scr, fl, bad, charac, s);
  if (e != hipSuccess) return e;
  return launch_update_unfused(g, xc, xb, unc, unb, outc, outb, coef, dt_dev, beta, nb, scr, s);
}

}  // namespace athmhd
