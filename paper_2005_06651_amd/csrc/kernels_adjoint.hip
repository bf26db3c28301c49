// kernels_adjoint.hip -- reverse-mode derivative of one stage's spatial
// operator on periodic blocks: given the stage input X = (U, B) and a
// cotangent v, accumulate  out += scale * J_L(X)^T v,  where L is the
// right-hand side of the 2S update (Eq. (rk-2s)): minus the flux divergence
// for U and minus the CT curl of the corner EMFs for the face field.
//
// The independent variables of a periodic block are its active cells and the
// lower face of each active cell in each direction (the upper face of the
// last cell is the periodic image of the first).  All scratch arrays are
// indexed by active cell (x1 fastest, no ghosts) and every neighbour index
// wraps periodically, as the forward stage kernel reads periodic images.
//
// Every kernel gathers (each output element is written by exactly one
// thread, in a fixed order), so the result is deterministic.  Pipeline:
//   1. k_adj_prim       primitives W and cell EMFs -v x B of the stage input
//   2. k_adj_face_fwd   per direction: face EMFs and CT upwind weights
//   3. (in k_adj_prim)  corner-EMF cotangents: transpose of the CT curl
//   4. k_adj_face_bwd   per direction: flux / face-EMF / weight cotangents
//                       gathered from the neighbouring cells and edges, then
//                       the Riemann solver's reverse sweep -> cotangents of
//                       the reconstructed states and of the normal field
//   5-6. k_adj_cell     per cell: reverse of the reconstruction along each
//                       direction into the primitive cotangents, the
//                       cell-EMF cotangents and the reverse of cons -> prim
//   7. k_adj_bface      face-field cotangents (normal field of the Riemann
//                       problems and the two cell-centred averages)
// Steps 6 and 7 write the stage's output cotangent O = g0 V + scale J^T V and
// the running sum Z of the U^n terms (Z += g1 V) of the 2S scheme.
#include "common.hpp"
#include "kernels.hpp"
#include "mhd_adjoint.hpp"

namespace athmhd {

namespace {

constexpr int kT = 256;
inline unsigned grid_of(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

// Slots of the per-block scratch (each nc doubles, nc = active cells).
enum : int {
  S_W = 0,     // 8: rho, v1, v2, v3, p, B1cc, B2cc, B3cc
  S_CE = 8,    // 3: cell EMF components
  S_FE = 11,   // 3 x 3: per face direction (EMF of component t1, of t2, weight)
  S_EB = 20,   // 3: corner-EMF cotangents
  S_LB = 23,   // 3 x 7: cotangents of the left states of the faces, per direction
  S_RB = 44,   // 3 x 7: of the right states
  S_BN = 65,   // 3: cotangent of the normal field of the Riemann problems
  S_BC = 68,   // 3: cotangent of the cell-centred field
  S_TOTAL = 71
};

struct Adj {
  Geo g;          // padded layout of the caller's arrays
  int n[3];       // active cells per direction
  int st[3];      // strides of the active-only arrays: 1, n1, n1 n2
  int64_t nc;     // active cells per block (< 2^31; 64-bit for slot offsets)
  double idx[3];  // 1 / dx
  Gas gas;
  double ct_eps;
};

__device__ __forceinline__ int wrapn(int t, int n) {
  while (t < 0) t += n;
  while (t >= n) t -= n;
  return t;
}

struct Cell {
  int x[3];
  int t;  // active index
};

__device__ __forceinline__ Cell cell_of(const Adj& a, int t) {
  Cell c;
  c.t = t;
  c.x[0] = t % a.n[0];
  const int r = t / a.n[0];
  c.x[1] = r % a.n[1];
  c.x[2] = r / a.n[1];
  return c;
}

// offset (in active-array elements) of the periodic neighbour o cells away
// from c along direction d
__device__ __forceinline__ int sh(const Adj& a, const Cell& c, int d, int o) {
  return (wrapn(c.x[d] + o, a.n[d]) - c.x[d]) * a.st[d];
}

// active index of c shifted along one direction, and along two directions
__device__ __forceinline__ int at1(const Adj& a, const Cell& c, int d, int o) { return c.t + sh(a, c, d, o); }
__device__ __forceinline__ int at2(const Adj& a, const Cell& c, int d, int o, int e, int p) {
  return c.t + sh(a, c, d, o) + sh(a, c, e, p);
}

// padded index of the (wrapped) active cell / lower face
__device__ __forceinline__ int pc(const Adj& a, const Cell& c) {
  return a.g.c(a.g.ng + c.x[0], a.g.ng + c.x[1], a.g.ng + c.x[2]);
}
__device__ __forceinline__ int pf(const Adj& a, const Cell& c, int d, int o) {
  int x[3] = {c.x[0], c.x[1], c.x[2]};
  x[d] = wrapn(x[d] + o, a.n[d]);
  return a.g.f(a.g.ng + x[0], a.g.ng + x[1], a.g.ng + x[2]);
}

// ---- 1. primitives and cell EMFs -------------------------------------------
// (also step 3: the corner-EMF cotangents, which need only the cotangent V)
__global__ void __launch_bounds__(kT) k_adj_prim(Adj a, const double* __restrict__ xc,
                                                const double* __restrict__ xb, const double* __restrict__ V,
                                                double* __restrict__ scr) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  const double* u = xc + blockIdx.y * a.g.cblock;
  const double* fb = xb + blockIdx.y * a.g.fblock;
  double* s = scr + blockIdx.y * (S_TOTAL * a.nc);
  const Cell c = cell_of(a, t);
  {
    const double* v = V + blockIdx.y * (8 * a.nc);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int ea = (e + 1) % 3, eb = (e + 2) % 3;
      const double* va = v + (5 + ea) * a.nc;
      const double* vb = v + (5 + eb) * a.nc;
      s[(S_EB + e) * a.nc + t] =
          (va[t] - va[at1(a, c, eb, -1)]) * a.idx[eb] - (vb[t] - vb[at1(a, c, ea, -1)]) * a.idx[ea];
    }
  }
  const int q = pc(a, c);
  double b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) b[d] = 0.5 * (fb[d * a.g.fvar + pf(a, c, d, 0)] + fb[d * a.g.fvar + pf(a, c, d, 1)]);
  const double rho = u[q], ir = 1.0 / rho;
  const double v[3] = {u[a.g.cvar + q] * ir, u[2 * a.g.cvar + q] * ir, u[3 * a.g.cvar + q] * ir};
  const double p = a.gas.gm1 * (u[4 * a.g.cvar + q] - 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                                0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
  s[(S_W + 0) * a.nc + t] = rho;
  s[(S_W + 4) * a.nc + t] = p;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    s[(S_W + 1 + d) * a.nc + t] = v[d];
    s[(S_W + 5 + d) * a.nc + t] = b[d];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int ea = (e + 1) % 3, eb = (e + 2) % 3;
    s[(S_CE + e) * a.nc + t] = -(v[ea] * b[eb] - v[eb] * b[ea]);
  }
}

// reconstructed left/right value of primitive slot w at the lower D-face of c
template <int RECON>
__device__ __forceinline__ void recon_lr(const Adj& a, const double* __restrict__ wv, const Cell& c, int D,
                                         double& ql, double& qr) {
  const double q0 = wv[at1(a, c, D, -1)], q1 = wv[at1(a, c, D, 0)];
  if (RECON == 0) {
    ql = q0;
    qr = q1;
  } else {
    const double qm = wv[at1(a, c, D, -2)], q2 = wv[at1(a, c, D, 1)];
    ql = q0 + 0.5 * vl_slope(qm, q0, q1);
    qr = q1 - 0.5 * vl_slope(q0, q1, q2);
  }
}

// primitive slot (in W) of the 7 reconstructed quantities of a D-face:
// rho, vn, vt1, vt2, p, bt1, bt2
__device__ __forceinline__ int wslot(int D, int m) {
  const int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  switch (m) {
    case 0: return 0;
    case 1: return 1 + D;
    case 2: return 1 + T1;
    case 3: return 1 + T2;
    case 4: return 4;
    case 5: return 5 + T1;
    default: return 5 + T2;
  }
}

template <int RECON>
__device__ __forceinline__ void face_states(const Adj& a, const double* __restrict__ s, const Cell& c, int D,
                                            FaceState& L, FaceState& R) {
  double l[7], r[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) recon_lr<RECON>(a, s + (S_W + wslot(D, m)) * a.nc, c, D, l[m], r[m]);
  L = FaceState{l[0], l[1], l[2], l[3], l[4], l[5], l[6]};
  R = FaceState{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
}

// ---- 2. face EMFs and upwind weights ---------------------------------------
template <int D, int RECON, int RS>
__global__ void __launch_bounds__(kT) k_adj_face_fwd(Adj a, const double* __restrict__ xb, double* __restrict__ scr) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  const double* fb = xb + blockIdx.y * a.g.fblock;
  double* s = scr + blockIdx.y * (S_TOTAL * a.nc);
  const Cell c = cell_of(a, t);
  FaceState L, R;
  face_states<RECON>(a, s, c, D, L, R);
  const double bn = fb[D * a.g.fvar + pf(a, c, D, 0)];
  FaceFlux F;
  double smax;
  if (RS == 1) hlld(L, R, bn, a.gas, F, smax);
  else hlle(L, R, bn, a.gas, F, smax);
  s[(S_FE + 3 * D + 0) * a.nc + t] = F.bt2;   // EMF of component t1
  s[(S_FE + 3 * D + 1) * a.nc + t] = -F.bt1;  // EMF of component t2
  s[(S_FE + 3 * D + 2) * a.nc + t] = ct_weight(F.rho, 0.5 * (L.rho + R.rho), smax, a.ct_eps);
}

// ---- 3. corner-EMF cotangents (computed in k_adj_prim) ---------------------
// The CT update of the face field is minus the curl of the corner EMFs; its
// transpose gives, for the edge of component e at the lower corner of c
// (a = e+1, b = e+2 cyclic):
//   Ebar_e = (v_Ba[c] - v_Ba[c - b]) / dx_b - (v_Bb[c] - v_Bb[c - a]) / dx_a

// ---- 4. face cotangents and the Riemann solver's reverse sweep ------------
template <int D, int RECON, int RS>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(2))) k_adj_face_bwd(Adj a, const double* __restrict__ xb,
                                                    const double* __restrict__ V, double* __restrict__ scr) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  const double* fb = xb + blockIdx.y * a.g.fblock;
  const double* v = V + blockIdx.y * (8 * a.nc);
  double* s = scr + blockIdx.y * (S_TOTAL * a.nc);
  const Cell c = cell_of(a, t);
  const double* EB = s + S_EB * a.nc;
  const double* CE = s + S_CE * a.nc;
  const double* wT1 = s + (S_FE + 3 * T1 + 2) * a.nc;  // weights of the t1-faces
  const double* wT2 = s + (S_FE + 3 * T2 + 2) * a.nc;  // weights of the t2-faces
  const double* e5T1 = s + (S_FE + 3 * T1 + 0) * a.nc;  // t1-faces, EMF of their t1 component (= T2)
  const double* e6T2 = s + (S_FE + 3 * T2 + 1) * a.nc;  // t2-faces, EMF of their t2 component (= T1)
  const int cm = at1(a, c, D, -1);

  // (a) EMF of component T2 carried by this face (edge component e = T2,
  //     edge directions a = D, b = T1): ea0 of the edge at c, ea1 of the edge
  //     at c + T1.
  const int cp1 = at1(a, c, T1, 1);
  const int cp1m = at2(a, c, T1, 1, D, -1);
  const double e6_b = EB[T2 * a.nc + t] * 0.25 * (3.0 - wT1[t] - wT1[cm]) +
                      EB[T2 * a.nc + cp1] * 0.25 * (1.0 + wT1[cp1] + wT1[cp1m]);
  // (b) EMF of component T1 (edge component T1, edge directions a = T2,
  //     b = D): eb0 of the edge at c, eb1 of the edge at c + T2.
  const int cp2 = at1(a, c, T2, 1);
  const int cp2m = at2(a, c, T2, 1, D, -1);
  const double e5_b = EB[T1 * a.nc + t] * 0.25 * (3.0 - wT2[t] - wT2[cm]) +
                      EB[T1 * a.nc + cp2] * 0.25 * (1.0 + wT2[cp2] + wT2[cp2m]);
  // (c) upwind weight: wa0 / wa1 of the T2-edges at c and c + T1, wb0 / wb1
  //     of the T1-edges at c and c + T2.
  double w_b = 0.0;
  {
    const double* ce = CE + T2 * a.nc;
    // edge x = c: eb0 = e5T1[x], eb1 = e5T1[x - D]; c00, ca = x - D, cb = x - T1, cab
    {
      const double eb0 = e5T1[t], eb1 = e5T1[cm];
      const double c00 = ce[t], ca = ce[cm];
      w_b += EB[T2 * a.nc + t] * (-0.25) * ((ca - eb1) - (c00 - eb0));
    }
    // edge x = c + T1 (this face is its wa1): eb0 = e5T1[x], eb1 = e5T1[x - D]
    {
      const double eb0 = e5T1[cp1], eb1 = e5T1[cp1m];
      const double cb = ce[t], cab = ce[cm];  // x - T1 = c, x - D - T1 = c - D
      w_b += EB[T2 * a.nc + cp1] * 0.25 * ((eb1 - cab) - (eb0 - cb));
    }
  }
  {
    const double* ce = CE + T1 * a.nc;
    // edge x = c (this face is its wb0): ea0 = e6T2[x], ea1 = e6T2[x - D];
    // c00 = ce[x], ca = ce[x - T2], cb = ce[x - D]
    {
      const double ea0 = e6T2[t], ea1 = e6T2[cm];
      const double c00 = ce[t], cb = ce[cm];
      w_b += EB[T1 * a.nc + t] * (-0.25) * ((cb - ea1) - (c00 - ea0));
    }
    // edge x = c + T2 (this face is its wb1): ca = ce[x - T2] = ce[c],
    // cab = ce[x - T2 - D] = ce[c - D]
    {
      const double ea0 = e6T2[cp2], ea1 = e6T2[cp2m];
      const double ca = ce[t], cab = ce[cm];
      w_b += EB[T1 * a.nc + cp2] * 0.25 * ((ea1 - cab) - (ea0 - ca));
    }
  }
  // (d) flux cotangents: the face is the upper face of c - D and the lower
  //     face of c, so dL/dF = (v[c] - v[c - D]) / dx_D per conserved variable
  const double id = a.idx[D];
  FaceFlux Fb;
  Fb.rho = (v[t] - v[cm]) * id;
  Fb.mn = (v[(1 + D) * a.nc + t] - v[(1 + D) * a.nc + cm]) * id;
  Fb.mt1 = (v[(1 + T1) * a.nc + t] - v[(1 + T1) * a.nc + cm]) * id;
  Fb.mt2 = (v[(1 + T2) * a.nc + t] - v[(1 + T2) * a.nc + cm]) * id;
  Fb.e = (v[4 * a.nc + t] - v[4 * a.nc + cm]) * id;
  Fb.bt1 = -e6_b;  // EMF of component T2 is -F.bt1
  Fb.bt2 = e5_b;   // EMF of component T1 is +F.bt2
  FaceState L, R;
  face_states<RECON>(a, s, c, D, L, R);
  const double bn = fb[D * a.g.fvar + pf(a, c, D, 0)];
  FaceState Lb{0, 0, 0, 0, 0, 0, 0}, Rb{0, 0, 0, 0, 0, 0, 0};
  double bn_b = 0.0;
  if (RS == 1) hlld_vjp(L, R, bn, a.gas, a.ct_eps, Fb, w_b, Lb, Rb, bn_b);
  else hlle_vjp(L, R, bn, a.gas, a.ct_eps, Fb, w_b, Lb, Rb, bn_b);
  const double lb[7] = {Lb.rho, Lb.vn, Lb.vt1, Lb.vt2, Lb.p, Lb.bt1, Lb.bt2};
  const double rb[7] = {Rb.rho, Rb.vn, Rb.vt1, Rb.vt2, Rb.p, Rb.bt1, Rb.bt2};
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    s[(S_LB + 7 * D + m) * a.nc + t] = lb[m];
    s[(S_RB + 7 * D + m) * a.nc + t] = rb[m];
  }
  s[(S_BN + D) * a.nc + t] = bn_b;
}

// ---- 5. reverse of the reconstruction along D ------------------------------
// Cell c feeds the right state of its lower face (c) and the left state of
// its upper face (c + D); with PLM it also enters the slopes of c - D, c and
// c + D.  Adds the contributions of direction D to the primitive cotangents.
template <int D, int RECON>
__device__ __forceinline__ void recon_bwd(const Adj& a, const double* __restrict__ s, const Cell& c, double* wb) {
  const int t = c.t;
  const int cp = at1(a, c, D, 1);
  int cm = 0, cm2 = 0, cp2 = 0;
  if (RECON == 1) {
    cm = at1(a, c, D, -1);
    cm2 = at1(a, c, D, -2);
    cp2 = at1(a, c, D, 2);
  }
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const double* lb = s + (S_LB + 7 * D + m) * a.nc;
    const double* rb = s + (S_RB + 7 * D + m) * a.nc;
    double g = rb[t] + lb[cp];
    if (RECON == 1) {
      const double* q = s + (S_W + wslot(D, m)) * a.nc;
      // slope cotangents: delta(x) enters q_L(x + D) with +1/2, q_R(x) with -1/2
      const double dbm = 0.5 * (lb[t] - rb[cm]);    // slope of c - D
      const double db0 = 0.5 * (lb[cp] - rb[t]);    // slope of c
      const double dbp = 0.5 * (lb[cp2] - rb[cp]);  // slope of c + D
      const double qm2 = q[cm2], qm = q[cm], q0 = q[t], qp = q[cp], qp2 = q[cp2];
      double x0 = 0.0, x1 = 0.0, x2 = 0.0;
      vl_slope_vjp(qm2, qm, q0, dbm, x0, x1, x2);  // c is the right point
      g += x2;
      x0 = x1 = x2 = 0.0;
      vl_slope_vjp(qm, q0, qp, db0, x0, x1, x2);  // c is the centre
      g += x1;
      x0 = x1 = x2 = 0.0;
      vl_slope_vjp(q0, qp, qp2, dbp, x0, x1, x2);  // c is the left point
      g += x0;
    }
    wb[wslot(D, m)] += g;
    if (RECON == 1) __builtin_amdgcn_sched_barrier(0);  // one variable's loads at a time
  }
}

// ---- 6. cell EMFs and cons -> prim in reverse -------------------------------
// Output of the stage (per cotangent slot): O = g0 V + scale J^T V, and, when
// Z is not NULL, Z = (zfirst ? 0 : Z) + g1 V.
struct StageOut {
  const double* V;
  double* O;
  double* Z;
  double g0, g1, scale;
  int zfirst;
};

__device__ __forceinline__ void stage_out(const StageOut& so, int64_t off, int m, int64_t nc, int t, double jt) {
  const int64_t e = off + m * nc + t;
  const double v = so.V[e];
  so.O[e] = so.g0 * v + so.scale * jt;
  if (so.Z) so.Z[e] = (so.zfirst ? 0.0 : so.Z[e]) + so.g1 * v;
}

template <int RECON>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(2))) k_adj_cell(Adj a,
                                                                                        double* __restrict__ scr,
                                                                                        StageOut so) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  double* s = scr + blockIdx.y * (S_TOTAL * a.nc);
  const int64_t off = blockIdx.y * (8 * a.nc);
  const Cell c = cell_of(a, t);
  double wb[8], w[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    wb[m] = 0.0;
    w[m] = s[(S_W + m) * a.nc + t];
  }
  // one direction at a time: keeps the loads of the three directions from
  // being hoisted together (register pressure)
  recon_bwd<0, RECON>(a, s, c, wb);
  __builtin_amdgcn_sched_barrier(0);
  recon_bwd<1, RECON>(a, s, c, wb);
  __builtin_amdgcn_sched_barrier(0);
  recon_bwd<2, RECON>(a, s, c, wb);
  __builtin_amdgcn_sched_barrier(0);
  // cell EMF of component e enters the four corner EMFs of component e
  // around it (as c00, ca, cb, cab of the edges at c, c+a, c+b, c+a+b)
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int ea = (e + 1) % 3, eb = (e + 2) % 3;
    const double* EB = s + (S_EB + e) * a.nc;
    const double* wa = s + (S_FE + 3 * ea + 2) * a.nc;
    const double* wbf = s + (S_FE + 3 * eb + 2) * a.nc;
    const int xa = at1(a, c, ea, 1), xb = at1(a, c, eb, 1), xab = at2(a, c, ea, 1, eb, 1);
    // weights of an edge x: wa0 = wa[x], wa1 = wa[x - b], wb0 = wbf[x], wb1 = wbf[x - a]
    const double g00 = -0.25 * ((1.0 - wa[t]) + (1.0 - wbf[t]));
    const double ga = -0.25 * (wa[xa] + (1.0 - wbf[t]));           // edge c+a: wa0 = wa[c+a], wb1 = wbf[c]
    const double gb = -0.25 * ((1.0 - wa[t]) + wbf[xb]);           // edge c+b: wa1 = wa[c], wb0 = wbf[c+b]
    const double gab = -0.25 * (wa[xa] + wbf[xb]);                  // edge c+a+b: wa1 = wa[c+a], wb1 = wbf[c+b]
    const double ce_b = EB[t] * g00 + EB[xa] * ga + EB[xb] * gb + EB[xab] * gab;
    // E_e = -(v_a B_b - v_b B_a)
    wb[1 + ea] -= ce_b * w[5 + eb];
    wb[5 + eb] -= ce_b * w[1 + ea];
    wb[1 + eb] += ce_b * w[5 + ea];
    wb[5 + ea] += ce_b * w[1 + eb];
  }
  // W = (rho, v = M / rho, p = (gamma - 1)(E - |M|^2 / (2 rho) - |Bcc|^2 / 2), Bcc)
  const double rho = w[0], ir = 1.0 / rho, gm1 = a.gas.gm1;
  const double pb = wb[4];
  const double vsq = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  double urho = wb[0] + 0.5 * gm1 * vsq * pb;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    urho -= wb[1 + d] * w[1 + d] * ir;
    stage_out(so, off, 1 + d, a.nc, t, wb[1 + d] * ir - gm1 * w[1 + d] * pb);
    s[(S_BC + d) * a.nc + t] = wb[5 + d] - gm1 * w[5 + d] * pb;
  }
  stage_out(so, off, 0, a.nc, t, urho);
  stage_out(so, off, 4, a.nc, t, gm1 * pb);
}

// ---- 7. face-field cotangents -----------------------------------------------
// B_d at the lower face of c: normal field of that face's Riemann problem and
// half of the cell-centred field of c and of c - d.
__global__ void __launch_bounds__(kT) k_adj_bface(Adj a, const double* __restrict__ scr, StageOut so) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  const double* s = scr + blockIdx.y * (S_TOTAL * a.nc);
  const int64_t off = blockIdx.y * (8 * a.nc);
  const Cell c = cell_of(a, t);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double* bc = s + (S_BC + d) * a.nc;
    stage_out(so, off, 5 + d, a.nc, t, s[(S_BN + d) * a.nc + t] + 0.5 * (bc[t] + bc[at1(a, c, d, -1)]));
  }
}

// ---- helpers: fill, axpby, padded <-> active ------------------------------
__global__ void __launch_bounds__(kT) k_adj_fill(double* __restrict__ p, double v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void __launch_bounds__(kT) k_adj_axpby(double* out, double x_coef, const double* x, double y_coef,
                                                 const double* y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < n) out[t] = x_coef * x[t] + y_coef * y[t];
}

// active entries of padded (cons, bface) -> 8 active-only arrays
__global__ void __launch_bounds__(kT) k_adj_gather(Adj a, const double* __restrict__ gc,
                                                  const double* __restrict__ gb, double* __restrict__ V) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= (int)a.nc) return;
  const double* uc = gc + blockIdx.y * a.g.cblock;
  const double* ub = gb + blockIdx.y * a.g.fblock;
  double* v = V + blockIdx.y * (8 * a.nc);
  const Cell c = cell_of(a, t);
  const int q = pc(a, c);
#pragma unroll
  for (int m = 0; m < 5; ++m) v[m * a.nc + t] = uc[m * a.g.cvar + q];
  const int f = a.g.f(a.g.ng + c.x[0], a.g.ng + c.x[1], a.g.ng + c.x[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) v[(5 + d) * a.nc + t] = ub[d * a.g.fvar + f];
}

// padded outputs: active entries = X + Y (active-only arrays); every other
// entry (ghosts, periodic-image faces, padding) passes its input through,
// since the step leaves those entries unchanged.
__global__ void __launch_bounds__(kT) k_adj_scatter_cons(Adj a, const double* __restrict__ X,
                                                        const double* __restrict__ Y, const double* gin,
                                                        double* gout) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= a.g.cvar) return;
  const int i = (int)(t % a.g.N1);
  const int r = (int)(t / a.g.N1);
  const int j = r % a.g.N2, k = r / a.g.N2;
  const int ng = a.g.ng;
  const bool act = i >= ng && i < ng + a.n[0] && j >= ng && j < ng + a.n[1] && k >= ng && k < ng + a.n[2];
  const int64_t at_ = act ? ((int64_t)(k - ng) * a.n[1] + (j - ng)) * a.n[0] + (i - ng) : 0;
  const double* x = X + blockIdx.y * (8 * a.nc);
  const double* y = Y + blockIdx.y * (8 * a.nc);
  const double* gi = gin + blockIdx.y * a.g.cblock;
  double* go = gout + blockIdx.y * a.g.cblock;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int64_t e = m * a.g.cvar + t;
    go[e] = act ? x[m * a.nc + at_] + y[m * a.nc + at_] : gi[e];
  }
}

__global__ void __launch_bounds__(kT) k_adj_scatter_bface(Adj a, const double* __restrict__ X,
                                                         const double* __restrict__ Y, const double* gin,
                                                         double* gout) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= a.g.fvar) return;
  const int i = (int)(t % a.g.F1);
  const int r = (int)(t / a.g.F1);
  const int j = r % a.g.F2, k = r / a.g.F2;
  const int ng = a.g.ng;
  const bool act = i >= ng && i < ng + a.n[0] && j >= ng && j < ng + a.n[1] && k >= ng && k < ng + a.n[2];
  const int64_t at_ = act ? ((int64_t)(k - ng) * a.n[1] + (j - ng)) * a.n[0] + (i - ng) : 0;
  const double* x = X + blockIdx.y * (8 * a.nc);
  const double* y = Y + blockIdx.y * (8 * a.nc);
  const double* gi = gin + blockIdx.y * a.g.fblock;
  double* go = gout + blockIdx.y * a.g.fblock;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t e = d * a.g.fvar + t;
    go[e] = act ? x[(5 + d) * a.nc + at_] + y[(5 + d) * a.nc + at_] : gi[e];
  }
}

// ---- reverse of prim -> cons (every stored cell) ----------------------------
// U = (rho, rho v, P / (gamma - 1) + rho |v|^2 / 2 + |Bcc|^2 / 2), Bcc the mean
// of the two bounding faces.  g_prim <- (dU/dW)^T g_cons on every stored cell.
__global__ void __launch_bounds__(kT) k_p2c_vjp_cell(Geo g, double igm1, const double* __restrict__ prim,
                                                    const double* __restrict__ gcons, double* __restrict__ gprim) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= g.cvar) return;
  const double* w = prim + blockIdx.y * g.cblock;
  const double* gu = gcons + blockIdx.y * g.cblock;
  double* gw = gprim + blockIdx.y * g.cblock;
  const double rho = w[t];
  const double ge = gu[4 * g.cvar + t];
  double grho = gu[t];
  double vsq = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double v = w[(1 + d) * g.cvar + t];
    const double gm = gu[(1 + d) * g.cvar + t];
    vsq += v * v;
    grho += v * gm;
    gw[(1 + d) * g.cvar + t] = rho * gm + rho * v * ge;
  }
  gw[t] = grho + 0.5 * vsq * ge;
  gw[4 * g.cvar + t] = igm1 * ge;
}

// g_bface += (dU/dB)^T g_cons: the energy of each stored cell depends on the
// two faces bounding it along each direction, with weight Bcc_d / 2.
__global__ void __launch_bounds__(kT) k_p2c_vjp_face(Geo g, const double* __restrict__ bface,
                                                    const double* __restrict__ gcons, double* __restrict__ gbface) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= g.fvar) return;
  const int i = (int)(t % g.F1);
  const int r = (int)(t / g.F1);
  const int j = r % g.F2, k = r / g.F2;
  const double* fb = bface + blockIdx.y * g.fblock;
  const double* ge = gcons + blockIdx.y * g.cblock + 4 * g.cvar;
  double* gb = gbface + blockIdx.y * g.fblock;
  const int x[3] = {i, j, k};
  const int N[3] = {g.N1, g.N2, g.N3};
  const int fs[3] = {1, g.F1, g.F1 * g.F2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // the transverse indices must name stored cells
    bool ok = true;
#pragma unroll
    for (int e = 0; e < 3; ++e)
      if (e != d && x[e] >= N[e]) ok = false;
    if (!ok) continue;
    const double* b = fb + d * g.fvar;
    double acc = 0.0;
    if (x[d] < N[d]) {  // cell on the upper side of the face
      const int q = g.c(i, j, k);
      acc += 0.5 * 0.5 * (b[t] + b[t + fs[d]]) * ge[q];
    }
    if (x[d] > 0) {  // cell on the lower side
      int xm[3] = {i, j, k};
      xm[d] -= 1;
      const int q = g.c(xm[0], xm[1], xm[2]);
      acc += 0.5 * 0.5 * (b[t - fs[d]] + b[t]) * ge[q];
    }
    gb[d * g.fvar + t] += acc;
  }
}

Adj make_adj(const Geo& g, double gamma, double ct_eps) {
  Adj a;
  a.g = g;
  a.n[0] = g.n1;
  a.n[1] = g.n2;
  a.n[2] = g.n3;
  a.nc = (int64_t)g.n1 * g.n2 * g.n3;
  a.st[0] = 1;
  a.st[1] = g.n1;
  a.st[2] = g.n1 * g.n2;
  a.idx[0] = 1.0 / g.dx1;
  a.idx[1] = 1.0 / g.dx2;
  a.idx[2] = 1.0 / g.dx3;
  a.gas = Gas{gamma, gamma - 1.0, 1.0 / (gamma - 1.0)};
  a.ct_eps = ct_eps;
  return a;
}

template <int D, int RECON>
void face_pair(const Adj& a, int rs, dim3 grid, const double* xb, const double* V, double* scr, hipStream_t s,
               bool bwd) {
  if (!bwd) {
    if (rs == 1) hipLaunchKernelGGL((k_adj_face_fwd<D, RECON, 1>), grid, dim3(kT), 0, s, a, xb, scr);
    else hipLaunchKernelGGL((k_adj_face_fwd<D, RECON, 0>), grid, dim3(kT), 0, s, a, xb, scr);
  } else {
    if (rs == 1) hipLaunchKernelGGL((k_adj_face_bwd<D, RECON, 1>), grid, dim3(kT), 0, s, a, xb, V, scr);
    else hipLaunchKernelGGL((k_adj_face_bwd<D, RECON, 0>), grid, dim3(kT), 0, s, a, xb, V, scr);
  }
}

template <int D>
void face_dir(const Adj& a, int recon, int rs, dim3 grid, const double* xb, const double* V, double* scr,
              hipStream_t s, bool bwd) {
  if (recon == 0) face_pair<D, 0>(a, rs, grid, xb, V, scr, s, bwd);
  else face_pair<D, 1>(a, rs, grid, xb, V, scr, s, bwd);
}


}  // namespace

int64_t adj_scratch_per_block(const Geo& g) { return (int64_t)S_TOTAL * g.n1 * g.n2 * g.n3; }

hipError_t launch_stage_vjp(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                            const double* xb, const double* V, double* O, double g0, double scale, double* Z,
                            double g1, int zfirst, double* scr, int nb, hipStream_t s) {
  if (recon != 0 && recon != 1) return hipErrorInvalidValue;
  const Adj a = make_adj(g, gamma, ct_eps);
  const dim3 grid(grid_of(a.nc), nb);
  hipLaunchKernelGGL(k_adj_prim, grid, dim3(kT), 0, s, a, xc, xb, V, scr);
  face_dir<0>(a, recon, rs, grid, xb, V, scr, s, false);
  face_dir<1>(a, recon, rs, grid, xb, V, scr, s, false);
  face_dir<2>(a, recon, rs, grid, xb, V, scr, s, false);
  face_dir<0>(a, recon, rs, grid, xb, V, scr, s, true);
  face_dir<1>(a, recon, rs, grid, xb, V, scr, s, true);
  face_dir<2>(a, recon, rs, grid, xb, V, scr, s, true);
  const StageOut so{V, O, Z, g0, g1, scale, zfirst};
  if (recon == 0) hipLaunchKernelGGL((k_adj_cell<0>), grid, dim3(kT), 0, s, a, scr, so);
  else hipLaunchKernelGGL((k_adj_cell<1>), grid, dim3(kT), 0, s, a, scr, so);
  hipLaunchKernelGGL(k_adj_bface, grid, dim3(kT), 0, s, a, scr, so);
  return hipGetLastError();
}

hipError_t launch_adj_fill(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_fill, dim3(grid_of(n)), dim3(kT), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_adj_axpby(double* out, double xc, const double* x, double yc, const double* y, int64_t n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_axpby, dim3(grid_of(n)), dim3(kT), 0, s, out, xc, x, yc, y, n);
  return hipGetLastError();
}

hipError_t launch_adj_gather(const Geo& g, const double* gc, const double* gb, double* V, int nb, hipStream_t s) {
  const Adj a = make_adj(g, 2.0, 0.0);
  hipLaunchKernelGGL(k_adj_gather, dim3(grid_of(a.nc), nb), dim3(kT), 0, s, a, gc, gb, V);
  return hipGetLastError();
}

hipError_t launch_adj_scatter(const Geo& g, const double* X, const double* Y, const double* gc_in,
                              const double* gb_in, double* gc_out, double* gb_out, int nb, hipStream_t s) {
  const Adj a = make_adj(g, 2.0, 0.0);
  hipLaunchKernelGGL(k_adj_scatter_cons, dim3(grid_of(g.cvar), nb), dim3(kT), 0, s, a, X, Y, gc_in, gc_out);
  hipLaunchKernelGGL(k_adj_scatter_bface, dim3(grid_of(g.fvar), nb), dim3(kT), 0, s, a, X, Y, gb_in, gb_out);
  return hipGetLastError();
}

hipError_t launch_prim2cons_vjp(const Geo& g, double gamma, const double* prim, const double* bface,
                                const double* gcons, double* gprim, double* gbface, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_p2c_vjp_cell, dim3(grid_of(g.cvar), nb), dim3(kT), 0, s, g, 1.0 / (gamma - 1.0), prim, gcons,
                     gprim);
  hipLaunchKernelGGL(k_p2c_vjp_face, dim3(grid_of(g.fvar), nb), dim3(kT), 0, s, g, bface, gcons, gbface);
  return hipGetLastError();
}

}  // namespace athmhd
