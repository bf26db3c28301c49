// athmhd_oracle.cpp -- plain, single-threaded, FP64 CPU oracle of the unsplit
// finite-volume ideal-MHD step of Stone, Tomida, White & Felker (2020),
// "The Athena++ Adaptive Mesh Refinement Framework: Design and
// Magnetohydrodynamic Solvers", Section 3 ("A Non-Relativistic MHD Solver").
//
// TEST INFRASTRUCTURE ONLY.  This file exists so that the HIP implementation
// can be checked against something obviously correct.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product library never does, and the two share no code, headers, tables or
// helpers.  Every routine is written in the order the method states its steps,
// with no blocking, fusion or reordering.  Compile with -ffp-contract=off so
// that no multiply-add is contracted (Section 3.3.5 explains why contraction
// breaks exact mirror symmetry).
//
// What the paper fixes and what is a reading (the paper defers the algorithm
// details to Stone et al. 2008, Gardiner & Stone 2005 and others, which are not
// reproduced in it):
//   * equations: ideal MHD, Eq. (cons) with Pi = eta = eta_AD = Q = 0, mu = 1,
//     total energy Eq. (total_energy), ideal-gas EOS P = (gamma-1) e (Sec. 3.1);
//   * volume-averaged conserved variables, face-area-averaged B, upwind CT for
//     the induction equation (Sec. 3.1);
//   * reconstruction DC / PLM with the original van Leer limiter on uniform
//     grids / PPM with the uniform-grid face weights Eq. (ppm-uniform-weights)
//     and a smooth-extremum-preserving limiter (Sec. 3.2.1).  The limiter
//     formulas are the published ones of van Leer (1974) and Colella & Sekora
//     (2008), restated here (readings: primitive variables, harmonic-mean
//     slope, limiter constant C = 1.25);
//   * Riemann solvers HLLE and HLLD (Sec. 3.2.2), restated from their
//     published definitions (HLLD: Miyoshi & Kusano 2005; HLLE with Davis
//     speed bounds; degeneracy thresholds 1e-8 of the star total pressure);
//   * time integration: the 2S low-storage scheme Eq. (rk-2s) with the RK1,
//     VL2, RK2 and RK3 coefficient sets listed in Sec. 3.2.3; the VL2
//     predictor always uses donor-cell fluxes (Sec. 3.2.3);
//   * corner EMFs: the upwind CT average of Gardiner & Stone (2005), with the
//     upwind direction taken from the sign of the face mass flux; an optional
//     continuous weight (ct_eps > 0) replaces the three-way switch;
//   * time step: one global dt from |v| + c_f (Sec. 2.1.7), per direction min;
//   * face-B registers follow the same 2S weights as the conserved variables;
//   * passive scalars (Sec. 3.2.6 "Additional Physics", Eq. (passive_scalars)):
//     the conserved variable is rho C_i and the primitive C_i.  Readings: C_i
//     is reconstructed like the other primitives, and the flux of rho C_i
//     through a face is the face mass flux times C_i on the upwind side (the
//     left state where the mass flux is >= 0, else the right state); with
//     floors, C_i = (rho C_i) / rho_W with the floored density, and the floor
//     pass after a stage leaves rho C_i alone;
//   * characteristic reconstruction (Sec. 3.2.1, C = L W, optional, PLM and
//     PPM): the paper defers the projection steps to another paper.  Reading:
//     for each cell the differences of the face-frame primitives of its
//     stencil from the cell's own are projected with the left eigenvectors of
//     that cell's primitive system, reconstructed per wave family (van Leer
//     slope, or the limited PPM parabola), and the edge offsets projected
//     back with the right eigenvectors.  Right eigenvectors follow the Roe &
//     Balsara (1996) normalisation; the left ones are their inverse.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

namespace orc {

// ---------------------------------------------------------------------------
// Scalar types: plain double, and a forward-mode dual number used only to get
// exact directional derivatives (Jacobian-vector products) of the same code.
// Branches always follow the value part.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: implicit on purpose
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(double a, Dual b) { return Dual(a) + b; }
inline Dual operator+(Dual a, double b) { return a + Dual(b); }
inline Dual operator-(double a, Dual b) { return Dual(a) - b; }
inline Dual operator-(Dual a, double b) { return a - Dual(b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }

// Operation-counting scalar: every add, subtract, multiply, divide and square
// root of the algorithm is tallied (comparisons and selects are not flops).
struct OpCount {
  unsigned long long add, mul, div, sqrt;
};
static OpCount g_ops = {0, 0, 0, 0};
struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}  // NOLINT: implicit on purpose
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_ops.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_ops.add; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_ops.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_ops.div; return Cnt(a.v / b.v); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt sqrt(Cnt a) { ++g_ops.sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double val(const Cnt& x) { return x.v; }
using std::fabs;
using std::sqrt;

template <class T> inline T vmin(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }
template <class T> inline T vmax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> inline double sgn(const T& a) { return val(a) > 0.0 ? 1.0 : (val(a) < 0.0 ? -1.0 : 0.0); }

// ---------------------------------------------------------------------------
// Problem description.  Mirrored field by field by a ctypes Structure.
// ---------------------------------------------------------------------------
enum { RECON_DC = 0, RECON_PLM = 1, RECON_PPM = 2 };
enum { RS_HLLE = 0, RS_HLLD = 1, RS_ROE = 2 };
enum { INT_RK1 = 0, INT_VL2 = 1, INT_RK2 = 2, INT_RK3 = 3 };

struct Cfg {
  int32_t n1, n2, n3, ng;       // active cells per direction, ghost layers
  double gamma;                 // adiabatic index, > 1
  double dx1, dx2, dx3;         // uniform Cartesian cell widths
  int32_t recon, riemann, integrator;
  int32_t nscalars;             // passive scalars rho C_i stored after the 5 MHD variables
  double cfl;                   // Courant number C0 used by newdt
  double ct_eps;                // 0: sign switch for the CT upwinding; >0: ramp width
  double dfloor, pfloor;        // optional density / pressure floors (0: off)
  int32_t charac;               // 1: PLM / PPM on characteristic variables (DC unchanged)
  int32_t pad_;
};

// Number of primitive evaluations (cells and reconstructed face states) that a
// floor changed since the counter was last read.
static long long g_floored = 0;

// Array geometry.  Cell arrays are [v][k][j][i] with N_d = n_d + 2 ng,
// i fastest.  Face arrays are [c][k][j][i] padded to (N3+1)(N2+1)(N1+1);
// component c at index (k,j,i) is the face at the lower side of cell (k,j,i)
// along direction c.  Edge arrays use the same padded shape; the edge of
// component e at index (k,j,i) sits at the lower corner of cell (k,j,i) in the
// two directions transverse to e.
struct Geo {
  int n[3], ng, N[3];
  int nv;  // cell arrays of the state: 5 MHD variables, then the passive scalars
  explicit Geo(const Cfg& c) {
    n[0] = c.n1; n[1] = c.n2; n[2] = c.n3; ng = c.ng;
    nv = 5 + c.nscalars;
    for (int d = 0; d < 3; ++d) N[d] = n[d] + 2 * ng;
  }
  size_t ncell() const { return (size_t)N[0] * N[1] * N[2]; }
  size_t nface() const { return (size_t)(N[0] + 1) * (N[1] + 1) * (N[2] + 1); }
  size_t c(int i, int j, int k) const { return ((size_t)k * N[1] + j) * N[0] + i; }
  size_t f(int i, int j, int k) const { return ((size_t)k * (N[1] + 1) + j) * (N[0] + 1) + i; }
  int s(int) const { return ng; }
  int e(int d) const { return ng + n[d] - 1; }
  int wrap(int idx, int d) const { return ng + (((idx - ng) % n[d]) + n[d]) % n[d]; }
};

// ---------------------------------------------------------------------------
// Periodic ghost fill (Sec. 2.1.1: every MeshBlock carries N_G ghost layers
// that hold copies of the neighbouring active cells; on a single periodic
// block the neighbour is the block itself).  Face arrays are filled by the
// same wrap, so the boundary face ie+1/2 is the image of is-1/2 and a shared
// face is stored once.
// ---------------------------------------------------------------------------
template <class T> void fill_ghosts(const Geo& g, T* cons, T* bf) {
  for (int v = 0; v < g.nv; ++v) {
    T* a = cons + (size_t)v * g.ncell();
    for (int k = 0; k < g.N[2]; ++k)
      for (int j = 0; j < g.N[1]; ++j)
        for (int i = 0; i < g.N[0]; ++i) {
          int ii = g.wrap(i, 0), jj = g.wrap(j, 1), kk = g.wrap(k, 2);
          if (ii != i || jj != j || kk != k) a[g.c(i, j, k)] = a[g.c(ii, jj, kk)];
        }
  }
  for (int cpt = 0; cpt < 3; ++cpt) {
    T* b = bf + (size_t)cpt * g.nface();
    for (int k = 0; k <= g.N[2]; ++k)
      for (int j = 0; j <= g.N[1]; ++j)
        for (int i = 0; i <= g.N[0]; ++i) {
          int ii = g.wrap(i, 0), jj = g.wrap(j, 1), kk = g.wrap(k, 2);
          if (ii != i || jj != j || kk != k) b[g.f(i, j, k)] = b[g.f(ii, jj, kk)];
        }
  }
}

// ---------------------------------------------------------------------------
// Conserved <-> primitive (Eq. (total_energy) with the ideal-gas law of
// Sec. 3.1).  The cell-centred field is the mean of the two face values that
// bound the cell along each direction.  Without floors, non-physical cells are
// counted and reported.  With floors (dfloor, pfloor > 0) the primitives -- and
// only they, never the conserved variables -- are limited from below:
// rho_W = max(rho, dfloor), v = M / rho_W, P = max(P(U, rho_W), pfloor); every
// change is counted; a non-finite input still counts as non-physical.
// ---------------------------------------------------------------------------
template <class T>
int cons_to_prim(const Geo& g, double gamma, const T* cons, const T* bf, T* w, T* bcc, double dfloor = 0.0,
                 double pfloor = 0.0) {
  const bool floors = dfloor > 0.0 || pfloor > 0.0;
  const size_t nc = g.ncell(), nf = g.nface();
  int bad = 0;
  for (int k = 0; k < g.N[2]; ++k)
    for (int j = 0; j < g.N[1]; ++j)
      for (int i = 0; i < g.N[0]; ++i) {
        size_t q = g.c(i, j, k);
        T b1 = 0.5 * (bf[0 * nf + g.f(i, j, k)] + bf[0 * nf + g.f(i + 1, j, k)]);
        T b2 = 0.5 * (bf[1 * nf + g.f(i, j, k)] + bf[1 * nf + g.f(i, j + 1, k)]);
        T b3 = 0.5 * (bf[2 * nf + g.f(i, j, k)] + bf[2 * nf + g.f(i, j, k + 1)]);
        T rho = cons[0 * nc + q];
        T m1 = cons[1 * nc + q], m2 = cons[2 * nc + q], m3 = cons[3 * nc + q];
        T en = cons[4 * nc + q];
        const bool finite_in = std::isfinite(val(rho)) && std::isfinite(val(en));
        bool floored = false;
        if (floors && finite_in && !(val(rho) >= dfloor)) {
          rho = T(dfloor);
          floored = true;
        }
        T kin = 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / rho;
        T mag = 0.5 * (b1 * b1 + b2 * b2 + b3 * b3);
        T p = (gamma - 1.0) * (en - kin - mag);
        if (floors && finite_in && !(val(p) >= pfloor)) {
          p = T(pfloor);
          floored = true;
        }
        if (floored) ++g_floored;
        w[0 * nc + q] = rho;
        w[1 * nc + q] = m1 / rho;
        w[2 * nc + q] = m2 / rho;
        w[3 * nc + q] = m3 / rho;
        w[4 * nc + q] = p;
        bcc[0 * nc + q] = b1;
        bcc[1 * nc + q] = b2;
        bcc[2 * nc + q] = b3;
        // passive scalars: specific densities C_i from the masses rho C_i
        for (int v = 5; v < g.nv; ++v) w[v * nc + q] = cons[v * nc + q] / rho;
        if (!(val(rho) > 0.0) || !(val(p) > 0.0) || !std::isfinite(val(rho)) || !std::isfinite(val(p)))
          ++bad;
      }
  return bad;
}

template <class T>
void prim_to_cons(const Geo& g, double gamma, const T* w, const T* bf, T* cons) {
  const size_t nc = g.ncell(), nf = g.nface();
  for (int k = 0; k < g.N[2]; ++k)
    for (int j = 0; j < g.N[1]; ++j)
      for (int i = 0; i < g.N[0]; ++i) {
        size_t q = g.c(i, j, k);
        T b1 = 0.5 * (bf[0 * nf + g.f(i, j, k)] + bf[0 * nf + g.f(i + 1, j, k)]);
        T b2 = 0.5 * (bf[1 * nf + g.f(i, j, k)] + bf[1 * nf + g.f(i, j + 1, k)]);
        T b3 = 0.5 * (bf[2 * nf + g.f(i, j, k)] + bf[2 * nf + g.f(i, j, k + 1)]);
        T rho = w[0 * nc + q], v1 = w[1 * nc + q], v2 = w[2 * nc + q], v3 = w[3 * nc + q];
        T p = w[4 * nc + q];
        cons[0 * nc + q] = rho;
        cons[1 * nc + q] = rho * v1;
        cons[2 * nc + q] = rho * v2;
        cons[3 * nc + q] = rho * v3;
        cons[4 * nc + q] = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) +
                           0.5 * (b1 * b1 + b2 * b2 + b3 * b3);
        for (int v = 5; v < g.nv; ++v) cons[v * nc + q] = rho * w[v * nc + q];
      }
}

// ---------------------------------------------------------------------------
// Reconstruction (Sec. 3.2.1).  All three act on one primitive variable along
// one line of cells.  `q` points at the cell whose LOWER face is the face being
// reconstructed (cell c, face c-1/2); q[-1] is cell c-1, and so on.
// ---------------------------------------------------------------------------
// van Leer (1974) harmonic-mean slope of cell c from its two one-sided
// differences; zero at extrema.
template <class T> T vanleer_slope(const T& qm, const T& q0, const T& qp) {
  T dm = q0 - qm, dp = qp - q0;
  T prod = dm * dp;
  if (val(prod) > 0.0) return 2.0 * prod / (dm + dp);
  return T(0.0);
}

// Colella & Sekora (2008) extremum-preserving PPM, uniform grid.
// Face value at c-1/2 from Eq. (ppm-uniform-weights), then limited.
const double kPpmC = 1.25;

template <class T> T cs_limit3(const T& a, const T& b, const T& c) {
  // sign(a) * min(|a|, C|b|, C|c|) if a, b, c share a sign, else 0
  if ((val(a) > 0.0 && val(b) > 0.0 && val(c) > 0.0) || (val(a) < 0.0 && val(b) < 0.0 && val(c) < 0.0)) {
    T m = vmin(fabs(a), vmin(kPpmC * fabs(b), kPpmC * fabs(c)));
    return sgn(a) * m;
  }
  return T(0.0);
}

template <class T> T ppm_face(const T* q) {  // face c-1/2, q = &q_c
  T qf = (7.0 / 12.0) * (q[-1] + q[0]) - (1.0 / 12.0) * (q[-2] + q[1]);
  // the face value must lie between its two neighbours; otherwise replace the
  // implied second derivative by a limited one
  if (val((qf - q[-1]) * (q[0] - qf)) < 0.0) {
    T d2 = 3.0 * (q[-1] - 2.0 * qf + q[0]);
    T d2l = q[-2] - 2.0 * q[-1] + q[0];
    T d2r = q[-1] - 2.0 * q[0] + q[1];
    T d2lim = cs_limit3(d2, d2l, d2r);
    qf = 0.5 * (q[-1] + q[0]) - d2lim / 6.0;
  }
  return qf;
}

// Limited parabola of cell c (q = &q_c): returns its left (c-1/2) and right
// (c+1/2) edge values.
template <class T> void ppm_cell(const T* q, T& left, T& right) {
  T qm = ppm_face(q), qp = ppm_face(q + 1);
  T qc = q[0];
  if (val((qp - qc) * (qc - qm)) <= 0.0 || val((q[-1] - qc) * (qc - q[1])) <= 0.0) {
    // local extremum: scale the parabola by the limited curvature
    T d2 = 6.0 * (qm + qp) - 12.0 * qc;
    T d2c = q[-1] - 2.0 * qc + q[1];
    T d2l = q[-2] - 2.0 * q[-1] + qc;
    T d2r = qc - 2.0 * q[1] + q[2];
    T d2lim(0.0);
    bool same = (val(d2) > 0.0 && val(d2c) > 0.0 && val(d2l) > 0.0 && val(d2r) > 0.0) ||
                (val(d2) < 0.0 && val(d2c) < 0.0 && val(d2l) < 0.0 && val(d2r) < 0.0);
    if (same) d2lim = sgn(d2) * vmin(fabs(d2), vmin(kPpmC * fabs(d2l), vmin(kPpmC * fabs(d2r), kPpmC * fabs(d2c))));
    if (val(d2) != 0.0) {
      qm = qc + (qm - qc) * d2lim / d2;
      qp = qc + (qp - qc) * d2lim / d2;
    } else {
      qm = qc;
      qp = qc;
    }
  } else {
    // monotone cell: remove the overshoot of the parabola (Colella & Woodward 1984)
    if (val(fabs(qp - qc)) >= val(2.0 * fabs(qm - qc))) qp = qc - 2.0 * (qm - qc);
    if (val(fabs(qm - qc)) >= val(2.0 * fabs(qp - qc))) qm = qc - 2.0 * (qp - qc);
  }
  left = qm;
  right = qp;
}

// Left and right states at face c-1/2 from the cells around it.
// ---------------------------------------------------------------------------
// Characteristic variables (Sec. 3.2.1: C = L W).  Face frame, primitive
// vector w = (rho, vn, vt1, vt2, P, Bt1, Bt2) with the normal field bn fixed.
// The system W_t + A W_x = 0 has the waves vn - cf, vn - ca, vn - cs, vn,
// vn + cs, vn + ca, vn + cf (fast, Alfven, slow magnetosonic and entropy).
// Columns of R are the right eigenvectors in that order, normalised after
// Roe & Balsara (1996): alpha_f^2 = (a^2 - cs^2)/(cf^2 - cs^2), alpha_s^2 =
// (cf^2 - a^2)/(cf^2 - cs^2), (beta_1, beta_2) the direction of the
// transverse field (1/sqrt2 each when it vanishes), and where cf = cs the
// pair alpha_f = 1, alpha_s = 0.
// ---------------------------------------------------------------------------
template <class T> void prim_right_eigenvectors(const T* w, const T& bn, double gamma, T R[7][7]) {
  const T rho = w[0], p = w[4], b1 = w[5], b2 = w[6];
  const T a2 = gamma * p / rho;
  const T ca2 = bn * bn / rho;
  const T bt2 = b1 * b1 + b2 * b2;
  const T bb2 = ca2 + bt2 / rho;
  T disc2 = (a2 + bb2) * (a2 + bb2) - 4.0 * a2 * ca2;
  if (!(val(disc2) > 0.0)) disc2 = T(0.0);
  const T cf2 = 0.5 * (a2 + bb2 + sqrt(disc2));
  const T cs2 = val(cf2) > 0.0 ? a2 * ca2 / cf2 : T(0.0);
  T af(1.0), as(0.0);
  if (val(cf2 - cs2) > 0.0) {
    T af2 = (a2 - cs2) / (cf2 - cs2), as2 = (cf2 - a2) / (cf2 - cs2);
    af2 = vmin(T(1.0), vmax(T(0.0), af2));
    as2 = vmin(T(1.0), vmax(T(0.0), as2));
    af = sqrt(af2);
    as = sqrt(as2);
  }
  T be1(1.0 / std::sqrt(2.0)), be2(1.0 / std::sqrt(2.0));
  if (val(bt2) > 0.0) {
    const T bt = sqrt(bt2);
    be1 = b1 / bt;
    be2 = b2 / bt;
  }
  const double sg = val(bn) >= 0.0 ? 1.0 : -1.0;
  const T a = sqrt(a2), cf = sqrt(cf2), cs = sqrt(cs2), sr = sqrt(rho);
  const T gp = gamma * p;
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) R[r][c] = T(0.0);
  // fast waves, vn -/+ cf (columns 0 and 6)
  for (int side = 0; side < 2; ++side) {
    const int c = side == 0 ? 0 : 6;
    const double m = side == 0 ? -1.0 : 1.0;  // sign of the wave speed relative to vn
    R[0][c] = rho * af;
    R[1][c] = m * cf * af;
    R[2][c] = -m * as * cs * be1 * sg;
    R[3][c] = -m * as * cs * be2 * sg;
    R[4][c] = gp * af;
    R[5][c] = as * sr * a * be1;
    R[6][c] = as * sr * a * be2;
  }
  // Alfven waves, vn -/+ ca (columns 1 and 5)
  for (int side = 0; side < 2; ++side) {
    const int c = side == 0 ? 1 : 5;
    const double m = side == 0 ? -1.0 : 1.0;
    R[2][c] = m * be2;
    R[3][c] = -m * be1;
    R[5][c] = -be2 * sg * sr;
    R[6][c] = be1 * sg * sr;
  }
  // slow waves, vn -/+ cs (columns 2 and 4)
  for (int side = 0; side < 2; ++side) {
    const int c = side == 0 ? 2 : 4;
    const double m = side == 0 ? -1.0 : 1.0;
    R[0][c] = rho * as;
    R[1][c] = m * cs * as;
    R[2][c] = m * af * cf * be1 * sg;
    R[3][c] = m * af * cf * be2 * sg;
    R[4][c] = gp * as;
    R[5][c] = -af * sr * a * be1;
    R[6][c] = -af * sr * a * be2;
  }
  // entropy wave, vn (column 3)
  R[0][3] = T(1.0);
}

// Inverse of a 7 x 7 matrix by Gauss-Jordan elimination with partial
// pivoting (pivots chosen by magnitude of the value part).
template <class T> void invert7(const T A[7][7], T X[7][7]) {
  T M[7][14];
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 14; ++c) M[r][c] = c < 7 ? A[r][c] : T(c - 7 == r ? 1.0 : 0.0);
  for (int c = 0; c < 7; ++c) {
    int piv = c;
    for (int r = c + 1; r < 7; ++r)
      if (std::fabs(val(M[r][c])) > std::fabs(val(M[piv][c]))) piv = r;
    if (piv != c)
      for (int k = 0; k < 14; ++k) std::swap(M[c][k], M[piv][k]);
    const T inv = 1.0 / M[c][c];
    for (int k = 0; k < 14; ++k) M[c][k] = M[c][k] * inv;
    for (int r = 0; r < 7; ++r) {
      if (r == c) continue;
      const T f = M[r][c];
      for (int k = 0; k < 14; ++k) M[r][k] = M[r][k] - f * M[c][k];
    }
  }
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) X[r][c] = M[r][c + 7];
}

// Characteristic PLM edges of cell c from its neighbours: wm = W_{c-1},
// w0 = W_c, wp = W_{c+1} (7 face-frame primitives each), bn the cell-centred
// normal field of c.  left = W_c - dW/2, right = W_c + dW/2 with dW = R lim(L
// dW-, L dW+), lim the van Leer harmonic mean applied per wave family.
template <class T>
void char_plm_edges(const T* wm, const T* w0, const T* wp, const T& bn, double gamma, T* left, T* right) {
  T R[7][7], L[7][7];
  prim_right_eigenvectors(w0, bn, gamma, R);
  invert7(R, L);
  T dc[7];
  for (int k = 0; k < 7; ++k) {
    T dl(0.0), dr(0.0);
    for (int j = 0; j < 7; ++j) {
      dl = dl + L[k][j] * (w0[j] - wm[j]);
      dr = dr + L[k][j] * (wp[j] - w0[j]);
    }
    const T prod = dl * dr;
    dc[k] = val(prod) > 0.0 ? 2.0 * prod / (dl + dr) : T(0.0);
  }
  for (int j = 0; j < 7; ++j) {
    T dw(0.0);
    for (int k = 0; k < 7; ++k) dw = dw + R[j][k] * dc[k];
    left[j] = w0[j] - 0.5 * dw;
    right[j] = w0[j] + 0.5 * dw;
  }
}

// Characteristic PPM edges of cell c from its five-cell stencil w[o] =
// W_{c-2+o}: the differences from W_c in characteristic variables, the limited
// parabola of Colella & Sekora per wave family, and the edge offsets projected
// back.
template <class T> void char_ppm_edges(const T w[5][7], const T& bn, double gamma, T* left, T* right) {
  T R[7][7], L[7][7];
  prim_right_eigenvectors(w[2], bn, gamma, R);
  invert7(R, L);
  T cl[7], cr[7];
  for (int k = 0; k < 7; ++k) {
    T q[5];
    for (int o = 0; o < 5; ++o) {
      q[o] = T(0.0);
      for (int j = 0; j < 7; ++j) q[o] = q[o] + L[k][j] * (w[o][j] - w[2][j]);
    }
    ppm_cell(&q[2], cl[k], cr[k]);
  }
  for (int j = 0; j < 7; ++j) {
    T dl(0.0), dr(0.0);
    for (int k = 0; k < 7; ++k) {
      dl = dl + R[j][k] * cl[k];
      dr = dr + R[j][k] * cr[k];
    }
    left[j] = w[2][j] + dl;
    right[j] = w[2][j] + dr;
  }
}

template <class T> void recon_face(int recon, const T* q, T& ql, T& qr) {
  if (recon == RECON_DC) {
    ql = q[-1];
    qr = q[0];
  } else if (recon == RECON_PLM) {
    ql = q[-1] + 0.5 * vanleer_slope(q[-2], q[-1], q[0]);
    qr = q[0] - 0.5 * vanleer_slope(q[-1], q[0], q[1]);
  } else {
    T a, b;
    ppm_cell(q - 1, a, ql);  // right edge of cell c-1
    ppm_cell(q, qr, b);      // left edge of cell c
  }
}

// ---------------------------------------------------------------------------
// Riemann solvers in the frame (n, t1, t2) of the face (Sec. 3.2.2).
// State vector w = (rho, vn, vt1, vt2, p, Bt1, Bt2); bn is the face-normal
// field; flux f = (F_rho, F_Mn, F_Mt1, F_Mt2, F_E, F_Bt1, F_Bt2).
// ---------------------------------------------------------------------------
template <class T> T fast_speed(const T& rho, const T& p, const T& bn, const T& bt1, const T& bt2, double gamma) {
  T asq = gamma * p / rho;
  T bsq = bn * bn + bt1 * bt1 + bt2 * bt2;
  T s = asq + bsq / rho;
  T disc = s * s - 4.0 * asq * bn * bn / rho;
  if (val(disc) < 0.0) disc = T(0.0);
  return sqrt(0.5 * (s + sqrt(disc)));
}

// physical flux and conserved state of Eq. (cons) in the face frame
template <class T> void phys_flux(const T* w, const T& bn, double gamma, T* u, T* f) {
  T rho = w[0], vn = w[1], vt1 = w[2], vt2 = w[3], p = w[4], bt1 = w[5], bt2 = w[6];
  T pmag = 0.5 * (bn * bn + bt1 * bt1 + bt2 * bt2);
  T pt = p + pmag;
  T en = p / (gamma - 1.0) + 0.5 * rho * (vn * vn + vt1 * vt1 + vt2 * vt2) + pmag;
  T vdotb = vn * bn + vt1 * bt1 + vt2 * bt2;
  u[0] = rho; u[1] = rho * vn; u[2] = rho * vt1; u[3] = rho * vt2; u[4] = en; u[5] = bt1; u[6] = bt2;
  f[0] = rho * vn;
  f[1] = rho * vn * vn + pt - bn * bn;
  f[2] = rho * vn * vt1 - bn * bt1;
  f[3] = rho * vn * vt2 - bn * bt2;
  f[4] = (en + pt) * vn - bn * vdotb;
  f[5] = bt1 * vn - bn * vt1;
  f[6] = bt2 * vn - bn * vt2;
}

// HLLE: two-wave HLL flux with Davis speed bounds.
template <class T> void hlle(const T* wl, const T* wr, const T& bn, double gamma, T* flux, T& smax) {
  T ul[7], fl[7], ur[7], fr[7];
  phys_flux(wl, bn, gamma, ul, fl);
  phys_flux(wr, bn, gamma, ur, fr);
  T cfl = fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gamma);
  T cfr = fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gamma);
  T sl = vmin(wl[1] - cfl, wr[1] - cfr);
  T sr = vmax(wl[1] + cfl, wr[1] + cfr);
  T bp = vmax(sr, T(0.0));
  T bm = vmin(sl, T(0.0));
  for (int n = 0; n < 7; ++n) flux[n] = (bp * fl[n] - bm * fr[n] + bp * bm * (ur[n] - ul[n])) / (bp - bm);
  smax = vmax(fabs(sl), fabs(sr));
}

// HLLD: five-wave solver of Miyoshi & Kusano (2005).
const double kHlldSmall = 1.0e-8;

// The states of the HLLD fan that are not the outer states: speeds
// S_L < S*_L <= S_M <= S*_R < S_R, the total pressure p_T* of the fan, and
// the conserved single-star (U*_L, U*_R) and double-star (U**_L, U**_R)
// states in the face frame.  Filled on request only (a test hook); the flux
// itself does not need every state.
template <class T> struct HlldFan {
  T sl, ssl, sm, ssr, sr, pts;
  T us_l[7], uss_l[7], uss_r[7], us_r[7];
};

// Double-star states from the single-star ones (rotational discontinuities
// at S*_L, S*_R; transverse velocity and field continuous across S_M).
// Identical to the single-star states when Bx is negligible against p_T*.
template <class T>
void hlld_double_star(const T& bx, const T& sm, const T& pts, const T* us_l, const T* us_r, const T* vys,
                      const T* vzs, const T* bys, const T* bzs, const T* rhos, const T* vdbs, const T& sqrl,
                      const T& sqrr, T* uss_l, T* uss_r) {
  if (val(0.5 * bx * bx) < kHlldSmall * val(pts)) {
    for (int n = 0; n < 7; ++n) { uss_l[n] = us_l[n]; uss_r[n] = us_r[n]; }
    return;
  }
  double sb = sgn(bx);
  T isum = 1.0 / (sqrl + sqrr);
  T vyss = (sqrl * vys[0] + sqrr * vys[1] + (bys[1] - bys[0]) * sb) * isum;
  T vzss = (sqrl * vzs[0] + sqrr * vzs[1] + (bzs[1] - bzs[0]) * sb) * isum;
  T byss = (sqrl * bys[1] + sqrr * bys[0] + sqrl * sqrr * (vys[1] - vys[0]) * sb) * isum;
  T bzss = (sqrl * bzs[1] + sqrr * bzs[0] + sqrl * sqrr * (vzs[1] - vzs[0]) * sb) * isum;
  T vdbss = sm * bx + vyss * byss + vzss * bzss;
  T ess_l = us_l[4] - sqrl * (vdbs[0] - vdbss) * sb;
  T ess_r = us_r[4] + sqrr * (vdbs[1] - vdbss) * sb;
  uss_l[0] = rhos[0]; uss_l[1] = rhos[0] * sm; uss_l[2] = rhos[0] * vyss; uss_l[3] = rhos[0] * vzss;
  uss_l[4] = ess_l; uss_l[5] = byss; uss_l[6] = bzss;
  uss_r[0] = rhos[1]; uss_r[1] = rhos[1] * sm; uss_r[2] = rhos[1] * vyss; uss_r[3] = rhos[1] * vzss;
  uss_r[4] = ess_r; uss_r[5] = byss; uss_r[6] = bzss;
}

// fan != NULL: also record every intermediate state (the flux is unchanged);
// returns false when an outer state is upwind (S_L > 0 or S_R < 0) and no
// fan is formed.
template <class T>
bool hlld(const T* wl, const T* wr, const T& bx, double gamma, T* flux, T& smax, HlldFan<T>* fan = nullptr) {
  T ul[7], fl[7], ur[7], fr[7];
  phys_flux(wl, bx, gamma, ul, fl);
  phys_flux(wr, bx, gamma, ur, fr);
  const T rl = wl[0], vxl = wl[1], byl = wl[5], bzl = wl[6];
  const T rr = wr[0], vxr = wr[1], byr = wr[5], bzr = wr[6];
  const T ptl = wl[4] + 0.5 * (bx * bx + byl * byl + bzl * bzl);
  const T ptr = wr[4] + 0.5 * (bx * bx + byr * byr + bzr * bzr);
  const T el = ul[4], er = ur[4];

  // outer wave speeds
  T cfl = fast_speed(rl, wl[4], bx, byl, bzl, gamma);
  T cfr = fast_speed(rr, wr[4], bx, byr, bzr, gamma);
  T cmax = vmax(cfl, cfr);
  T sl = vmin(vxl, vxr) - cmax;
  T sr = vmax(vxl, vxr) + cmax;
  smax = vmax(fabs(sl), fabs(sr));
  if (val(sl) > 0.0) { for (int n = 0; n < 7; ++n) flux[n] = fl[n]; return false; }
  if (val(sr) < 0.0) { for (int n = 0; n < 7; ++n) flux[n] = fr[n]; return false; }

  // contact speed and star total pressure
  T sdl = sl - vxl, sdr = sr - vxr;
  T den = sdr * rr - sdl * rl;
  T sm = (sdr * rr * vxr - sdl * rl * vxl - ptr + ptl) / den;
  T pts = (sdr * rr * ptl - sdl * rl * ptr + rl * rr * sdr * sdl * (vxr - vxl)) / den;

  // single-star states on each side
  T us_l[7], us_r[7];
  T vys[2], vzs[2], bys[2], bzs[2], rhos[2], vdbs[2];
  for (int side = 0; side < 2; ++side) {
    const T* w = side == 0 ? wl : wr;
    const T s = side == 0 ? sl : sr;
    const T sd = side == 0 ? sdl : sdr;
    const T e = side == 0 ? el : er;
    const T pt = side == 0 ? ptl : ptr;
    T* us = side == 0 ? us_l : us_r;
    T rho = w[0], vx = w[1], vy = w[2], vz = w[3], by = w[5], bz = w[6];
    T rhostar = rho * sd / (s - sm);
    T d = rho * sd * (s - sm) - bx * bx;
    T vy_s, vz_s, by_s, bz_s;
    if (val(fabs(d)) < kHlldSmall * val(pts)) {
      vy_s = vy; vz_s = vz; by_s = by; bz_s = bz;
    } else {
      T ratio = bx * (sm - vx) / d;
      vy_s = vy - by * ratio;
      vz_s = vz - bz * ratio;
      T ratio2 = (rho * sd * sd - bx * bx) / d;
      by_s = by * ratio2;
      bz_s = bz * ratio2;
    }
    T vdotb = vx * bx + vy * by + vz * bz;
    T vdotb_s = sm * bx + vy_s * by_s + vz_s * bz_s;
    T e_s = (sd * e - pt * vx + pts * sm + bx * (vdotb - vdotb_s)) / (s - sm);
    us[0] = rhostar; us[1] = rhostar * sm; us[2] = rhostar * vy_s; us[3] = rhostar * vz_s;
    us[4] = e_s; us[5] = by_s; us[6] = bz_s;
    vys[side] = vy_s; vzs[side] = vz_s; bys[side] = by_s; bzs[side] = bz_s;
    rhos[side] = rhostar; vdbs[side] = vdotb_s;
  }
  T sqrl = sqrt(rhos[0]), sqrr = sqrt(rhos[1]);
  T ssl = sm - fabs(bx) / sqrl;
  T ssr = sm + fabs(bx) / sqrr;
  if (fan) {
    fan->sl = sl; fan->ssl = ssl; fan->sm = sm; fan->ssr = ssr; fan->sr = sr; fan->pts = pts;
    for (int n = 0; n < 7; ++n) { fan->us_l[n] = us_l[n]; fan->us_r[n] = us_r[n]; }
    hlld_double_star(bx, sm, pts, us_l, us_r, vys, vzs, bys, bzs, rhos, vdbs, sqrl, sqrr, fan->uss_l, fan->uss_r);
  }

  if (val(ssl) >= 0.0) {
    for (int n = 0; n < 7; ++n) flux[n] = fl[n] + sl * (us_l[n] - ul[n]);
    return true;
  }
  if (val(ssr) <= 0.0) {
    for (int n = 0; n < 7; ++n) flux[n] = fr[n] + sr * (us_r[n] - ur[n]);
    return true;
  }
  T uss_l[7], uss_r[7];
  hlld_double_star(bx, sm, pts, us_l, us_r, vys, vzs, bys, bzs, rhos, vdbs, sqrl, sqrr, uss_l, uss_r);
  if (val(sm) >= 0.0) {
    for (int n = 0; n < 7; ++n) flux[n] = fl[n] + sl * (us_l[n] - ul[n]) + ssl * (uss_l[n] - us_l[n]);
  } else {
    for (int n = 0; n < 7; ++n) flux[n] = fr[n] + sr * (us_r[n] - ur[n]) + ssr * (uss_r[n] - us_r[n]);
  }
  return true;
}

// ---------------------------------------------------------------------------
// Roe's linearised solver (Sec. 3.2.2 names it beside HLLE and HLLD and
// prints no formula).  Reading R-34: the Roe matrix A of the pair is the
// matrix with A (U_R - U_L) = F_R - F_L built from exact identities for
// differences, with the averages
//   s_a = sqrt(rho_a),  D = s_L + s_R,  rho_bar = s_L s_R,
//   q_bar = (s_L q_L + s_R q_R) / D      for q = v (3 components), H,
//   Bt_bar = (s_R Bt_L + s_L Bt_R) / D   (weights swapped),
//   X = |Bt_R - Bt_L|^2 / (2 D^2),
// where H = (E + p + B^2/2) / rho.  For these,
//   d(rho q) = rho_bar dq + q_bar d rho,   d(rho q r) = rho_bar (q_bar dr +
//   r_bar dq) + q_bar r_bar d rho,   d(q Bt) = q_bar dBt + Bt_bar dq,
//   d(B^2 / 2) = Bt_bar . dBt + X d rho
// hold exactly (d = right minus left).  Writing every difference of U and
// of the flux F through the primitive differences dW = (d rho, dv, dp, dBt)
// gives dU = M dW and dF = G dW with M, G built from the averages below, and
// A = G M^{-1}.  The flux is F = (F_L + F_R)/2 - |A| (U_R - U_L) / 2 with
// |A| = A sign(A), sign(A) from Newton's iteration S <- (S + S^{-1}) / 2.
// No entropy fix is applied.
// ---------------------------------------------------------------------------
template <class T> void roe_matrix(const T* wl, const T* wr, const T& bx, double gamma, T A[7][7]) {
  const T sl = sqrt(wl[0]), sr = sqrt(wr[0]);
  const T D = sl + sr;
  const T rho = sl * sr;
  const T u = (sl * wl[1] + sr * wr[1]) / D;
  const T v = (sl * wl[2] + sr * wr[2]) / D;
  const T w = (sl * wl[3] + sr * wr[3]) / D;
  T ul[7], fl[7], ur[7], fr[7];
  phys_flux(wl, bx, gamma, ul, fl);
  phys_flux(wr, bx, gamma, ur, fr);
  const T hl = (ul[4] + wl[4] + 0.5 * (bx * bx + wl[5] * wl[5] + wl[6] * wl[6])) / wl[0];
  const T hr = (ur[4] + wr[4] + 0.5 * (bx * bx + wr[5] * wr[5] + wr[6] * wr[6])) / wr[0];
  const T H = (sl * hl + sr * hr) / D;
  const T by = (sr * wl[5] + sl * wr[5]) / D;
  const T bz = (sr * wl[6] + sl * wr[6]) / D;
  const T dby = wr[5] - wl[5], dbz = wr[6] - wl[6];
  const T X = (dby * dby + dbz * dbz) / (2.0 * D * D);
  const T ke = 0.5 * (u * u + v * v + w * w);
  const T z(0.0);
  // dU = M dW, dW = (d rho, du, dv, dw, dp, dBy, dBz)
  const T M[7][7] = {
      {T(1.0), z, z, z, z, z, z},
      {u, rho, z, z, z, z, z},
      {v, z, rho, z, z, z, z},
      {w, z, z, rho, z, z, z},
      {ke + X, rho * u, rho * v, rho * w, T(1.0 / (gamma - 1.0)), by, bz},
      {z, z, z, z, z, T(1.0), z},
      {z, z, z, z, z, z, T(1.0)},
  };
  // d(rho H) = dE + dp + d(B^2/2)
  T drh[7];
  for (int c = 0; c < 7; ++c) drh[c] = M[4][c];
  drh[0] = drh[0] + X;
  drh[4] = drh[4] + 1.0;
  drh[5] = drh[5] + by;
  drh[6] = drh[6] + bz;
  // dF = G dW
  T G[7][7] = {
      {u, rho, z, z, z, z, z},
      {u * u + X, 2.0 * rho * u, z, z, T(1.0), by, bz},
      {u * v, rho * v, rho * u, z, z, -bx, z},
      {u * w, rho * w, z, rho * u, z, z, -bx},
      {z, H * rho - bx * bx, -bx * by, -bx * bz, z, -bx * v, -bx * w},
      {z, by, -bx, z, z, u, z},
      {z, bz, z, -bx, z, z, u},
  };
  for (int c = 0; c < 7; ++c) G[4][c] = G[4][c] + u * drh[c];
  T Mi[7][7];
  invert7(M, Mi);
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) {
      T acc(0.0);
      for (int k = 0; k < 7; ++k) acc = acc + G[r][k] * Mi[k][c];
      A[r][c] = acc;
    }
}

// sign(A) by Newton's iteration; false if it did not converge (A singular
// or nearly so).
template <class T> bool matrix_sign(const T A[7][7], T S[7][7]) {
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) S[r][c] = A[r][c];
  for (int it = 0; it < 200; ++it) {
    T Si[7][7];
    invert7(S, Si);
    double change = 0.0, size = 0.0;
    bool finite = true;
    for (int r = 0; r < 7; ++r)
      for (int c = 0; c < 7; ++c) {
        const T nx = 0.5 * (S[r][c] + Si[r][c]);
        if (!std::isfinite(val(nx))) finite = false;
        change = std::max(change, std::fabs(val(nx) - val(S[r][c])));
        size = std::max(size, std::fabs(val(nx)));
        S[r][c] = nx;
      }
    if (!finite) return false;
    if (change <= 1e-15 * size) return true;
  }
  return false;
}

// y = |A| x = A sign(A) x.  With an eigenvalue at (or within rounding of)
// zero the iteration fails; |A| is then taken as (|A + d I| + |A - d I|)/2,
// which differs from |A| only for eigenvalues below d = 1e-14 max|A_ij|.
template <class T> void abs_apply(const T A[7][7], const T* x, T* y) {
  T S[7][7];
  double amax = 0.0;
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) amax = std::max(amax, std::fabs(val(A[r][c])));
  if (matrix_sign(A, S)) {
    T sx[7];
    for (int r = 0; r < 7; ++r) {
      sx[r] = T(0.0);
      for (int c = 0; c < 7; ++c) sx[r] = sx[r] + S[r][c] * x[c];
    }
    for (int r = 0; r < 7; ++r) {
      y[r] = T(0.0);
      for (int c = 0; c < 7; ++c) y[r] = y[r] + A[r][c] * sx[c];
    }
    return;
  }
  const double d = 1e-14 * amax;
  for (int r = 0; r < 7; ++r) y[r] = T(0.0);
  for (int side = -1; side <= 1; side += 2) {
    T B[7][7];
    for (int r = 0; r < 7; ++r)
      for (int c = 0; c < 7; ++c) B[r][c] = A[r][c] + (r == c ? side * d : 0.0);
    if (!matrix_sign(B, S)) {
      for (int r = 0; r < 7; ++r) y[r] = T(NAN);
      return;
    }
    T sx[7];
    for (int r = 0; r < 7; ++r) {
      sx[r] = T(0.0);
      for (int c = 0; c < 7; ++c) sx[r] = sx[r] + S[r][c] * x[c];
    }
    for (int r = 0; r < 7; ++r)
      for (int c = 0; c < 7; ++c) y[r] = y[r] + 0.5 * (B[r][c] * sx[c]);
  }
}

template <class T> void roe(const T* wl, const T* wr, const T& bx, double gamma, T* flux, T& smax) {
  T ul[7], fl[7], ur[7], fr[7];
  phys_flux(wl, bx, gamma, ul, fl);
  phys_flux(wr, bx, gamma, ur, fr);
  // wave-speed bound for the CT weight: the larger |u| + c_f of the two states
  const T cfl = fast_speed(wl[0], wl[4], bx, wl[5], wl[6], gamma);
  const T cfr = fast_speed(wr[0], wr[4], bx, wr[5], wr[6], gamma);
  smax = vmax(fabs(wl[1]) + cfl, fabs(wr[1]) + cfr);
  T du[7];
  bool same = true;
  for (int n = 0; n < 7; ++n) {
    du[n] = ur[n] - ul[n];
    if (val(du[n]) != 0.0) same = false;
  }
  if (same) {
    for (int n = 0; n < 7; ++n) flux[n] = fl[n];
    return;
  }
  T A[7][7], d[7];
  roe_matrix(wl, wr, bx, gamma, A);
  abs_apply(A, du, d);
  for (int n = 0; n < 7; ++n) flux[n] = 0.5 * (fl[n] + fr[n]) - 0.5 * d[n];
}

template <class T> void riemann(int rs, const T* wl, const T* wr, const T& bn, double gamma, T* flux, T& smax) {
  if (rs == RS_HLLD) hlld(wl, wr, bn, gamma, flux, smax);
  else if (rs == RS_ROE) roe(wl, wr, bn, gamma, flux, smax);
  else hlle(wl, wr, bn, gamma, flux, smax);
}

// ---------------------------------------------------------------------------
// Spatial operator L(U): flux divergence of the conserved variables and the
// CT curl of the corner EMFs.  The inputs must have their ghosts filled.
// ---------------------------------------------------------------------------
template <class T> struct Work {
  std::vector<T> w, bcc;            // 5 and 3 cell arrays
  std::vector<T> flux[3];           // per direction: 5 face arrays (lab-frame components)
  std::vector<T> emf_t1[3], emf_t2[3];  // face EMFs of components t1 and t2 of each direction
  std::vector<T> wgt[3];            // upwind weight of each face (1: take the lower-side cell)
  std::vector<T> ecc;               // 3 cell arrays: cell-centred EMF -v x B
  std::vector<T> edge;              // 3 edge arrays: corner EMFs
};

// Face fluxes, face EMFs, upwind weights, cell EMFs and corner EMFs of a
// block whose ghosts are filled (steps 2-6 of the stage); returns the count
// of non-physical cells.
template <class T>
int compute_fluxes(const Cfg& cfg, const Geo& g, int recon, const T* cons, const T* bf, Work<T>& wk) {
  const size_t nc = g.ncell(), nf = g.nface();
  wk.w.assign(g.nv * nc, T(0.0));
  wk.bcc.assign(3 * nc, T(0.0));
  int bad = cons_to_prim(g, cfg.gamma, cons, bf, wk.w.data(), wk.bcc.data(), cfg.dfloor, cfg.pfloor);
  const int sten = recon == RECON_PPM ? 3 : (recon == RECON_PLM ? 2 : 1);

  // fluxes on every face that the update or the corner EMFs need:
  // normal index [s, e+1], transverse indices [s-1, e+1]
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    wk.flux[d].assign(g.nv * nf, T(0.0));
    wk.emf_t1[d].assign(nf, T(0.0));
    wk.emf_t2[d].assign(nf, T(0.0));
    wk.wgt[d].assign(nf, T(0.0));
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = g.s(a) - 1; hi[a] = g.e(a) + 1; }
    lo[d] = g.s(d);
    hi[d] = g.e(d) + 1;
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          // gather the line of cells c-sten-? .. c+sten-1 along d, c = (i,j,k)
          // rotated primitive order: rho, v_d, v_t1, v_t2, p, B_t1, B_t2
          T line[7][8];
          for (int o = -3; o <= 2; ++o) {
            int idx[3] = {i, j, k};
            idx[d] += o;
            if (o < -sten || o > sten - 1) { for (int n = 0; n < 7; ++n) line[n][o + 3] = T(0.0); continue; }
            size_t q = g.c(idx[0], idx[1], idx[2]);
            line[0][o + 3] = wk.w[0 * nc + q];
            line[1][o + 3] = wk.w[(1 + d) * nc + q];
            line[2][o + 3] = wk.w[(1 + t1) * nc + q];
            line[3][o + 3] = wk.w[(1 + t2) * nc + q];
            line[4][o + 3] = wk.w[4 * nc + q];
            line[5][o + 3] = wk.bcc[t1 * nc + q];
            line[6][o + 3] = wk.bcc[t2 * nc + q];
          }
          T wl[7], wr[7];
          if (cfg.charac && recon == RECON_PLM) {
            // characteristic PLM: right edge of cell c-1 and left edge of cell c,
            // each with the eigenvectors of its own cell
            T w[4][7], bnc[2];
            for (int o = 0; o < 4; ++o)
              for (int n = 0; n < 7; ++n) w[o][n] = line[n][o + 1];  // cells c-2 .. c+1
            for (int o = 0; o < 2; ++o) {
              int idx[3] = {i, j, k};
              idx[d] += o - 1;
              bnc[o] = wk.bcc[(size_t)d * nc + g.c(idx[0], idx[1], idx[2])];
            }
            T lft[7], rgt[7];
            char_plm_edges(w[0], w[1], w[2], bnc[0], cfg.gamma, lft, wl);  // cell c-1
            char_plm_edges(w[1], w[2], w[3], bnc[1], cfg.gamma, wr, rgt);  // cell c
          } else if (cfg.charac && recon == RECON_PPM) {
            // characteristic PPM: right edge of cell c-1, left edge of cell c
            T st[2][5][7], bnc[2];
            for (int cell = 0; cell < 2; ++cell)
              for (int o = 0; o < 5; ++o)
                for (int n = 0; n < 7; ++n) st[cell][o][n] = line[n][cell + o];  // cells c-3+cell .. c+1+cell
            for (int o = 0; o < 2; ++o) {
              int idx[3] = {i, j, k};
              idx[d] += o - 1;
              bnc[o] = wk.bcc[(size_t)d * nc + g.c(idx[0], idx[1], idx[2])];
            }
            T lft[7], rgt[7];
            char_ppm_edges(st[0], bnc[0], cfg.gamma, lft, wl);  // cell c-1
            char_ppm_edges(st[1], bnc[1], cfg.gamma, wr, rgt);  // cell c
          } else {
            for (int n = 0; n < 7; ++n) recon_face(recon, &line[n][3], wl[n], wr[n]);
          }
          // floors, when enabled, also apply to the reconstructed face states
          if (cfg.dfloor > 0.0 || cfg.pfloor > 0.0) {
            T* st[2] = {wl, wr};
            for (T* q : st) {
              bool floored = false;
              if (!(val(q[0]) >= cfg.dfloor)) { q[0] = T(cfg.dfloor); floored = true; }
              if (!(val(q[4]) >= cfg.pfloor)) { q[4] = T(cfg.pfloor); floored = true; }
              if (floored) ++g_floored;
            }
          }
          T bn = bf[d * nf + g.f(i, j, k)];
          T fx[7], smax;
          riemann(cfg.riemann, wl, wr, bn, cfg.gamma, fx, smax);
          size_t fi = g.f(i, j, k);
          wk.flux[d][0 * nf + fi] = fx[0];
          wk.flux[d][(1 + d) * nf + fi] = fx[1];
          wk.flux[d][(1 + t1) * nf + fi] = fx[2];
          wk.flux[d][(1 + t2) * nf + fi] = fx[3];
          wk.flux[d][4 * nf + fi] = fx[4];
          // passive scalars: C_i reconstructed on the face like the other
          // primitives and carried by the mass flux from the upwind side
          for (int v = 5; v < g.nv; ++v) {
            T cline[6];
            for (int o = -3; o <= 2; ++o) {
              int idx[3] = {i, j, k};
              idx[d] += o;
              cline[o + 3] = (o < -sten || o > sten - 1) ? T(0.0) : wk.w[v * nc + g.c(idx[0], idx[1], idx[2])];
            }
            T cl, cr;
            recon_face(recon, &cline[3], cl, cr);
            wk.flux[d][v * nf + fi] = val(fx[0]) >= 0.0 ? fx[0] * cl : fx[0] * cr;
          }
          // E = -v x B: the flux of B_t1 along d is -E_t2, that of B_t2 is +E_t1
          wk.emf_t2[d][fi] = -fx[5];
          wk.emf_t1[d][fi] = fx[6];
          // upwind weight from the sign of the mass flux (Gardiner & Stone 2005)
          T wgt;
          if (cfg.ct_eps > 0.0) {
            T rhobar = 0.5 * (wl[0] + wr[0]);
            T ramp = 0.5 + 0.5 * (fx[0] / rhobar) / (cfg.ct_eps * smax);
            wgt = vmin(T(1.0), vmax(T(0.0), ramp));
          } else {
            wgt = val(fx[0]) > 0.0 ? T(1.0) : (val(fx[0]) < 0.0 ? T(0.0) : T(0.5));
          }
          wk.wgt[d][fi] = wgt;
        }
  }

  // cell-centred EMF E = -v x B over the active cells and one ring around them
  wk.ecc.assign(3 * nc, T(0.0));
  for (int k = g.s(2) - 1; k <= g.e(2) + 1; ++k)
    for (int j = g.s(1) - 1; j <= g.e(1) + 1; ++j)
      for (int i = g.s(0) - 1; i <= g.e(0) + 1; ++i) {
        size_t q = g.c(i, j, k);
        T v1 = wk.w[1 * nc + q], v2 = wk.w[2 * nc + q], v3 = wk.w[3 * nc + q];
        T b1 = wk.bcc[0 * nc + q], b2 = wk.bcc[1 * nc + q], b3 = wk.bcc[2 * nc + q];
        wk.ecc[0 * nc + q] = -(v2 * b3 - v3 * b2);
        wk.ecc[1 * nc + q] = -(v3 * b1 - v1 * b3);
        wk.ecc[2 * nc + q] = -(v1 * b2 - v2 * b1);
      }

  // corner EMFs: component e on the edge at the lower corner, in directions
  // a = e+1 and b = e+2 (cyclic), of cell c
  wk.edge.assign(3 * nf, T(0.0));
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    const std::vector<T>& ea = wk.emf_t2[a];  // component e from faces normal to a
    const std::vector<T>& eb = wk.emf_t1[b];  // component e from faces normal to b
    const std::vector<T>& wa = wk.wgt[a];
    const std::vector<T>& wb = wk.wgt[b];
    const T* ec = wk.ecc.data() + (size_t)e * nc;
    int lo[3], hi[3];
    for (int x = 0; x < 3; ++x) { lo[x] = g.s(x); hi[x] = g.e(x) + 1; }
    hi[e] = g.e(e);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int c0[3] = {i, j, k};
          int cA[3] = {i, j, k}; cA[a] -= 1;           // c - a
          int cB[3] = {i, j, k}; cB[b] -= 1;           // c - b
          int cAB[3] = {i, j, k}; cAB[a] -= 1; cAB[b] -= 1;
          T Ea_c = ea[g.f(c0[0], c0[1], c0[2])], Ea_mb = ea[g.f(cB[0], cB[1], cB[2])];
          T Eb_c = eb[g.f(c0[0], c0[1], c0[2])], Eb_ma = eb[g.f(cA[0], cA[1], cA[2])];
          T wa_c = wa[g.f(c0[0], c0[1], c0[2])], wa_mb = wa[g.f(cB[0], cB[1], cB[2])];
          T wb_c = wb[g.f(c0[0], c0[1], c0[2])], wb_ma = wb[g.f(cA[0], cA[1], cA[2])];
          T Ec_c = ec[g.c(c0[0], c0[1], c0[2])], Ec_a = ec[g.c(cA[0], cA[1], cA[2])];
          T Ec_b = ec[g.c(cB[0], cB[1], cB[2])], Ec_ab = ec[g.c(cAB[0], cAB[1], cAB[2])];
          T avg = 0.25 * (Ea_c + Ea_mb + Eb_c + Eb_ma);
          // derivatives along b at the two quarter points, upwinded by the a-face mass flux
          T db_p = wa_c * (Ec_a - Eb_ma) + (1.0 - wa_c) * (Ec_c - Eb_c);
          T db_m = wa_mb * (Eb_ma - Ec_ab) + (1.0 - wa_mb) * (Eb_c - Ec_b);
          // derivatives along a, upwinded by the b-face mass flux
          T da_p = wb_c * (Ec_b - Ea_mb) + (1.0 - wb_c) * (Ec_c - Ea_c);
          T da_m = wb_ma * (Ea_mb - Ec_ab) + (1.0 - wb_ma) * (Ea_c - Ec_a);
          wk.edge[(size_t)e * nf + g.f(i, j, k)] = avg + 0.25 * (db_m - db_p) + 0.25 * (da_m - da_p);
        }
  }
  return bad;
}

// -(curl E)_d on face (i, j, k) normal to d, from the corner EMFs of wk.
template <class T> T face_curl(const Geo& g, const double* dx, const Work<T>& wk, int d, int i, int j, int k) {
  const size_t nf = g.nface();
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  int p1[3] = {i, j, k}; p1[t1] += 1;
  int p2[3] = {i, j, k}; p2[t2] += 1;
  size_t f0 = g.f(i, j, k);
  T curl = (wk.edge[(size_t)t2 * nf + g.f(p1[0], p1[1], p1[2])] - wk.edge[(size_t)t2 * nf + f0]) / dx[t1] -
           (wk.edge[(size_t)t1 * nf + g.f(p2[0], p2[1], p2[2])] - wk.edge[(size_t)t1 * nf + f0]) / dx[t2];
  return -curl;
}

// Flux divergence on the active cells and the CT update rate of the active
// faces (step 7 without the 2S weights) from the fluxes and EMFs of wk.
template <class T> void apply_operator(const Cfg& cfg, const Geo& g, const Work<T>& wk, T* du, T* db) {
  const size_t nc = g.ncell(), nf = g.nface();
  const double dx[3] = {cfg.dx1, cfg.dx2, cfg.dx3};
  // flux divergence on the active cells
  for (int k = g.s(2); k <= g.e(2); ++k)
    for (int j = g.s(1); j <= g.e(1); ++j)
      for (int i = g.s(0); i <= g.e(0); ++i) {
        size_t q = g.c(i, j, k);
        for (int v = 0; v < g.nv; ++v) {
          T sum(0.0);
          for (int d = 0; d < 3; ++d) {
            int up[3] = {i, j, k};
            up[d] += 1;
            sum = sum + (wk.flux[d][v * nf + g.f(up[0], up[1], up[2])] - wk.flux[d][v * nf + g.f(i, j, k)]) / dx[d];
          }
          du[v * nc + q] = -sum;
        }
      }
  // CT: dB_d/dt = -(curl E)_d on the active faces (index [s, e] in every
  // direction; the periodic image face is set by the ghost fill)
  for (int d = 0; d < 3; ++d)
    for (int k = g.s(2); k <= g.e(2); ++k)
      for (int j = g.s(1); j <= g.e(1); ++j)
        for (int i = g.s(0); i <= g.e(0); ++i) db[(size_t)d * nf + g.f(i, j, k)] = face_curl(g, dx, wk, d, i, j, k);
}

template <class T>
int spatial_operator(const Cfg& cfg, const Geo& g, int recon, const T* cons, const T* bf, T* du, T* db, Work<T>& wk) {
  const int bad = compute_fluxes(cfg, g, recon, cons, bf, wk);
  apply_operator(cfg, g, wk, du, db);
  return bad;
}

// ---------------------------------------------------------------------------
// 2S low-storage time integration, Eq. (rk-2s), coefficient sets of
// Sec. 3.2.3.  delta_s, gamma_s0, gamma_s1, beta_s per stage.
// ---------------------------------------------------------------------------
struct Scheme {
  int nstage;
  double delta[3], g0[3], g1[3], beta[3];
};

inline bool scheme_for(int integrator, Scheme& s) {
  switch (integrator) {
    case INT_RK1: s = {1, {1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {1.0, 0, 0}}; return true;
    case INT_VL2: s = {2, {1, 0, 0}, {0, 0, 0}, {1, 1, 0}, {0.5, 1.0, 0}}; return true;
    case INT_RK2: s = {2, {1, 0, 0}, {0, 0.5, 0}, {1, 0.5, 0}, {1.0, 0.5, 0}}; return true;
    case INT_RK3:
      s = {3, {1, 0, 0}, {0, 0.25, 2.0 / 3.0}, {1, 0.75, 1.0 / 3.0}, {1.0, 0.25, 2.0 / 3.0}};
      return true;
  }
  return false;
}

// One step of the 2S driver for a generic state vector; `rhs(stage, u0, L)`
// evaluates the spatial operator.  Elements with mask==0 (ghosts, padding) are
// left as they are.
template <class T, class Rhs>
int drive_2s(const Scheme& sc, size_t n, T* u0, const unsigned char* mask, double dt, Rhs rhs) {
  return drive_2s(sc, n, u0, mask, dt, rhs, [](T*) {});
}

// Same, with `post(u0)` applied to the state after every stage.
template <class T, class Rhs, class Post>
int drive_2s(const Scheme& sc, size_t n, T* u0, const unsigned char* mask, double dt, Rhs rhs, Post post) {
  std::vector<T> u1(n, T(0.0)), L(n, T(0.0));
  int bad = 0;
  for (int s = 0; s < sc.nstage; ++s) {
    for (size_t q = 0; q < n; ++q) u1[q] = u1[q] + sc.delta[s] * u0[q];
    int b = rhs(s, u0, L.data());
    if (b < 0) return b;
    bad += b;
    for (size_t q = 0; q < n; ++q)
      if (mask[q]) u0[q] = sc.g0[s] * u0[q] + sc.g1[s] * u1[q] + sc.beta[s] * dt * L[q];
    post(u0);
  }
  return bad;
}

// Floors on the conserved state after a stage (only with floors enabled):
// density below dfloor is raised to dfloor, and where the pressure implied by
// (U, B) is below pfloor the total energy is raised so that it equals pfloor
// (kinetic and magnetic energy unchanged).  The cell-centred field uses the
// lower face and the periodic image of the upper one.  Returns the number of
// cells changed.
template <class T> int floor_state(const Cfg& cfg, const Geo& g, T* cons, const T* bf) {
  const size_t nc = g.ncell(), nf = g.nface();
  int changed = 0;
  for (int k = g.s(2); k <= g.e(2); ++k)
    for (int j = g.s(1); j <= g.e(1); ++j)
      for (int i = g.s(0); i <= g.e(0); ++i) {
        const size_t q = g.c(i, j, k);
        T b[3];
        for (int d = 0; d < 3; ++d) {
          int up[3] = {i, j, k};
          up[d] = g.wrap(up[d] + 1, d);
          b[d] = 0.5 * (bf[d * nf + g.f(i, j, k)] + bf[d * nf + g.f(up[0], up[1], up[2])]);
        }
        bool hit = false;
        if (!(val(cons[q]) >= cfg.dfloor)) {
          cons[q] = T(cfg.dfloor);
          hit = true;
        }
        const T rho = cons[q];
        const T kin = 0.5 * (cons[nc + q] * cons[nc + q] + cons[2 * nc + q] * cons[2 * nc + q] +
                             cons[3 * nc + q] * cons[3 * nc + q]) / rho;
        const T mag = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        const T p = (cfg.gamma - 1.0) * (cons[4 * nc + q] - kin - mag);
        if (!(val(p) >= cfg.pfloor)) {
          cons[4 * nc + q] = cfg.pfloor / (cfg.gamma - 1.0) + kin + mag;
          hit = true;
        }
        if (hit) ++changed;
      }
  return changed;
}

// Full MHD step: state = cons (5 cell arrays) followed by bface (3 face arrays)
template <class T> int step(const Cfg& cfg, T* cons, T* bf, double dt) {
  Geo g(cfg);
  Scheme sc;
  if (!scheme_for(cfg.integrator, sc)) return -1;
  const size_t nc = g.ncell(), nf = g.nface();
  const size_t ncv = g.nv * nc;  // cell part of the state: MHD variables and scalars
  const size_t n = ncv + 3 * nf;
  std::vector<T> u(n);
  std::copy(cons, cons + ncv, u.begin());
  std::copy(bf, bf + 3 * nf, u.begin() + ncv);
  std::vector<unsigned char> mask(n, 0);
  for (int v = 0; v < g.nv; ++v)
    for (int k = g.s(2); k <= g.e(2); ++k)
      for (int j = g.s(1); j <= g.e(1); ++j)
        for (int i = g.s(0); i <= g.e(0); ++i) mask[v * nc + g.c(i, j, k)] = 1;
  for (int d = 0; d < 3; ++d)
    for (int k = g.s(2); k <= g.e(2); ++k)
      for (int j = g.s(1); j <= g.e(1); ++j)
        for (int i = g.s(0); i <= g.e(0); ++i) mask[ncv + d * nf + g.f(i, j, k)] = 1;
  Work<T> wk;
  auto rhs = [&](int s, T* state, T* L) -> int {
    fill_ghosts(g, state, state + ncv);
    std::fill(L, L + n, T(0.0));
    // the VL2 predictor always uses donor-cell fluxes
    int recon = (cfg.integrator == INT_VL2 && s == 0) ? RECON_DC : cfg.recon;
    return spatial_operator(cfg, g, recon, state, state + ncv, L, L + ncv, wk);
  };
  int bad;
  if (cfg.dfloor > 0.0 || cfg.pfloor > 0.0)
    bad = drive_2s(sc, n, u.data(), mask.data(), dt, rhs,
                   [&](T* state) { g_floored += floor_state(cfg, g, state, state + ncv); });
  else
    bad = drive_2s(sc, n, u.data(), mask.data(), dt, rhs);
  if (bad < 0) return bad;
  fill_ghosts(g, u.data(), u.data() + ncv);
  std::copy(u.begin(), u.begin() + ncv, cons);
  std::copy(u.begin() + ncv, u.end(), bf);
  return bad;
}

// Global time step: C0 times the smallest dx_d / (|v_d| + c_f,d) over the
// active cells (Sec. 2.1.7 and the CFL limits of Sec. 3.2.3).
inline int newdt(const Cfg& cfg, const double* cons, const double* bf, double* dt_out) {
  Geo g(cfg);
  const size_t nc = g.ncell();
  std::vector<double> w(g.nv * nc), bcc(3 * nc);
  int bad = cons_to_prim(g, cfg.gamma, cons, bf, w.data(), bcc.data(), cfg.dfloor, cfg.pfloor);
  const double dx[3] = {cfg.dx1, cfg.dx2, cfg.dx3};
  double best = INFINITY;
  for (int k = g.s(2); k <= g.e(2); ++k)
    for (int j = g.s(1); j <= g.e(1); ++j)
      for (int i = g.s(0); i <= g.e(0); ++i) {
        size_t q = g.c(i, j, k);
        for (int d = 0; d < 3; ++d) {
          int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
          double cf = fast_speed(w[q], w[4 * nc + q], bcc[d * nc + q], bcc[t1 * nc + q], bcc[t2 * nc + q], cfg.gamma);
          double dtd = dx[d] / (std::fabs(w[(1 + d) * nc + q]) + cf);
          if (dtd < best) best = dtd;
        }
      }
  *dt_out = cfg.cfl * best;
  return bad;
}

// ---------------------------------------------------------------------------
// Restriction and prolongation between a coarse block and the fine block that
// refines one octant of it (Sec. 2.1.5), for block refinement / derefinement.
// Both blocks have the geometry of cfg (n cells per side, even; ng ghosts;
// the fine cells half as wide).  (ox, oy, oz): the octant's first active
// coarse cell, 0 or n/2 along each direction.
//   restriction: volume average of the 8 fine cells (all nv cell arrays);
//     area average of the 4 fine faces on each coarse face of the octant
//     (the octant's upper faces read the fine block's image faces);
//   prolongation of cells: U_C + the minmod-limited slopes along each
//     direction times the offsets +-1/4 (coarse cell units) of the children;
//   prolongation of faces (Toth & Roe 2002): each coarse face of the octant
//     (and its upper neighbours) split into 4 fine faces by the 2D
//     minmod-limited linear profile on the face; the 12 faces inside each
//     coarse cell from the conditions that every fine cell has the coarse
//     cell's divergence and that the curl at each of the 6 interior edges
//     equals its estimate from the outer faces (the mean of the tangential
//     differences on the two outer faces parallel to the edge's planes) --
//     14 equations of rank 12, solved here by least squares (normal
//     equations), consistent when the outer values are.
// ---------------------------------------------------------------------------
template <class T> T minmod(const T& a, const T& b) {
  if (val(a) > 0.0 && val(b) > 0.0) return vmin(a, b);
  if (val(a) < 0.0 && val(b) < 0.0) return vmax(a, b);
  return T(0.0);
}

// A box of the level operators: fine cells [f, f + 2 h) and coarse cells
// [c, c + h) along each direction (stored indices, ghosts included); an
// octant is f = ng, c = ng + o_d n_d / 2, h = n / 2.
struct LevelBox {
  int f[3], c[3], h[3];
};

inline LevelBox octant_box(const Geo& g, const int o[3]) {
  LevelBox B;
  for (int d = 0; d < 3; ++d) {
    B.f[d] = g.ng;
    B.c[d] = g.ng + o[d];
    B.h[d] = g.n[d] / 2;
  }
  return B;
}

inline void restrict_box(const Geo& g, const double* fc, const double* fb, double* cc, double* cb, const LevelBox& B) {
  const size_t nc = g.ncell(), nf = g.nface();
  const int* h = B.h;
  for (int v = 0; v < g.nv; ++v)
    for (int c = 0; c < h[2]; ++c)
      for (int b = 0; b < h[1]; ++b)
        for (int a = 0; a < h[0]; ++a) {
          double sum = 0.0;
          for (int s3 = 0; s3 < 2; ++s3)
            for (int s2 = 0; s2 < 2; ++s2)
              for (int s1 = 0; s1 < 2; ++s1)
                sum += fc[v * nc + g.c(B.f[0] + 2 * a + s1, B.f[1] + 2 * b + s2, B.f[2] + 2 * c + s3)];
          cc[v * nc + g.c(B.c[0] + a, B.c[1] + b, B.c[2] + c)] = sum / 8.0;
        }
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int lim[3] = {h[0], h[1], h[2]};
    lim[d] = h[d] + 1;  // the box's upper faces too
    for (int c = 0; c < lim[2]; ++c)
      for (int b = 0; b < lim[1]; ++b)
        for (int a = 0; a < lim[0]; ++a) {
          const int q[3] = {a, b, c};
          double sum = 0.0;
          for (int u = 0; u < 2; ++u)
            for (int w = 0; w < 2; ++w) {
              int f[3];
              f[d] = B.f[d] + 2 * q[d];
              f[t1] = B.f[t1] + 2 * q[t1] + u;
              f[t2] = B.f[t2] + 2 * q[t2] + w;
              sum += fb[d * nf + g.f(f[0], f[1], f[2])];
            }
          cb[d * nf + g.f(B.c[0] + a, B.c[1] + b, B.c[2] + c)] = sum / 4.0;
        }
  }
}

// Solve the least-squares problem min |A x - r| (rows x 12) by the normal
// equations with Gaussian elimination (partial pivoting).
inline void lsq12(const std::vector<std::array<double, 12>>& A, const std::vector<double>& r, double* x) {
  double N[12][13];
  for (int i = 0; i < 12; ++i) {
    for (int j = 0; j < 12; ++j) {
      double s = 0.0;
      for (size_t k = 0; k < A.size(); ++k) s += A[k][i] * A[k][j];
      N[i][j] = s;
    }
    double s = 0.0;
    for (size_t k = 0; k < A.size(); ++k) s += A[k][i] * r[k];
    N[i][12] = s;
  }
  for (int c = 0; c < 12; ++c) {
    int piv = c;
    for (int i = c + 1; i < 12; ++i)
      if (std::fabs(N[i][c]) > std::fabs(N[piv][c])) piv = i;
    for (int k = 0; k < 13; ++k) std::swap(N[c][k], N[piv][k]);
    for (int i = c + 1; i < 12; ++i) {
      const double f = N[i][c] / N[c][c];
      for (int k = c; k < 13; ++k) N[i][k] -= f * N[c][k];
    }
  }
  for (int c = 11; c >= 0; --c) {
    double s = N[c][12];
    for (int k = c + 1; k < 12; ++k) s -= N[c][k] * x[k];
    x[c] = s / N[c][c];
  }
}

// Cell-centred field of cell (i, j, k) from the stored faces: the mean of the
// two faces that bound it along each direction (no periodic wrap).
inline void cell_field_stored(const Geo& g, const double* bf, int i, int j, int k, double b[3]) {
  const size_t nf = g.nface();
  for (int d = 0; d < 3; ++d) {
    int up[3] = {i, j, k};
    up[d] += 1;
    b[d] = 0.5 * (bf[d * nf + g.f(i, j, k)] + bf[d * nf + g.f(up[0], up[1], up[2])]);
  }
}

// primitive = false: the cell arrays prolonged are the conserved variables
// themselves (new blocks); with pfloor > 0 the pressure floor follows.
// primitive = true: the coarse cells the octant reads (the octant and one
// layer around it) are converted to primitives (rho, v, P, C_i) with their
// cell-centred field, the primitives are prolonged, and each fine cell is
// converted back to conserved variables with the cell-centred field of the
// prolonged fine faces (Sec. 2.1.5 uses this between levels: conserved
// values are exchanged, prolongation acts on primitives).
// keep: bit 2 d + S set -> the fine faces of component d on side S (0 lower,
// 1 upper) of the box already hold fine-level values; they are neither
// overwritten nor recomputed, and the interior faces are solved with them
// (Sec. 2.1.5: fine faces that exist at the fine level are used instead of
// prolonged ones).
inline void prolong_box(const Geo& g, const double* cc, const double* cb, double* fc, double* fb, const LevelBox& B,
                        double gamma, double pfloor, bool primitive, int keep = 0) {
  const size_t nc = g.ncell(), nf = g.nface();
  const int* h = B.h;
  std::vector<double> wc, wf;
  if (primitive) {
    wc.assign(g.nv * nc, 0.0);
    wf.assign(g.nv * nc, 0.0);
    for (int k = B.c[2] - 1; k <= B.c[2] + h[2]; ++k)
      for (int j = B.c[1] - 1; j <= B.c[1] + h[1]; ++j)
        for (int i = B.c[0] - 1; i <= B.c[0] + h[0]; ++i) {
          const size_t q = g.c(i, j, k);
          double b[3];
          cell_field_stored(g, cb, i, j, k, b);
          const double rho = cc[q];
          const double v1 = cc[nc + q] / rho, v2 = cc[2 * nc + q] / rho, v3 = cc[3 * nc + q] / rho;
          const double kin = 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3);
          const double mag = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
          wc[q] = rho;
          wc[nc + q] = v1;
          wc[2 * nc + q] = v2;
          wc[3 * nc + q] = v3;
          wc[4 * nc + q] = (gamma - 1.0) * (cc[4 * nc + q] - kin - mag);
          for (int v = 5; v < g.nv; ++v) wc[v * nc + q] = cc[v * nc + q] / rho;
        }
  }
  const double* src = primitive ? wc.data() : cc;
  double* dst = primitive ? wf.data() : fc;
  // cells: U_C + sum_d minmod slope_d * (+-1/4)
  for (int v = 0; v < g.nv; ++v)
    for (int c = 0; c < h[2]; ++c)
      for (int b = 0; b < h[1]; ++b)
        for (int a = 0; a < h[0]; ++a) {
          const int C[3] = {B.c[0] + a, B.c[1] + b, B.c[2] + c};
          const double u0 = src[v * nc + g.c(C[0], C[1], C[2])];
          double sl[3];
          for (int d = 0; d < 3; ++d) {
            int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
            m[d] -= 1;
            p[d] += 1;
            sl[d] = minmod(u0 - src[v * nc + g.c(m[0], m[1], m[2])], src[v * nc + g.c(p[0], p[1], p[2])] - u0);
          }
          for (int s3 = 0; s3 < 2; ++s3)
            for (int s2 = 0; s2 < 2; ++s2)
              for (int s1 = 0; s1 < 2; ++s1)
                dst[v * nc + g.c(B.f[0] + 2 * a + s1, B.f[1] + 2 * b + s2, B.f[2] + 2 * c + s3)] =
                    u0 + 0.25 * ((2 * s1 - 1) * sl[0] + (2 * s2 - 1) * sl[1] + (2 * s3 - 1) * sl[2]);
        }
  // outer fine faces: each coarse face of the octant (upper ones included)
  // split by the minmod-limited linear profile along its two transverse
  // directions
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int lim[3] = {h[0], h[1], h[2]};
    lim[d] = h[d] + 1;
    for (int c = 0; c < lim[2]; ++c)
      for (int b = 0; b < lim[1]; ++b)
        for (int a = 0; a < lim[0]; ++a) {
          const int q[3] = {a, b, c};
          if ((q[d] == 0 && ((keep >> (2 * d)) & 1)) || (q[d] == h[d] && ((keep >> (2 * d + 1)) & 1))) continue;
          const int C[3] = {B.c[0] + a, B.c[1] + b, B.c[2] + c};
          const double b0 = cb[d * nf + g.f(C[0], C[1], C[2])];
          double sl[2];
          for (int e = 0; e < 2; ++e) {
            const int t = e == 0 ? t1 : t2;
            int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
            m[t] -= 1;
            p[t] += 1;
            sl[e] = minmod(b0 - cb[d * nf + g.f(m[0], m[1], m[2])], cb[d * nf + g.f(p[0], p[1], p[2])] - b0);
          }
          for (int u = 0; u < 2; ++u)
            for (int w = 0; w < 2; ++w) {
              int f[3];
              f[d] = B.f[d] + 2 * q[d];
              f[t1] = B.f[t1] + 2 * q[t1] + u;
              f[t2] = B.f[t2] + 2 * q[t2] + w;
              fb[d * nf + g.f(f[0], f[1], f[2])] = b0 + 0.25 * ((2 * u - 1) * sl[0] + (2 * w - 1) * sl[1]);
            }
        }
  }
  // interior fine faces of each coarse cell
  for (int c = 0; c < h[2]; ++c)
    for (int b = 0; b < h[1]; ++b)
      for (int a = 0; a < h[0]; ++a) {
        const int base[3] = {B.f[0] + 2 * a, B.f[1] + 2 * b, B.f[2] + 2 * c};
        // face value of component d at fine offset (x, y, z) in {0, 1, 2} from base
        auto face = [&](int d, int x, int y, int z) -> double& {
          return fb[d * nf + g.f(base[0] + x, base[1] + y, base[2] + z)];
        };
        // unknown numbering: component d, halves (p, q) of its transverse
        // directions (t1, t2) in {0, 1}: 4 d + 2 p + q
        auto unk = [](int d, int p, int q) { return 4 * d + 2 * p + q; };
        // offset of the interior face of component d with its t1-half p and t2-half q
        auto at = [](int d, int mid, int p, int q, int* x) {
          x[d] = mid;
          x[(d + 1) % 3] = p;
          x[(d + 2) % 3] = q;
        };
        std::vector<std::array<double, 12>> A;
        std::vector<double> r;
        // coarse divergence density (unit fine spacing): sum over directions
        // of (mean upper outer value - mean lower outer value) / 2
        double dc = 0.0;
        for (int d = 0; d < 3; ++d) {
          double up = 0.0, lo = 0.0;
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
              int x[3];
              at(d, 2, p, q, x);
              up += face(d, x[0], x[1], x[2]);
              at(d, 0, p, q, x);
              lo += face(d, x[0], x[1], x[2]);
            }
          dc += (up - lo) / 4.0 / 2.0;
        }
        // every fine cell (s1, s2, s3): its divergence equals dc
        for (int s3 = 0; s3 < 2; ++s3)
          for (int s2 = 0; s2 < 2; ++s2)
            for (int s1 = 0; s1 < 2; ++s1) {
              const int s[3] = {s1, s2, s3};
              std::array<double, 12> row{};
              double rhs = dc;
              for (int d = 0; d < 3; ++d) {
                const int p = s[(d + 1) % 3], q = s[(d + 2) % 3];
                int x[3];
                at(d, 2 * s[d], p, q, x);  // outer face of this cell along d
                const double outer = face(d, x[0], x[1], x[2]);
                const double sg = s[d] == 1 ? 1.0 : -1.0;  // upper cell: outer - inner, lower: inner - outer
                rhs -= sg * outer;
                row[unk(d, p, q)] -= sg;
              }
              A.push_back(row);
              r.push_back(rhs);
            }
        // interior edges along e, at half h of direction e: curl_e =
        // d(B_b)/d(a) - d(B_a)/d(b) with (a, b) = (e+1, e+2)
        for (int e = 0; e < 3; ++e) {
          const int ea = (e + 1) % 3, eb = (e + 2) % 3;
          for (int hh = 0; hh < 2; ++hh) {
            std::array<double, 12> row{};
            // interior faces of component eb (normal to eb) at the two halves
            // of ea; of component ea at the two halves of eb
            // unknown halves of component eb: (t1, t2) = (e, ea)
            row[unk(eb, hh, 1)] += 1.0;
            row[unk(eb, hh, 0)] -= 1.0;
            // component ea: (t1, t2) = (eb, e)
            row[unk(ea, 1, hh)] -= 1.0;
            row[unk(ea, 0, hh)] += 1.0;
            // estimate from the outer faces: means over the two outer planes
            double est = 0.0;
            for (int side = 0; side < 2; ++side) {
              int x[3];
              at(eb, 2 * side, hh, 1, x);
              est += 0.5 * face(eb, x[0], x[1], x[2]);
              at(eb, 2 * side, hh, 0, x);
              est -= 0.5 * face(eb, x[0], x[1], x[2]);
              at(ea, 2 * side, 1, hh, x);
              est -= 0.5 * face(ea, x[0], x[1], x[2]);
              at(ea, 2 * side, 0, hh, x);
              est += 0.5 * face(ea, x[0], x[1], x[2]);
            }
            A.push_back(row);
            r.push_back(est);
          }
        }
        double xs[12];
        lsq12(A, r, xs);
        for (int d = 0; d < 3; ++d)
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
              int x[3];
              at(d, 1, p, q, x);
              face(d, x[0], x[1], x[2]) = xs[unk(d, p, q)];
            }
      }
  // primitive prolongation: back to conserved variables with the fine
  // cell-centred field
  if (primitive)
    for (int k = B.f[2]; k < B.f[2] + 2 * h[2]; ++k)
      for (int j = B.f[1]; j < B.f[1] + 2 * h[1]; ++j)
        for (int i = B.f[0]; i < B.f[0] + 2 * h[0]; ++i) {
          const size_t q = g.c(i, j, k);
          double b[3];
          cell_field_stored(g, fb, i, j, k, b);
          const double rho = wf[q], v1 = wf[nc + q], v2 = wf[2 * nc + q], v3 = wf[3 * nc + q];
          fc[q] = rho;
          fc[nc + q] = rho * v1;
          fc[2 * nc + q] = rho * v2;
          fc[3 * nc + q] = rho * v3;
          fc[4 * nc + q] = wf[4 * nc + q] / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) +
                           0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
          for (int v = 5; v < g.nv; ++v) fc[v * nc + q] = rho * wf[v * nc + q];
        }
  // Pressure floor on the refined cells (pfloor > 0 only; Sec. 2.1.5 applies
  // one when prolonged conserved variables give a negative pressure): where
  // the pressure implied by the fine U and the cell-centred field of the fine
  // faces (mean of the two bounding faces) is below pfloor, E is raised to
  // give pfloor; rho and M, hence mass and momentum, are unchanged.
  if (pfloor > 0.0 && !primitive)
    for (int k = B.f[2]; k < B.f[2] + 2 * h[2]; ++k)
      for (int j = B.f[1]; j < B.f[1] + 2 * h[1]; ++j)
        for (int i = B.f[0]; i < B.f[0] + 2 * h[0]; ++i) {
          const size_t q = g.c(i, j, k);
          double b[3];
          for (int d = 0; d < 3; ++d) {
            int up[3] = {i, j, k};
            up[d] += 1;
            b[d] = 0.5 * (fb[d * nf + g.f(i, j, k)] + fb[d * nf + g.f(up[0], up[1], up[2])]);
          }
          const double rho = fc[q];
          const double kin = 0.5 * (fc[nc + q] * fc[nc + q] + fc[2 * nc + q] * fc[2 * nc + q] +
                                    fc[3 * nc + q] * fc[3 * nc + q]) / rho;
          const double mag = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
          const double p = (gamma - 1.0) * (fc[4 * nc + q] - kin - mag);
          if (!(p >= pfloor)) fc[4 * nc + q] = pfloor / (gamma - 1.0) + kin + mag;
        }
}


// ---------------------------------------------------------------------------
// Two-level composite (Sec. 2.1.3: communication between levels; Sec. 2.1.4:
// flux and EMF correction; reading R-35).  Nine blocks of one shape (n cells
// per direction, ng ghosts).  Block 0 is coarse (widths dx of cfg) and covers
// [X, 2X) x [0, Y) x [0, Z) with X = n1 dx1, Y = n2 dx2, Z = n3 dx3; block
// 1 + a + 2b + 4c (a, b, c in {0, 1}) is fine (widths dx / 2) and covers the
// octant (a, b, c) of [0, X) x [0, Y) x [0, Z).  The domain
// [0, 2X) x [0, Y) x [0, Z) is periodic.  n1, n2, n3 are even and at least
// 2 ng, and ng is even.
//
// Faces: a block owns the lower faces of its active cells.  Both coarse-fine
// interfaces (x1 = X and x1 = 2X = 0) are owned by the fine side: the fine
// blocks with a = 1 also own their upper x1 faces, and the coarse block's two
// x1 boundary faces are area averages of the fine faces there (restriction),
// which the EMF correction keeps equal to what the coarse CT update would
// give.
// ---------------------------------------------------------------------------
struct TwoLevel {
  Cfg cc, cf;  // coarse and fine configuration (fine: dx / 2)
  Geo g;
  size_t ncv, nf, bs;  // cell part, face array, doubles per block
  explicit TwoLevel(const Cfg& c) : cc(c), cf(c), g(c) {
    cf.dx1 = 0.5 * c.dx1;
    cf.dx2 = 0.5 * c.dx2;
    cf.dx3 = 0.5 * c.dx3;
    ncv = g.nv * g.ncell();
    nf = g.nface();
    bs = ncv + 3 * nf;
  }
  const Cfg& cfg(int b) const { return b == 0 ? cc : cf; }
};

inline bool two_level_ok(const Cfg& c) {
  return c.ng % 2 == 0 && c.n1 % 2 == 0 && c.n2 % 2 == 0 && c.n3 % 2 == 0 && c.n1 >= 2 * c.ng &&
         c.n2 >= 2 * c.ng && c.n3 >= 2 * c.ng && c.nscalars == 0;
}

// Same-level ghosts of the fine blocks: every stored cell or face of a fine
// block that lies inside the fine region (periodic along x2 and x3) and is
// not owned by that block is copied from the fine block that owns it.
// Entries beyond the region along x1 are left to prolongation.
inline void two_level_fine_exchange(const TwoLevel& L, std::vector<double*>& cons, std::vector<double*>& bf) {
  const Geo& g = L.g;
  const int n[3] = {g.n[0], g.n[1], g.n[2]}, ng = g.ng;
  for (int blk = 1; blk <= 8; ++blk) {
    const int pos[3] = {(blk - 1) & 1, ((blk - 1) >> 1) & 1, ((blk - 1) >> 2) & 1};
    // cells
    for (int k = 0; k < g.N[2]; ++k)
      for (int j = 0; j < g.N[1]; ++j)
        for (int i = 0; i < g.N[0]; ++i) {
          const int idx[3] = {i, j, k};
          bool act = true;
          int src[3], sb[3];
          bool inside = true;
          for (int d = 0; d < 3; ++d) {
            int gl = pos[d] * n[d] + idx[d] - ng;  // index in the fine region
            if (idx[d] < ng || idx[d] >= ng + n[d]) act = false;
            if (d == 0) {
              if (gl < 0 || gl >= 2 * n[0]) inside = false;
            } else {
              gl = ((gl % (2 * n[d])) + 2 * n[d]) % (2 * n[d]);
            }
            sb[d] = gl / n[d];
            src[d] = ng + gl - sb[d] * n[d];
          }
          if (act || !inside) continue;
          const int sblk = 1 + sb[0] + 2 * sb[1] + 4 * sb[2];
          for (int v = 0; v < g.nv; ++v)
            cons[blk][v * g.ncell() + g.c(i, j, k)] = cons[sblk][v * g.ncell() + g.c(src[0], src[1], src[2])];
        }
    // faces of component d
    for (int d = 0; d < 3; ++d)
      for (int k = 0; k <= g.N[2]; ++k)
        for (int j = 0; j <= g.N[1]; ++j)
          for (int i = 0; i <= g.N[0]; ++i) {
            const int idx[3] = {i, j, k};
            // owned: lower faces of active cells, and for a = 1 the upper x1 faces
            bool owned = true;
            for (int e = 0; e < 3; ++e) {
              const int hi = (e == 0 && d == 0 && pos[0] == 1) ? ng + n[0] : ng + n[e] - 1;
              if (idx[e] < ng || idx[e] > hi) owned = false;
            }
            if (owned) continue;
            int src[3], sb[3];
            bool inside = true;
            for (int e = 0; e < 3; ++e) {
              int gl = pos[e] * n[e] + idx[e] - ng;
              if (e == 0) {
                // x1 faces up to the interface x1 = X (index 2 n1) are in the region
                const int top = d == 0 ? 2 * n[0] : 2 * n[0] - 1;
                if (gl < 0 || gl > top) inside = false;
                sb[e] = std::min(gl / n[e], 1);
              } else {
                gl = ((gl % (2 * n[e])) + 2 * n[e]) % (2 * n[e]);
                sb[e] = gl / n[e];
              }
              src[e] = ng + gl - sb[e] * n[e];
            }
            if (!inside) continue;
            const int sblk = 1 + sb[0] + 2 * sb[1] + 4 * sb[2];
            bf[blk][d * L.nf + g.f(i, j, k)] = bf[sblk][d * L.nf + g.f(src[0], src[1], src[2])];
          }
  }
}

// Ghosts of the whole composite: fine same-level exchange; the coarse block's
// periodic images along x2 and x3, with its x1 ghost slabs and x1 boundary
// faces restricted from the fine blocks; the fine blocks' x1 ghost slabs
// beyond the fine region prolongated from the coarse block (keeping the fine
// interface faces).
inline void two_level_ghosts(const TwoLevel& L, double* cons, double* bf) {
  const Geo& g = L.g;
  const int n1 = g.n[0], n2 = g.n[1], n3 = g.n[2], ng = g.ng;
  std::vector<double*> cb(9), bb(9);
  for (int b = 0; b < 9; ++b) {
    cb[b] = cons + b * L.ncv;
    bb[b] = bf + b * 3 * L.nf;
  }
  two_level_fine_exchange(L, cb, bb);
  fill_ghosts(g, cb[0], bb[0]);
  // coarse x1 slabs: segments of coarse stored indices along x2 (x3) and the
  // fine block and fine start index they restrict from
  struct Seg { int c, h, fb, f; };
  const Seg sj[4] = {{0, ng, 1, n2 - ng}, {ng, n2 / 2, 0, ng}, {ng + n2 / 2, n2 / 2, 1, ng}, {ng + n2, ng, 0, ng}};
  const Seg sk[4] = {{0, ng, 1, n3 - ng}, {ng, n3 / 2, 0, ng}, {ng + n3 / 2, n3 / 2, 1, ng}, {ng + n3, ng, 0, ng}};
  for (int side = 0; side < 2; ++side)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        LevelBox B;
        B.c[0] = side == 0 ? 0 : ng + n1;
        B.h[0] = ng;
        B.f[0] = side == 0 ? n1 - ng : ng;
        const int fa = side == 0 ? 1 : 0;
        B.c[1] = sj[a].c; B.h[1] = sj[a].h; B.f[1] = sj[a].f;
        B.c[2] = sk[c].c; B.h[2] = sk[c].h; B.f[2] = sk[c].f;
        const int fblk = 1 + fa + 2 * sj[a].fb + 4 * sk[c].fb;
        restrict_box(g, cb[fblk], bb[fblk], cb[0], bb[0], B);
      }
  // fine x1 slabs beyond the fine region, prolongated from the coarse block
  for (int blk = 1; blk <= 8; ++blk) {
    const int a = (blk - 1) & 1, b = ((blk - 1) >> 1) & 1, c = ((blk - 1) >> 2) & 1;
    LevelBox B;
    B.h[0] = ng / 2;
    B.f[0] = a == 1 ? ng + n1 : 0;
    B.c[0] = a == 1 ? ng : ng + n1 - ng / 2;
    B.f[1] = 0; B.h[1] = g.N[1] / 2; B.c[1] = ng + b * n2 / 2 - ng / 2;
    B.f[2] = 0; B.h[2] = g.N[2] / 2; B.c[2] = ng + c * n3 / 2 - ng / 2;
    const int keep = a == 1 ? 1 : 2;  // the interface face: lower x1 side (a = 1), upper (a = 0)
    prolong_box(g, cb[0], bb[0], cb[blk], bb[blk], B, L.cc.gamma, L.cc.pfloor, false, keep);
  }
}

// Fine block and stored index of global fine index gl (periodic over 2 n)
// along a direction with n cells per block.
inline void fine_pos(int gl, int n, int ng, int& blk, int& idx) {
  gl = ((gl % (2 * n)) + 2 * n) % (2 * n);
  blk = gl / n;
  idx = ng + gl - blk * n;
}

// Flux correction (the coarse fluxes through both interfaces replaced by the
// area average of the four fine fluxes) and EMF correction (Eq. emfcorr: the
// coarse E2, E3 on the interface planes replaced by the mean of the two fine
// edges along them).
inline void two_level_correct(const TwoLevel& L, std::vector<Work<double>>& wk) {
  const Geo& g = L.g;
  const int n1 = g.n[0], n2 = g.n[1], n3 = g.n[2], ng = g.ng;
  const size_t nf = L.nf;
  for (int side = 0; side < 2; ++side) {
    const int ci = side == 0 ? ng : ng + n1;  // coarse x1 face / edge plane
    const int fi = side == 0 ? ng + n1 : ng;  // the same plane in the fine blocks
    const int fa = side == 0 ? 1 : 0;
    for (int k = ng; k < ng + n3; ++k)
      for (int j = ng; j < ng + n2; ++j)
        for (int v = 0; v < g.nv; ++v) {
          double sum = 0.0;
          for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj) {
              int bj, jj, bk, kk;
              fine_pos(2 * (j - ng) + dj, n2, ng, bj, jj);
              fine_pos(2 * (k - ng) + dk, n3, ng, bk, kk);
              sum += wk[1 + fa + 2 * bj + 4 * bk].flux[0][v * nf + g.f(fi, jj, kk)];
            }
          wk[0].flux[0][v * nf + g.f(ci, j, k)] = 0.25 * sum;
        }
    // E2: along x2 over coarse cell j, at the lower x3 face k (k up to ng + n3)
    for (int k = ng; k <= ng + n3; ++k)
      for (int j = ng; j < ng + n2; ++j) {
        double sum = 0.0;
        for (int dj = 0; dj < 2; ++dj) {
          int bj, jj, bk, kk;
          fine_pos(2 * (j - ng) + dj, n2, ng, bj, jj);
          fine_pos(2 * (k - ng), n3, ng, bk, kk);
          sum += wk[1 + fa + 2 * bj + 4 * bk].edge[1 * nf + g.f(fi, jj, kk)];
        }
        wk[0].edge[1 * nf + g.f(ci, j, k)] = 0.5 * sum;
      }
    // E3: along x3 over coarse cell k, at the lower x2 face j (j up to ng + n2)
    for (int k = ng; k < ng + n3; ++k)
      for (int j = ng; j <= ng + n2; ++j) {
        double sum = 0.0;
        for (int dk = 0; dk < 2; ++dk) {
          int bj, jj, bk, kk;
          fine_pos(2 * (j - ng), n2, ng, bj, jj);
          fine_pos(2 * (k - ng) + dk, n3, ng, bk, kk);
          sum += wk[1 + fa + 2 * bj + 4 * bk].edge[2 * nf + g.f(fi, jj, kk)];
        }
        wk[0].edge[2 * nf + g.f(ci, j, k)] = 0.5 * sum;
      }
  }
}

inline int two_level_step(const Cfg& cfg, double* cons, double* bf, double dt) {
  if (!two_level_ok(cfg)) return -1;
  TwoLevel L(cfg);
  const Geo& g = L.g;
  Scheme sc;
  if (!scheme_for(cfg.integrator, sc)) return -1;
  const size_t n = 9 * L.bs;
  // state: block b's cells then its faces
  std::vector<double> u(n);
  for (int b = 0; b < 9; ++b) {
    std::copy(cons + b * L.ncv, cons + (b + 1) * L.ncv, u.begin() + b * L.bs);
    std::copy(bf + b * 3 * L.nf, bf + (b + 1) * 3 * L.nf, u.begin() + b * L.bs + L.ncv);
  }
  std::vector<unsigned char> mask(n, 0);
  const int ng = g.ng;
  for (int b = 0; b < 9; ++b) {
    const size_t o = b * L.bs;
    for (int v = 0; v < g.nv; ++v)
      for (int k = ng; k <= g.e(2); ++k)
        for (int j = ng; j <= g.e(1); ++j)
          for (int i = ng; i <= g.e(0); ++i) mask[o + v * g.ncell() + g.c(i, j, k)] = 1;
    for (int d = 0; d < 3; ++d)
      for (int k = ng; k <= g.e(2); ++k)
        for (int j = ng; j <= g.e(1); ++j) {
          const int ilo = (b == 0 && d == 0) ? ng + 1 : ng;  // coarse x1 boundary faces: fine-owned
          const int ihi = (b != 0 && d == 0 && ((b - 1) & 1) == 1) ? g.e(0) + 1 : g.e(0);
          for (int i = ilo; i <= ihi; ++i) mask[o + L.ncv + d * L.nf + g.f(i, j, k)] = 1;
        }
  }
  std::vector<Work<double>> wk(9);
  // state in the two-array layout for the ghost fill
  std::vector<double> sc_(9 * L.ncv), sb_(9 * 3 * L.nf);
  auto split = [&](const double* st) {
    for (int b = 0; b < 9; ++b) {
      std::copy(st + b * L.bs, st + b * L.bs + L.ncv, sc_.begin() + b * L.ncv);
      std::copy(st + b * L.bs + L.ncv, st + (b + 1) * L.bs, sb_.begin() + b * 3 * L.nf);
    }
  };
  auto join = [&](double* st) {
    for (int b = 0; b < 9; ++b) {
      std::copy(sc_.begin() + b * L.ncv, sc_.begin() + (b + 1) * L.ncv, st + b * L.bs);
      std::copy(sb_.begin() + b * 3 * L.nf, sb_.begin() + (b + 1) * 3 * L.nf, st + b * L.bs + L.ncv);
    }
  };
  auto rhs = [&](int s, double* state, double* R) -> int {
    split(state);
    two_level_ghosts(L, sc_.data(), sb_.data());
    join(state);
    std::fill(R, R + n, 0.0);
    const int recon = (cfg.integrator == INT_VL2 && s == 0) ? RECON_DC : cfg.recon;
    int bad = 0;
    for (int b = 0; b < 9; ++b)
      bad += compute_fluxes(L.cfg(b), g, recon, state + b * L.bs, state + b * L.bs + L.ncv, wk[b]);
    two_level_correct(L, wk);
    for (int b = 0; b < 9; ++b) {
      double* du = R + b * L.bs;
      double* db = du + L.ncv;
      apply_operator(L.cfg(b), g, wk[b], du, db);
      if (b != 0 && ((b - 1) & 1) == 1) {  // a = 1: the interface faces x1 = X
        const double dx[3] = {L.cf.dx1, L.cf.dx2, L.cf.dx3};
        for (int k = ng; k <= g.e(2); ++k)
          for (int j = ng; j <= g.e(1); ++j) db[g.f(g.e(0) + 1, j, k)] = face_curl(g, dx, wk[b], 0, g.e(0) + 1, j, k);
      }
    }
    return bad;
  };
  const int bad = drive_2s(sc, n, u.data(), mask.data(), dt, rhs);
  if (bad < 0) return bad;
  split(u.data());
  two_level_ghosts(L, sc_.data(), sb_.data());
  std::copy(sc_.begin(), sc_.end(), cons);
  std::copy(sb_.begin(), sb_.end(), bf);
  return bad;
}

inline int two_level_newdt(const Cfg& cfg, const double* cons, const double* bf, double* dt_out) {
  if (!two_level_ok(cfg)) return -1;
  TwoLevel L(cfg);
  double best = INFINITY;
  int bad = 0;
  for (int b = 0; b < 9; ++b) {
    double dt;
    bad += newdt(L.cfg(b), cons + b * L.ncv, bf + b * 3 * L.nf, &dt);
    best = std::min(best, dt);
  }
  *dt_out = best;
  return bad;
}

}  // namespace orc

// ---------------------------------------------------------------------------
// C entry points for the Python test harness (ctypes).
// ---------------------------------------------------------------------------
extern "C" {

int orc_fill_ghosts(const orc::Cfg* c, double* cons, double* bface) {
  orc::Geo g(*c);
  orc::fill_ghosts(g, cons, bface);
  return 0;
}

int orc_cons2prim(const orc::Cfg* c, const double* cons, const double* bface, double* prim, double* bcc) {
  orc::Geo g(*c);
  return orc::cons_to_prim(g, c->gamma, cons, bface, prim, bcc, c->dfloor, c->pfloor);
}

int orc_prim2cons(const orc::Cfg* c, const double* prim, const double* bface, double* cons) {
  orc::Geo g(*c);
  orc::prim_to_cons(g, c->gamma, prim, bface, cons);
  return 0;
}

int orc_step(const orc::Cfg* c, double* cons, double* bface, double dt) {
  return orc::step<double>(*c, cons, bface, dt);
}

// Directional derivative of one step: (cons, bface) advance as in orc_step and
// (dcons, dbface) are replaced by J * (dcons, dbface).
int orc_step_jvp(const orc::Cfg* c, double* cons, double* bface, double* dcons, double* dbface, double dt) {
  orc::Geo g(*c);
  const size_t nc = g.ncell(), nf = g.nface();
  const size_t ncv = g.nv * nc;
  std::vector<orc::Dual> uc(ncv), ub(3 * nf);
  for (size_t q = 0; q < ncv; ++q) uc[q] = orc::Dual(cons[q], dcons[q]);
  for (size_t q = 0; q < 3 * nf; ++q) ub[q] = orc::Dual(bface[q], dbface[q]);
  int r = orc::step<orc::Dual>(*c, uc.data(), ub.data(), dt);
  for (size_t q = 0; q < ncv; ++q) { cons[q] = uc[q].v; dcons[q] = uc[q].d; }
  for (size_t q = 0; q < 3 * nf; ++q) { bface[q] = ub[q].v; dbface[q] = ub[q].d; }
  return r;
}

// Floating-point operations of one step of the algorithm on this state:
// out = (adds+subtracts, multiplies, divides, square roots).  The state is not
// modified.
int orc_count_ops(const orc::Cfg* c, const double* cons, const double* bface, double dt, unsigned long long* out) {
  orc::Geo g(*c);
  const size_t nc = g.ncell(), nf = g.nface();
  std::vector<orc::Cnt> uc(cons, cons + g.nv * nc), ub(bface, bface + 3 * nf);
  orc::g_ops = {0, 0, 0, 0};
  int r = orc::step<orc::Cnt>(*c, uc.data(), ub.data(), dt);
  out[0] = orc::g_ops.add;
  out[1] = orc::g_ops.mul;
  out[2] = orc::g_ops.div;
  out[3] = orc::g_ops.sqrt;
  return r;
}

// Floor activations since the previous call (then reset to zero).
long long orc_take_floor_count(void) {
  const long long n = orc::g_floored;
  orc::g_floored = 0;
  return n;
}

// Two-level composite of nine blocks (block 0 coarse, 1..8 fine; see
// TwoLevel): one step, the ghost fill, and the CFL time step.  -1 when the
// geometry does not satisfy two_level_ok.
int orc_two_level_step(const orc::Cfg* c, double* cons, double* bface, double dt) {
  return orc::two_level_step(*c, cons, bface, dt);
}

int orc_two_level_fill(const orc::Cfg* c, double* cons, double* bface) {
  if (!orc::two_level_ok(*c)) return -1;
  orc::TwoLevel L(*c);
  orc::two_level_ghosts(L, cons, bface);
  return 0;
}

int orc_two_level_newdt(const orc::Cfg* c, const double* cons, const double* bface, double* dt_out) {
  return orc::two_level_newdt(*c, cons, bface, dt_out);
}

int orc_newdt(const orc::Cfg* c, const double* cons, const double* bface, double* dt_out) {
  return orc::newdt(*c, cons, bface, dt_out);
}

// One interface: w = (rho, vn, vt1, vt2, p, Bt1, Bt2), bn normal field.
int orc_riemann(int rs, double gamma, const double* wl, const double* wr, double bn, double* flux, double* smax) {
  double s;
  orc::riemann<double>(rs, wl, wr, bn, gamma, flux, s);
  if (smax) *smax = s;
  return 0;
}

// HLLD fan of one face (test hook): out[0..5] = S_L, S*_L, S_M, S*_R, S_R,
// p_T*; out[6..33] = U*_L, U**_L, U**_R, U*_R (7 each, face frame); flux as
// orc_riemann.  Returns 1 when an outer state is upwind (out not written).
int orc_hlld_fan(double gamma, const double* wl, const double* wr, double bn, double* flux, double* out) {
  double s;
  orc::HlldFan<double> fan;
  if (!orc::hlld<double>(wl, wr, bn, gamma, flux, s, &fan)) return 1;
  const double head[6] = {fan.sl, fan.ssl, fan.sm, fan.ssr, fan.sr, fan.pts};
  for (int n = 0; n < 6; ++n) out[n] = head[n];
  for (int n = 0; n < 7; ++n) {
    out[6 + n] = fan.us_l[n];
    out[13 + n] = fan.uss_l[n];
    out[20 + n] = fan.uss_r[n];
    out[27 + n] = fan.us_r[n];
  }
  return 0;
}

// Roe matrix of a pair (test hook): A (7 x 7, row-major, face frame).
int orc_roe_matrix(double gamma, const double* wl, const double* wr, double bn, double* A) {
  double M[7][7];
  orc::roe_matrix<double>(wl, wr, bn, gamma, M);
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) A[7 * r + c] = M[r][c];
  return 0;
}

// Physical flux and conserved state of one state in the face frame.
int orc_phys_flux(double gamma, const double* w, double bn, double* u, double* f) {
  orc::phys_flux<double>(w, bn, gamma, u, f);
  return 0;
}

double orc_fast_speed(double rho, double p, double bn, double bt1, double bt2, double gamma) {
  return orc::fast_speed<double>(rho, p, bn, bt1, bt2, gamma);
}

// Right eigenvectors (columns, row-major 7 x 7) and their inverse for one
// face-frame primitive state w (7 values) with normal field bn.
int orc_prim_eigen(double gamma, const double* w, double bn, double* R, double* L) {
  double r[7][7], l[7][7];
  orc::prim_right_eigenvectors<double>(w, bn, gamma, r);
  orc::invert7<double>(r, l);
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) {
      R[i * 7 + j] = r[i][j];
      L[i * 7 + j] = l[i][j];
    }
  return 0;
}

// Restriction of the fine block (fcons, fbface) into the octant (ox, oy, oz)
// of the coarse block, and prolongation of that octant into the fine block.
int orc_restrict(const orc::Cfg* c, const double* fcons, const double* fbface, double* ccons, double* cbface, int ox,
                 int oy, int oz) {
  orc::Geo g(*c);
  const int o[3] = {ox, oy, oz};
  orc::restrict_box(g, fcons, fbface, ccons, cbface, orc::octant_box(g, o));
  return 0;
}

// The same on a box: fine cells [flo, flo + 2 ext), coarse cells [clo, clo + ext).
int orc_restrict_box(const orc::Cfg* c, const double* fcons, const double* fbface, double* ccons, double* cbface,
                     const int* flo, const int* clo, const int* ext) {
  orc::Geo g(*c);
  orc::LevelBox B;
  for (int d = 0; d < 3; ++d) {
    B.f[d] = flo[d];
    B.c[d] = clo[d];
    B.h[d] = ext[d];
  }
  orc::restrict_box(g, fcons, fbface, ccons, cbface, B);
  return 0;
}

int orc_prolong(const orc::Cfg* c, const double* ccons, const double* cbface, double* fcons, double* fbface, int ox,
                int oy, int oz, int primitive) {
  orc::Geo g(*c);
  const int o[3] = {ox, oy, oz};
  orc::prolong_box(g, ccons, cbface, fcons, fbface, orc::octant_box(g, o), c->gamma, c->pfloor, primitive != 0);
  return 0;
}

int orc_prolong_box(const orc::Cfg* c, const double* ccons, const double* cbface, double* fcons, double* fbface,
                    const int* flo, const int* clo, const int* ext, int primitive, int keep) {
  orc::Geo g(*c);
  orc::LevelBox B;
  for (int d = 0; d < 3; ++d) {
    B.f[d] = flo[d];
    B.c[d] = clo[d];
    B.h[d] = ext[d];
  }
  orc::prolong_box(g, ccons, cbface, fcons, fbface, B, c->gamma, c->pfloor, primitive != 0, keep);
  return 0;
}

// Characteristic PPM edges of one cell from its five-cell stencil w (5 x 7,
// row-major, cells c-2 .. c+2).
int orc_char_ppm(double gamma, const double* w, double bn, double* left, double* right) {
  double st[5][7];
  for (int o = 0; o < 5; ++o)
    for (int n = 0; n < 7; ++n) st[o][n] = w[o * 7 + n];
  orc::char_ppm_edges<double>(st, bn, gamma, left, right);
  return 0;
}

// Characteristic PLM edges of one cell (w0) from its neighbours (wm, wp).
int orc_char_plm(double gamma, const double* wm, const double* w0, const double* wp, double bn, double* left,
                 double* right) {
  orc::char_plm_edges<double>(wm, w0, wp, bn, gamma, left, right);
  return 0;
}

// Reconstruct along a 1D line of n cells: for every face c-1/2 whose stencil
// fits (c in [3, n-3]), ql[c] and qr[c] receive the two states; other entries
// are left untouched.
int orc_recon_line(int recon, int n, const double* q, double* ql, double* qr) {
  for (int c = 3; c <= n - 3; ++c) orc::recon_face<double>(recon, q + c, ql[c], qr[c]);
  return 0;
}

// The 2S driver applied to the scalar test equation u' = lambda u (complex
// lambda), n steps of size dt from u = 1.  Exercises the same driver and
// coefficient tables as orc_step.
int orc_drive_scalar(int integrator, double lre, double lim, double dt, int nsteps, double* out_re, double* out_im) {
  orc::Scheme sc;
  if (!orc::scheme_for(integrator, sc)) return -1;
  double u[2] = {1.0, 0.0};
  unsigned char mask[2] = {1, 1};
  for (int it = 0; it < nsteps; ++it) {
    auto rhs = [&](int, double* st, double* L) -> int {
      L[0] = lre * st[0] - lim * st[1];
      L[1] = lre * st[1] + lim * st[0];
      return 0;
    };
    orc::drive_2s(sc, 2, u, mask, dt, rhs);
  }
  *out_re = u[0];
  *out_im = u[1];
  return 0;
}

}  // extern "C"
