// kernels_fused.hip -- one stage of the MHD update in a single kernel.
//
// Each workgroup (34 x 15 threads, 8 wave64s) owns a tile of 32 x 13 active
// columns in (x1, x2) plus a one-cell ring, and marches along x3 over a
// segment of KZ planes.  Per plane everything stays on chip:
//   * every thread owns one column of the 34 x 15 region; it converts its
//     column's conserved state to primitives (Sec. 3.1) one plane ahead of use
//     and keeps a short window of planes in registers for the reconstruction
//     along x3;
//   * the primitives of the current plane, plus LA extra rings, go to LDS for
//     the reconstructions along x1 and x2 (DC / PLM / PPM, Sec. 3.2.1);
//   * each thread solves the Riemann problems (HLLD / HLLE, Sec. 3.2.2) on the
//     lower x1-face and x2-face of its column in this plane and on the lower
//     x3-face of its column's cell;
//   * face fluxes, face EMFs, upwind weights and cell-centred EMFs are
//     exchanged through LDS to form the upwind-CT corner EMFs (Sec. 3.1);
//   * the flux divergence and the CT curl accumulate in registers and the
//     plane below is written out once its upper x3 fluxes / EMFs exist
//     (2S stage update, Eq. (rk-2s)).
// Two barriers per plane: after the primitives are in LDS, and after the face
// results are.  The face-field update that reads a plane's corner EMFs runs
// after the next plane's first barrier, and the exchange slots read by the
// corner EMFs are written after that barrier too, so no third barrier is
// needed to keep one plane's reads apart from the next plane's writes.
// HBM traffic per stage is the input state (with the halo overlap of
// neighbouring tiles), U^n where the stage needs it, and the output state.
#include "common.hpp"
#include "kernels.hpp"
#include "mhd_math.hpp"

namespace athmhd {

namespace {

// Thread tile: BX x BY threads, one per column of a (BX-2) x (BY-2) tile of
// active columns plus a one-column ring.
template <int BX_, int BY_>
struct Tile {
  static constexpr int BX = BX_, BY = BY_, NT = BX_ * BY_, TX = BX_ - 2, TY = BY_ - 2;
};
// uniform blocks: 32 x 13 active columns in one 8-wave workgroup per CU; of
// the tiles that fit the register and LDS budget this one keeps the largest
// share of lanes on active columns on large blocks (80 % at 256^3)
using TileU = Tile<34, 15>;

// Arguments shared by every tile of a stage.
struct StageArgs {
  Gas gas;
  double ct_eps;
  StageCoef cf;          // g0, g1 and (when dt_dev is NULL) beta * dt
  const double* dt_dev;  // optional device copy of dt: bdt = beta * (*dt_dev)
  double beta;
  Floors fl;             // optional primitive floors
  int* bad;              // [0]: threads that met a non-physical cell; floor activations (add_floor_count)
};

// Arrays of one block: stage input (periodic images are read by index wrap,
// ghost entries are not used), U^n (the u^(1) register), stage output (active
// cells and their lower faces).
struct BlockPtrs {
  const double* xc;
  const double* xb;
  const double* unc;
  const double* unb;
  double* oc;
  double* ob;
  double* fm = nullptr;  // optional: mass fluxes through the lower faces of the active cells (3 face arrays)
};

struct UniformArgs {
  Geo g;
  StageArgs sa;
  const double* xc;
  const double* xb;
  const double* unc;
  const double* unb;
  double* oc;
  double* ob;
  double* fm;  // NULL, or the face mass-flux output of every block (3 face arrays per block)
  int ntx, nty, nseg, kz;
  int64_t total;    // workgroups doing work
  int64_t per_xcd;  // ceil(total / 8)
};

struct BatchArgs {
  const BatchDesc* desc;
  const WorkItem* items;
  int nitems;
  unsigned* queue;  // work counter, zero at launch
  StageArgs sa;
  const double* xc;
  const double* xb;
  const double* unc;
  const double* unb;
  double* oc;
  double* ob;
  double* fm;  // NULL, or the face mass-flux output, laid out like bface
};

// z-frame primitive vector of a cell: (rho, v3, v1, v2, P, B1cc, B2cc) plus
// B3cc kept alongside
struct ZCell {
  double q[7];
  double b3;
};

// Raw data of one cell needed to form its primitives.
struct Raw {
  double u[5];
  double b1lo, b1hi, b2lo, b2hi, b3lo, b3hi;
};

// Column of a block: stored indices of a column and of its upper neighbours
// along x1 and x2.  A block that is its own periodic neighbour is read at the
// periodic images directly, so its ghost entries are never needed; the blocks
// of a coupled mesh read their ghost entries, which the mesh exchange fills
// before every stage.
struct Col {
  int i0, i1, j0, j1;
};

// Stored index read for position idx (cell, or face when hi = N) along a
// direction with n active cells: its periodic image when the block is its own
// neighbour, else the stored entry itself (ghosts filled by the mesh
// exchange), clamped into the array for the columns of a ragged tile past the
// block edge, whose results are never written out.
template <bool MESH>
__device__ __forceinline__ int read_index(const Geo& g, int idx, int n, int hi) {
  if (!MESH) return wrap_index(idx, n, g.ng);
  return idx < 0 ? 0 : (idx > hi ? hi : idx);
}

template <bool MESH>
__device__ __forceinline__ Col make_col(const Geo& g, int i, int j) {
  Col c;
  c.i0 = read_index<MESH>(g, i, g.n1, g.N1 - 1);
  c.i1 = read_index<MESH>(g, i + 1, g.n1, g.N1);
  c.j0 = read_index<MESH>(g, j, g.n2, g.N2 - 1);
  c.j1 = read_index<MESH>(g, j + 1, g.n2, g.N2);
  return c;
}

// Conserved state and the six bounding face fields of the cell of column c in
// (unwrapped) plane k.
template <bool MESH>
__device__ __forceinline__ void load_raw(const Geo& g, const double* __restrict__ xc, const double* __restrict__ xb,
                                         const Col& c, int k, Raw& r) {
  const int k0 = read_index<MESH>(g, k, g.n3, g.N3 - 1), k1 = read_index<MESH>(g, k + 1, g.n3, g.N3);
  const int q = g.c(c.i0, c.j0, k0);
#pragma unroll
  for (int v = 0; v < 5; ++v) r.u[v] = xc[v * g.cvar + q];
  const int f = g.f(c.i0, c.j0, k0);
  r.b1lo = xb[f];
  r.b1hi = xb[g.f(c.i1, c.j0, k0)];
  r.b2lo = xb[g.fvar + f];
  r.b2hi = xb[g.fvar + g.f(c.i0, c.j1, k0)];
  r.b3lo = xb[2 * g.fvar + f];
  r.b3hi = xb[2 * g.fvar + g.f(c.i0, c.j0, k1)];
}

// cons -> prim: w = (rho, v1, v2, v3, P, B1cc, B2cc, B3cc); returns the flags
// of cell_prim (bit 0 non-physical, bit 1 floored).  The same cell is
// converted at several places (the register window along x3, the primitive
// plane, the extra rings, and again by the neighbouring tile or x3 segment);
// cell_prim computes without contraction, so all of them get the same bits.
// Fluxes and EMFs on tile and segment boundaries are computed twice and must
// agree exactly, or the CT update no longer preserves div B (reconstruction
// limiters can turn an ulp of difference into an O(1) one).
template <bool FL>
__device__ __forceinline__ int to_prim(const Raw& r, double gm1, const Floors& fl, double* w) {
  double b[3];
  {
#pragma clang fp contract(off)
    b[0] = 0.5 * (r.b1lo + r.b1hi);
    b[1] = 0.5 * (r.b2lo + r.b2hi);
    b[2] = 0.5 * (r.b3lo + r.b3hi);
  }
  const int flags = cell_prim(r.u, b, gm1, FL ? fl : Floors{0.0, 0.0}, w);
  w[5] = b[0];
  w[6] = b[1];
  w[7] = b[2];
  return flags;
}

__device__ __forceinline__ void to_zcell(const double* w, ZCell& z) {
  z.q[0] = w[0]; z.q[1] = w[3]; z.q[2] = w[1]; z.q[3] = w[2]; z.q[4] = w[4]; z.q[5] = w[5]; z.q[6] = w[6];
  z.b3 = w[7];
}

__device__ __forceinline__ FaceState make_state(const double* q) {
  FaceState s;
  s.rho = q[0]; s.vn = q[1]; s.vt1 = q[2]; s.vt2 = q[3]; s.p = q[4]; s.bt1 = q[5]; s.bt2 = q[6];
  return s;
}

template <int RS, bool FL>
__device__ __forceinline__ void riemann(const double* ql, const double* qr, double bn, const Gas& gas, double ct_eps,
                                        const Floors& fl, int& nfl, FaceFlux& F, double& w) {
  FaceState L = make_state(ql), R = make_state(qr);
  if (FL) nfl += floor_state(L, fl) + floor_state(R, fl);
  double smax;
  riemann_flux<RS>(L, R, bn, gas, F, smax);
  w = ct_weight(F.rho, 0.5 * (L.rho + R.rho), smax, ct_eps);
}

// LDS layout: the primitive plane (with LA extra rings), the per-thread
// exchange slots and the corner EMFs are separate, so a thread can publish
// each Riemann result as soon as it has it.
template <int LA, class T>
struct Smem {
  static constexpr int PW = T::BX + 2 * LA;  // width of the primitive plane incl. extra rings
  static constexpr int PH = T::BY + 2 * LA;
  static constexpr int PL = PW * PH;
};

enum {
  X_FX = 0, X_FY = 5, X_E3X = 10, X_WX, X_E3Y, X_WY, X_E3C, X_E1Z, X_E2Z, X_WZ, X_E1C, X_E2C, X_E1CP, X_E2CP,
  // the previous plane's x1-face E2 and weight, x2-face E1 and (DC, PLM) weight:
  // read only by the own thread, kept here rather than in registers
  X_E2XP, X_WXP, X_E1YP, X_WYP, X_N
};
// exchange slots of a stage: PPM's wider primitive plane leaves room for all
// but the last (its x2-face weight stays in a register)
template <int RECON>
constexpr int exchange_slots() { return RECON >= 2 ? X_N - 1 : X_N; }

// Face-field update of plane q from its corner EMFs in sc (E1, E2, E3 of the
// own column's edges; the neighbours' at tid + 1 and tid + BX): completes B1
// and B2 on the lower faces of cell q-1, writes B3 on the face q-1/2, and
// leaves the partial B1, B2 of plane q in bacc[5], bacc[6].  pwb holds the
// pointwise terms (g1 U^n + g0 X) of B1, B2 at q-1 and B3 at q.
__device__ __forceinline__ void face_update(const Geo& g, const double* __restrict__ sc, int tid, int BX, int NT,
                                            int gi, int gj, int q, int k0, int kend, double i1, double i2,
                                            double i3, double bdt, const double* pwb, double* bacc,
                                            double* __restrict__ ob) {
  const int tE = tid + 1, tN = tid + BX;
  const double e1 = sc[0 * NT + tid], e2 = sc[1 * NT + tid], e3 = sc[2 * NT + tid];
  // B1(i-1/2, j): -(E3(j+1/2) - E3(j-1/2))/dx2 + (E2(k+1/2) - E2(k-1/2))/dx3
  const double a5 = -(sc[2 * NT + tN] - e3) * i2 - e2 * i3;
  bacc[5] += e2 * i3;
  // B2(i, j-1/2): -(E1(k+1/2) - E1(k-1/2))/dx3 + (E3(i+1/2) - E3(i-1/2))/dx1
  const double a6 = (sc[2 * NT + tE] - e3) * i1 + e1 * i3;
  bacc[6] -= e1 * i3;
  // B3(i, j, q-1/2): -(E2(i+1/2) - E2(i-1/2))/dx1 + (E1(j+1/2) - E1(j-1/2))/dx2
  const double db3 = -(sc[1 * NT + tE] - e2) * i1 + (sc[0 * NT + tN] - e1) * i2;
  if (q < kend) ob[2 * g.fvar + g.f(gi, gj, q)] = pwb[2] + bdt * db3;
  if (q - 1 >= k0) {
    const int f = g.f(gi, gj, q - 1);
    ob[f] = pwb[0] + bdt * bacc[5];
    ob[g.fvar + f] = pwb[1] + bdt * bacc[6];
  }
  bacc[5] = a5;
  bacc[6] = a6;
}

// The same, with the pointwise terms read here instead of carried in pwb
// through the plane's registers.
__device__ __forceinline__ void face_update_read(const Geo& g, const double* __restrict__ sc, int tid, int BX,
                                                 int NT, int gi, int gj, int q, int k0, int kend, double i1,
                                                 double i2, double i3, double bdt, const StageCoef& cf,
                                                 const double* unb, const double* xb, double* bacc, double* ob) {
  double pwb[3] = {0.0, 0.0, 0.0};
  if (q < kend) {
    const int f3 = 2 * g.fvar + g.f(gi, gj, q);
    pwb[2] = cf.g1 * unb[f3];
    if (cf.g0 != 0.0) pwb[2] += cf.g0 * xb[f3];
  }
  if (q - 1 >= k0) {
    const int f = g.f(gi, gj, q - 1);
    pwb[0] = cf.g1 * unb[f];
    pwb[1] = cf.g1 * unb[g.fvar + f];
    if (cf.g0 != 0.0) {
      pwb[0] += cf.g0 * xb[f];
      pwb[1] += cf.g0 * xb[g.fvar + f];
    }
  }
  face_update(g, sc, tid, BX, NT, gi, gj, q, k0, kend, i1, i2, i3, bdt, pwb, bacc, ob);
}

// One tile (tile_x, tile_y) of a block over the active planes [k0, kend).
// MF: also store the mass flux through the lower faces of the active cells,
// which passive scalars are carried by.
// SAME (donor cell only): the stage input is U^n itself (the first stage of
// every scheme), so the output's pointwise terms come from the raw cell read
// for the window one plane earlier, carried, instead of being read again.
template <int RECON, int RS, class T, bool FL, bool MESH = false, bool MF = false, bool SAME = false>
__device__ __forceinline__ void stage_tile(const Geo& g, const BlockPtrs& bp, const StageArgs& sa, int tile_x,
                                           int tile_y, int k0, int kend, double* __restrict__ sp,
                                           double* __restrict__ sx, double* __restrict__ sc) {
  constexpr int LA = RECON;  // cells of look-ahead / extra LDS rings: DC 0, PLM 1, PPM 2
  constexpr int NW = 2 * LA + 1;
  constexpr int BX = T::BX, BY = T::BY, NT = T::NT, TX = T::TX, TY = T::TY;
  using S = Smem<LA, T>;
  constexpr int PW = S::PW, PL = S::PL;
  const double* __restrict__ xc = bp.xc;
  const double* __restrict__ xb = bp.xb;
  const double* __restrict__ unc = bp.unc;
  const double* __restrict__ unb = bp.unb;
  double* __restrict__ oc = bp.oc;
  double* __restrict__ ob = bp.ob;
  const double bdt = sa.dt_dev ? sa.beta * *sa.dt_dev : sa.cf.bdt;

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int x0 = g.ng + tile_x * TX, y0 = g.ng + tile_y * TY;
  // own column (columns of a ragged tile past the block edge only feed values
  // that are never written out); reads use the periodic images
  const int gi = x0 - 1 + tx, gj = y0 - 1 + ty;
  const Col own = make_col<MESH>(g, gi, gj);
  const bool act = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && gi < g.ng + g.n1 && gj < g.ng + g.n2;

  // ---- extra LDS rings (LA per side): left and right columns (BY cells per
  // depth), bottom and top rows (BX cells per depth), one cell per thread
  constexpr int NRING = 2 * LA * (BX + BY);
  static_assert(NRING <= NT, "ring cells must fit the workgroup");
  const bool ring = tid < NRING;
  int rl = 0;
  Col rcol{0, 0, 0, 0};
  if (ring) {
    constexpr int LD = LA > 0 ? LA : 1;  // no ring cells when LA = 0
    int rlx, rly;
    if (tid < 2 * LA * BY) {
      const int side = tid / (LD * BY), e = tid % (LD * BY), d = e / BY, pos = e % BY;
      rly = LA + pos;
      rlx = side == 0 ? LA - 1 - d : LA + BX + d;
    } else {
      const int u = tid - 2 * LA * BY;
      const int side = u / (LD * BX), e = u % (LD * BX), d = e / BX, pos = e % BX;
      rlx = LA + pos;
      rly = side == 0 ? LA - 1 - d : LA + BY + d;
    }
    rl = rly * PW + rlx;
    rcol = make_col<MESH>(g, x0 - 1 - LA + rlx, y0 - 1 - LA + rly);
  }

  const double i1 = 1.0 / g.dx1, i2 = 1.0 / g.dx2, i3 = 1.0 / g.dx3;
  const double gm1 = sa.gas.gm1;
  int nbad = 0, nfl = 0;

  // ---- z window: planes p-LA .. p+LA of the own column
  ZCell win[NW];
  // normal fields (lower x1, x2, x3 faces of the own cell) of planes
  // p .. p+LA, carried from the look-ahead loads; with PPM's five-plane window
  // they are read again from the cache each plane instead (fewer registers
  // live through the plane: 4.6 % faster for PPM, 2.2 % slower for PLM)
  constexpr bool RELOAD_BN = LA >= 2;
  constexpr int NBQ = RELOAD_BN ? 1 : LA + 1;
  double bnq[NBQ][3];
  {
    double w[8];
    Raw raw;
#pragma unroll
    for (int o = 0; o < NW - 1; ++o) {
      load_raw<MESH>(g, xc, xb, own, k0 - 1 - LA + o, raw);
      const int f = to_prim<FL>(raw, gm1, sa.fl, w);
      nbad += f & 1;
      nfl += f >> 1;
      to_zcell(w, win[o + 1]);
      if (!RELOAD_BN && o >= LA) {
        bnq[o - LA][0] = raw.b1lo;
        bnq[o - LA][1] = raw.b2lo;
        bnq[o - LA][2] = raw.b3lo;
      }
    }
  }
  Raw pre;   // raw data of the next look-ahead plane
  load_raw<MESH>(g, xc, xb, own, k0 - 1 + LA, pre);
  Raw rpre;  // raw data of this thread's ring cell in the next plane
  if (ring) load_raw<MESH>(g, xc, xb, rcol, k0 - 1, rpre);

  double qz_carry[7];  // left state of the next x3-face (right edge of the cell below)
  constexpr bool WY_REG = exchange_slots<RECON>() < X_N;
  double wy_prev = 0.5;  // PPM: the previous plane's x2-face weight
  double acc_prev[7];  // partial update of the plane below: 5 conserved, B1, B2
  // pointwise terms of the face fields: carried from the plane that loads them
  // to the next plane's face update on the uniform DC / PLM tile, read in the
  // face update elsewhere, where registers are scarcer (PPM's window, the
  // batch tiles): measured 0.9 % faster carried on the uniform PLM stage,
  // 5.6 % (PPM) and 3.5 % (batch) faster read
  constexpr bool CARRY_PW = (LA < 2 && NT == TileU::NT) || SAME;
  static_assert(!SAME || LA == 0, "the raw cell of the output plane is carried with the donor-cell window only");
  // SAME: conserved state and lower B1, B2 of the previous plane's cell, and
  // of the current plane's (from its look-ahead load, until the output step)
  double ucar[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double unext[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // the look-ahead loads for the next plane: issued before the corner EMFs
  // (more time to arrive), or after them where the registers they occupy
  // through the corner EMFs would be spilled (PPM, the batch tiles): measured
  // 4.3 % slower late on the uniform PLM stage, 1.1 % (PPM) and 1.0 % (batch)
  // faster late
  constexpr bool LATE_PREFETCH = LA >= 2 || NT != TileU::NT;
  double pwb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < 7; ++v) { acc_prev[v] = 0.0; qz_carry[v] = 0.0; }

  for (int p = k0 - 1; p <= kend; ++p) {
    const bool zface = p >= k0;
    // ---- 1-2. shift the window and convert the look-ahead plane p+LA
#pragma unroll
    for (int o = 0; o < NW - 1; ++o) win[o] = win[o + 1];
    {
      double w[8];
      const int f = to_prim<FL>(pre, gm1, sa.fl, w);
      nbad += f & 1;
      nfl += f >> 1;
      to_zcell(w, win[NW - 1]);
      if (SAME) {
#pragma unroll
        for (int v = 0; v < 5; ++v) unext[v] = pre.u[v];
        unext[5] = pre.b1lo;
        unext[6] = pre.b2lo;
      }
      if (RELOAD_BN) {
        const int f = g.f(own.i0, own.j0, read_index<MESH>(g, p, g.n3, g.N3 - 1));
        bnq[0][0] = xb[f];
        bnq[0][1] = xb[g.fvar + f];
        bnq[0][2] = xb[2 * g.fvar + f];
      } else {
        bnq[NBQ - 1][0] = pre.b1lo;
        bnq[NBQ - 1][1] = pre.b2lo;
        bnq[NBQ - 1][2] = pre.b3lo;
      }
    }

    // ---- 3. own cell of plane p: primitives to LDS, cell EMFs
    double e1c, e2c, e3c;
    {
      const ZCell& cur = win[LA];
      const int l = (ty + LA) * PW + tx + LA;
      sp[0 * PL + l] = cur.q[0];
      sp[1 * PL + l] = cur.q[2];
      sp[2 * PL + l] = cur.q[3];
      sp[3 * PL + l] = cur.q[1];
      sp[4 * PL + l] = cur.q[4];
      sp[5 * PL + l] = cur.q[5];
      sp[6 * PL + l] = cur.q[6];
      sp[7 * PL + l] = cur.b3;
      // E = -v x B at the cell centre
      const double v1 = cur.q[2], v2 = cur.q[3], v3 = cur.q[1];
      const double b1c = cur.q[5], b2c = cur.q[6], b3c = cur.b3;
      e1c = -(v2 * b3c - v3 * b2c);
      e2c = -(v3 * b1c - v1 * b3c);
      e3c = -(v1 * b2c - v2 * b1c);
    }

    // ---- 4. ring cells to LDS
    if (ring) {
      double w[8];
      to_prim<FL>(rpre, gm1, sa.fl, w);
#pragma unroll
      for (int v = 0; v < 8; ++v) sp[v * PL + rl] = w[v];
    }

    // ---- 5. reconstruction along x3 and the Riemann problem on the lower
    // x3-face (p-1/2) of the own cell
    double fz_cons[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double wz = 0.5, e1z = 0.0, e2z = 0.0;
    {
      double zl[7], zr[7];
#pragma unroll
      for (int v = 0; v < 7; ++v) {
        double line[NW];
#pragma unroll
        for (int o = 0; o < NW; ++o) line[o] = win[o].q[v];
        double left, right;
        cell_edges<RECON>(line, left, right);
        zl[v] = qz_carry[v];
        zr[v] = left;
        qz_carry[v] = right;
      }
      if (zface) {
        const double bn3 = bnq[0][2];
        FaceFlux fz;
        riemann<RS, FL>(zl, zr, bn3, sa.gas, sa.ct_eps, sa.fl, nfl, fz, wz);
        // z-frame -> (rho, M1, M2, M3, E); x3-face E2 = -F(B1), E1 = +F(B2)
        fz_cons[0] = fz.rho; fz_cons[1] = fz.mt1; fz_cons[2] = fz.mt2; fz_cons[3] = fz.mn; fz_cons[4] = fz.e;
        e2z = -fz.bt1;
        e1z = fz.bt2;
        if (MF && act && p < kend) bp.fm[2 * g.fvar + g.f(gi, gj, p)] = fz.rho;
      }
    }
    __syncthreads();

    // exchange values read only after the next barrier (writing them here, not
    // before the barrier above, lets the previous plane's corner EMFs read the
    // same slots without a third barrier per plane)
    sx[X_E3C * NT + tid] = e3c;
    // the previous plane's cell EMFs move to their own slots first (the slots
    // of the current plane still hold them: nobody reads these between the
    // previous plane's corner EMFs and here)
    sx[X_E1CP * NT + tid] = sx[X_E1C * NT + tid];
    sx[X_E2CP * NT + tid] = sx[X_E2C * NT + tid];
    sx[X_E1C * NT + tid] = e1c;
    sx[X_E2C * NT + tid] = e2c;
    sx[X_E1Z * NT + tid] = e1z;
    sx[X_E2Z * NT + tid] = e2z;
    sx[X_WZ * NT + tid] = wz;
    // ---- 8, for plane p-1: its face-field updates from the corner EMFs that
    // the previous iteration left in sc
    if (act && p - 1 >= k0) {
      if constexpr (CARRY_PW)
        face_update(g, sc, tid, BX, NT, gi, gj, p - 1, k0, kend, i1, i2, i3, bdt, pwb, acc_prev, ob);
      else
        face_update_read(g, sc, tid, BX, NT, gi, gj, p - 1, k0, kend, i1, i2, i3, bdt, sa.cf, unb, xb, acc_prev, ob);
    }

    // ---- 6. Riemann problems on the lower x1-face and x2-face in plane p
    double e2x = 0.0, wx = 0.5, e1y = 0.0, wy = 0.5;
    {
      double e3x = 0.0;
      if (tx >= 1) {
        double ql[7], qr[7];
        const int row = (ty + LA) * PW + tx + LA;
        // x-frame order: rho, v1, v2, v3, P, B2, B3
        const int map[7] = {0, 1, 2, 3, 4, 6, 7};
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          const double* s = sp + map[v] * PL + row;
          double lineL[NW], lineR[NW];
#pragma unroll
          for (int o = 0; o < NW; ++o) {
            lineL[o] = s[o - LA - 1];
            lineR[o] = s[o - LA];
          }
          double a0, a1, b0, b1;
          cell_edges<RECON>(lineL, a0, a1);
          cell_edges<RECON>(lineR, b0, b1);
          ql[v] = a1;
          qr[v] = b0;
        }
        const double bn1 = bnq[0][0];
        FaceFlux fx;
        riemann<RS, FL>(ql, qr, bn1, sa.gas, sa.ct_eps, sa.fl, nfl, fx, wx);
        if (MF && act && p >= k0 && p < kend) bp.fm[g.f(gi, gj, p)] = fx.rho;
        sx[(X_FX + 0) * NT + tid] = fx.rho;
        sx[(X_FX + 1) * NT + tid] = fx.mn;   // M1
        sx[(X_FX + 2) * NT + tid] = fx.mt1;  // M2
        sx[(X_FX + 3) * NT + tid] = fx.mt2;  // M3
        sx[(X_FX + 4) * NT + tid] = fx.e;
        // x1-face E3 = -F(B2), E2 = +F(B3)
        e3x = -fx.bt1;
        e2x = fx.bt2;
      }
      sx[X_E3X * NT + tid] = e3x;
      sx[X_WX * NT + tid] = wx;
    }
    {
      double e3y = 0.0;
      if (ty >= 1) {
        double ql[7], qr[7];
        const int col = (ty + LA) * PW + tx + LA;
        // y-frame order: rho, v2, v3, v1, P, B3, B1
        const int map[7] = {0, 2, 3, 1, 4, 7, 5};
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          const double* s = sp + map[v] * PL + col;
          double lineL[NW], lineR[NW];
#pragma unroll
          for (int o = 0; o < NW; ++o) {
            lineL[o] = s[(o - LA - 1) * PW];
            lineR[o] = s[(o - LA) * PW];
          }
          double a0, a1, b0, b1;
          cell_edges<RECON>(lineL, a0, a1);
          cell_edges<RECON>(lineR, b0, b1);
          ql[v] = a1;
          qr[v] = b0;
        }
        const double bn2 = bnq[0][1];
        FaceFlux fy;
        riemann<RS, FL>(ql, qr, bn2, sa.gas, sa.ct_eps, sa.fl, nfl, fy, wy);
        if (MF && act && p >= k0 && p < kend) bp.fm[g.fvar + g.f(gi, gj, p)] = fy.rho;
        sx[(X_FY + 0) * NT + tid] = fy.rho;
        sx[(X_FY + 1) * NT + tid] = fy.mt2;  // M1
        sx[(X_FY + 2) * NT + tid] = fy.mn;   // M2
        sx[(X_FY + 3) * NT + tid] = fy.mt1;  // M3
        sx[(X_FY + 4) * NT + tid] = fy.e;
        // x2-face E1 = -F(B3), E3 = +F(B1)
        e1y = -fy.bt1;
        e3y = fy.bt2;
      }
      sx[X_E3Y * NT + tid] = e3y;
      sx[X_WY * NT + tid] = wy;
    }
    // prefetch the look-ahead plane and the ring cell of the next iteration
    // (on PPM stages only after the corner EMFs, see LATE_PREFETCH), and the
    // pointwise terms of this iteration's output (U^n, and the stage input
    // where g0 != 0)
    if (!LATE_PREFETCH && p + 1 <= kend) {
      load_raw<MESH>(g, xc, xb, own, p + 1 + LA, pre);
      if (ring) load_raw<MESH>(g, xc, xb, rcol, p + 1, rpre);
    }
    const bool out_cell = act && zface && p - 1 >= k0;
    const bool out_b3 = act && zface && p < kend;
    double pw[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // g1 U^n + g0 X of cell p-1 (5), B1, B2 at p-1, B3 at p (carried)
    {
      const int q = g.c(gi, gj, p - 1), f = g.f(gi, gj, p - 1), f3 = g.f(gi, gj, p);
      if (SAME) {
        // the same sums from the carried raw values of cell p-1 and the lower
        // B3 of plane p (its look-ahead load)
        if (out_cell) {
#pragma unroll
          for (int v = 0; v < 7; ++v) pw[v] = sa.cf.g1 * ucar[v];
          if (sa.cf.g0 != 0.0) {
#pragma unroll
            for (int v = 0; v < 7; ++v) pw[v] += sa.cf.g0 * ucar[v];
          }
        }
        if (out_b3) {
          pw[7] = sa.cf.g1 * bnq[0][2];
          if (sa.cf.g0 != 0.0) pw[7] += sa.cf.g0 * bnq[0][2];
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) ucar[v] = unext[v];
      } else {
        if (out_cell) {
#pragma unroll
          for (int v = 0; v < 5; ++v) pw[v] = sa.cf.g1 * unc[v * g.cvar + q];
          if (CARRY_PW) {
            pw[5] = sa.cf.g1 * unb[f];
            pw[6] = sa.cf.g1 * unb[g.fvar + f];
          }
          if (sa.cf.g0 != 0.0) {
#pragma unroll
            for (int v = 0; v < 5; ++v) pw[v] += sa.cf.g0 * xc[v * g.cvar + q];
            if (CARRY_PW) {
              pw[5] += sa.cf.g0 * xb[f];
              pw[6] += sa.cf.g0 * xb[g.fvar + f];
            }
          }
        }
        if (CARRY_PW && out_b3) {
          pw[7] = sa.cf.g1 * unb[2 * g.fvar + f3];
          if (sa.cf.g0 != 0.0) pw[7] += sa.cf.g0 * xb[2 * g.fvar + f3];
        }
      }
    }
    __syncthreads();

    // ---- 7. corner EMFs of the own edges and the conserved update
    const int tW = tid - 1, tS = tid - BX, tSW = tid - BX - 1, tE = tid + 1, tN = tid + BX;
    double c1 = 0.0, c2 = 0.0, c3 = 0.0;
    if (tx >= 1 && ty >= 1 && p >= k0 && p < kend) {
      // E3 at (i-1/2, j-1/2, p): a = x1, b = x2
      c3 = corner_emf(sx[X_E3X * NT + tid], sx[X_E3X * NT + tS], sx[X_E3Y * NT + tid], sx[X_E3Y * NT + tW],
                      sx[X_E3C * NT + tid], sx[X_E3C * NT + tW], sx[X_E3C * NT + tS], sx[X_E3C * NT + tSW], wx,
                      sx[X_WX * NT + tS], wy, sx[X_WY * NT + tW]);
    }
    if (ty >= 1 && zface) {
      // E1 at (i, j-1/2, p-1/2): a = x2, b = x3
      double wyp = wy_prev;
      if constexpr (!WY_REG) wyp = sx[X_WYP * NT + tid];
      c1 = corner_emf(e1y, sx[X_E1YP * NT + tid], sx[X_E1Z * NT + tid], sx[X_E1Z * NT + tS],
                      sx[X_E1C * NT + tid], sx[X_E1C * NT + tS], sx[X_E1CP * NT + tid], sx[X_E1CP * NT + tS], wy, wyp,
                      sx[X_WZ * NT + tid], sx[X_WZ * NT + tS]);
    }
    if (tx >= 1 && zface) {
      // E2 at (i-1/2, j, p-1/2): a = x3, b = x1
      c2 = corner_emf(sx[X_E2Z * NT + tid], sx[X_E2Z * NT + tW], e2x, sx[X_E2XP * NT + tid],
                      sx[X_E2C * NT + tid], sx[X_E2CP * NT + tid], sx[X_E2C * NT + tW], sx[X_E2CP * NT + tW],
                      sx[X_WZ * NT + tid], sx[X_WZ * NT + tW], wx, sx[X_WXP * NT + tid]);
    }
    sc[0 * NT + tid] = c1;
    sc[1 * NT + tid] = c2;
    sc[2 * NT + tid] = c3;

    double acc[7];
    if (act && zface) {
      // flux divergence of plane p (x1, x2) and the x3 flux through p-1/2
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double dfx = sx[(X_FX + v) * NT + tE] - sx[(X_FX + v) * NT + tid];
        const double dfy = sx[(X_FY + v) * NT + tN] - sx[(X_FY + v) * NT + tid];
        acc[v] = -(dfx * i1 + dfy * i2) + fz_cons[v] * i3;
        acc_prev[v] -= fz_cons[v] * i3;
      }
      if (out_cell) {
        const int q = g.c(gi, gj, p - 1);
#pragma unroll
        for (int v = 0; v < 5; ++v) oc[v * g.cvar + q] = pw[v] + bdt * acc_prev[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) acc_prev[v] = acc[v];
      // the face fields of this plane are updated after the next barrier
      if (CARRY_PW) {
        pwb[0] = pw[5];
        pwb[1] = pw[6];
        pwb[2] = pw[7];
      }
    }

    // ---- 9. carry this plane's face EMFs / weights / cell EMFs upward
#pragma unroll
    for (int o = 0; o < NBQ - 1; ++o) {
      bnq[o][0] = bnq[o + 1][0];
      bnq[o][1] = bnq[o + 1][1];
      bnq[o][2] = bnq[o + 1][2];
    }
    sx[X_E2XP * NT + tid] = e2x;
    sx[X_WXP * NT + tid] = wx;
    sx[X_E1YP * NT + tid] = e1y;
    if constexpr (WY_REG) wy_prev = wy;
    else sx[X_WYP * NT + tid] = wy;
    if (LATE_PREFETCH && p + 1 <= kend) {
      load_raw<MESH>(g, xc, xb, own, p + 1 + LA, pre);
      if (ring) load_raw<MESH>(g, xc, xb, rcol, p + 1, rpre);
    }
  }
  __syncthreads();
  if (act && kend >= k0) {
    if constexpr (CARRY_PW)
      face_update(g, sc, tid, BX, NT, gi, gj, kend, k0, kend, i1, i2, i3, bdt, pwb, acc_prev, ob);
    else
      face_update_read(g, sc, tid, BX, NT, gi, gj, kend, k0, kend, i1, i2, i3, bdt, sa.cf, unb, xb, acc_prev, ob);
  }
  if (nbad && act) atomicAdd(sa.bad, 1);
  if (nfl && act) add_floor_count(sa.bad, (unsigned long long)nfl);
}

// Uniform blocks: one workgroup per (tile, x3 segment, block), XCD-aware:
// consecutive logical tiles land on the same XCD so that halo overlap hits its
// L2.
template <int RECON, int RS, bool FL, bool MESH, bool MF, bool SAME = false>
__global__ void __launch_bounds__(TileU::NT) __attribute__((amdgpu_waves_per_eu(2)))
k_stage_fused(UniformArgs a) {
  using T = TileU;
  using S = Smem<RECON, T>;
  __shared__ double sp[8 * S::PL];      // primitives of the current plane
  __shared__ double sx[exchange_slots<RECON>() * T::NT];  // exchange slots
  __shared__ double sc[3 * T::NT];      // corner EMFs E1, E2, E3 of the current (half-)plane
  const int64_t bid = blockIdx.x;
  const int64_t logical = (bid % 8) * a.per_xcd + bid / 8;
  if (logical >= a.total) return;
  const Geo& g = a.g;
  int64_t r = logical;
  const int tile_x = (int)(r % a.ntx); r /= a.ntx;
  const int tile_y = (int)(r % a.nty); r /= a.nty;
  const int seg = (int)(r % a.nseg); r /= a.nseg;
  const int64_t blk = r;
  BlockPtrs bp{a.xc + blk * g.cblock, a.xb + blk * g.fblock, a.unc + blk * g.cblock,
               a.unb + blk * g.fblock, a.oc + blk * g.cblock, a.ob + blk * g.fblock,
               MF ? a.fm + blk * 3 * g.fvar : nullptr};
  const int k0 = g.ng + seg * a.kz;
  const int kend = min(k0 + a.kz, g.ng + g.n3);
  stage_tile<RECON, RS, T, FL, MESH, MF, SAME>(g, bp, a.sa, tile_x, tile_y, k0, kend, sp, sx, sc);
}

// Batched blocks of uneven sizes: a persistent grid whose workgroups pull
// (block, tile, x3 segment) items from a device queue until it is drained.
// MESH: the blocks tile one domain and read their exchanged ghost entries.
template <int RECON, int RS, class T, bool FL, bool MF, bool SAME = false, bool MESH = false>
__global__ void __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(2))) k_stage_batch(BatchArgs a) {
  using S = Smem<RECON, T>;
  __shared__ double sp[8 * S::PL];
  __shared__ double sx[exchange_slots<RECON>() * T::NT];
  __shared__ double sc[3 * T::NT];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= a.nitems) break;
    const WorkItem w = a.items[it];
    const BatchDesc& d = a.desc[w.block];
    BlockPtrs bp{a.xc + d.coff, a.xb + d.foff, a.unc + d.coff, a.unb + d.foff, a.oc + d.coff, a.ob + d.foff,
                 MF ? a.fm + d.foff : nullptr};
    stage_tile<RECON, RS, T, FL, MESH, MF, SAME>(d.g, bp, a.sa, w.tile_x, w.tile_y, w.k0, w.kend, sp, sx, sc);
    __syncthreads();
  }
}

// MESH: the blocks of a coupled mesh read their (exchanged) ghost entries; MF:
// the face mass fluxes are stored for passive scalars.  Compile-time switches,
// so that the plain periodic-block kernels keep their code.
template <int RECON, int RS, bool MESH, bool MF>
hipError_t launch_fl(const UniformArgs& fa, hipStream_t s) {
  const unsigned grid = (unsigned)(8 * fa.per_xcd);
  constexpr int NT = TileU::NT;
  if constexpr (RECON == 0) {
    // the first stage of a scheme reads U^n as its input: carry its raw cells
    if (fa.xc == fa.unc && fa.xb == fa.unb) {
      if (fa.sa.fl.on())
        hipLaunchKernelGGL((k_stage_fused<RECON, RS, true, MESH, MF, true>), dim3(grid), dim3(NT), 0, s, fa);
      else
        hipLaunchKernelGGL((k_stage_fused<RECON, RS, false, MESH, MF, true>), dim3(grid), dim3(NT), 0, s, fa);
      return hipGetLastError();
    }
  }
  if (fa.sa.fl.on()) hipLaunchKernelGGL((k_stage_fused<RECON, RS, true, MESH, MF>), dim3(grid), dim3(NT), 0, s, fa);
  else hipLaunchKernelGGL((k_stage_fused<RECON, RS, false, MESH, MF>), dim3(grid), dim3(NT), 0, s, fa);
  return hipGetLastError();
}

template <int RECON, bool MESH, bool MF>
hipError_t launch_rs_m(int rs, const UniformArgs& fa, hipStream_t s) {
  if (rs == 1) return launch_fl<RECON, 1, MESH, MF>(fa, s);
  if (rs == 2) return launch_fl<RECON, 2, MESH, MF>(fa, s);
  return launch_fl<RECON, 0, MESH, MF>(fa, s);
}

template <int RECON>
hipError_t launch_rs(int rs, const UniformArgs& fa, hipStream_t s) {
  if (fa.fm)
    return fa.g.mesh[0] ? launch_rs_m<RECON, true, true>(rs, fa, s) : launch_rs_m<RECON, false, true>(rs, fa, s);
  return fa.g.mesh[0] ? launch_rs_m<RECON, true, false>(rs, fa, s) : launch_rs_m<RECON, false, false>(rs, fa, s);
}

__global__ void k_zero_u32(unsigned* p) {
  if (threadIdx.x == 0) *p = 0u;
}

template <class T, int RECON, bool MF, bool SAME>
hipError_t launch_batch_s(int rs, const BatchArgs& ba, int grid, hipStream_t s) {
  const bool fl = ba.sa.fl.on();
  if (rs == 1 && fl)
    hipLaunchKernelGGL((k_stage_batch<RECON, 1, T, true, MF, SAME>), dim3(grid), dim3(T::NT), 0, s, ba);
  else if (rs == 1)
    hipLaunchKernelGGL((k_stage_batch<RECON, 1, T, false, MF, SAME>), dim3(grid), dim3(T::NT), 0, s, ba);
  else if (fl)
    hipLaunchKernelGGL((k_stage_batch<RECON, 0, T, true, MF, SAME>), dim3(grid), dim3(T::NT), 0, s, ba);
  else
    hipLaunchKernelGGL((k_stage_batch<RECON, 0, T, false, MF, SAME>), dim3(grid), dim3(T::NT), 0, s, ba);
  return hipGetLastError();
}

template <class T, int RECON, bool MF>
hipError_t launch_batch_m(int rs, const BatchArgs& ba, int grid, hipStream_t s) {
  // the first stage of a scheme reads U^n as its input: carry its raw cells
  if constexpr (RECON == 0) {
    if (ba.xc == ba.unc && ba.xb == ba.unb) return launch_batch_s<T, RECON, MF, true>(rs, ba, grid, s);
  }
  return launch_batch_s<T, RECON, MF, false>(rs, ba, grid, s);
}

template <class T, int RECON>
hipError_t launch_batch_t(int rs, const BatchArgs& ba, int grid, hipStream_t s) {
  return ba.fm ? launch_batch_m<T, RECON, true>(rs, ba, grid, s) : launch_batch_m<T, RECON, false>(rs, ba, grid, s);
}

// blocks that tile one domain (no floors, no mass fluxes)
template <class T, int RECON>
hipError_t launch_batch_mesh(int rs, const BatchArgs& ba, int grid, hipStream_t s) {
  if constexpr (RECON == 0) {
    if (ba.xc == ba.unc && ba.xb == ba.unb) {
      if (rs == 1)
        hipLaunchKernelGGL((k_stage_batch<RECON, 1, T, false, false, true, true>), dim3(grid), dim3(T::NT), 0, s, ba);
      else
        hipLaunchKernelGGL((k_stage_batch<RECON, 0, T, false, false, true, true>), dim3(grid), dim3(T::NT), 0, s, ba);
      return hipGetLastError();
    }
  }
  if (rs == 1)
    hipLaunchKernelGGL((k_stage_batch<RECON, 1, T, false, false, false, true>), dim3(grid), dim3(T::NT), 0, s, ba);
  else
    hipLaunchKernelGGL((k_stage_batch<RECON, 0, T, false, false, false, true>), dim3(grid), dim3(T::NT), 0, s, ba);
  return hipGetLastError();
}

template <class T>
hipError_t launch_batch_recon(int recon, int rs, const BatchArgs& ba, int grid, hipStream_t s, bool mesh) {
  if (mesh) {
    if (recon == 0) return launch_batch_mesh<T, 0>(rs, ba, grid, s);
    if (recon == 1) return launch_batch_mesh<T, 1>(rs, ba, grid, s);
    return launch_batch_mesh<T, 2>(rs, ba, grid, s);
  }
  if (recon == 0) return launch_batch_t<T, 0>(rs, ba, grid, s);
  if (recon == 1) return launch_batch_t<T, 1>(rs, ba, grid, s);
  return launch_batch_t<T, 2>(rs, ba, grid, s);
}

}  // namespace

int fused_default_kz(const Geo& g, int nb, int cus) {
  // the longest x3 segment (32 planes down to 4) that still gives the launch
  // at least 2.5 workgroups per CU: longer segments repeat less of the
  // window start-up, more segments fill the chip on small blocks.  64 planes
  // where that still leaves 16 workgroups per CU (512^3: 0.9 % faster with
  // PPM; 256^3, with 2.5 per CU, 12 % slower)
  const int64_t tiles = (int64_t)((g.n1 + TileU::TX - 1) / TileU::TX) * ((g.n2 + TileU::TY - 1) / TileU::TY) * nb;
  if (tiles * ((g.n3 + 63) / 64) >= 16 * (int64_t)cus) return 64 < g.n3 ? 64 : g.n3;
  int kz = 32;
  while (kz > 4 && 2 * tiles * ((g.n3 + kz - 1) / kz) < 5 * (int64_t)cus) kz /= 2;
  return kz < g.n3 ? kz : g.n3;
}

static StageArgs make_stage_args(double gamma, double ct_eps, StageCoef coef, const double* dt_dev, double beta,
                                 Floors fl, int* bad) {
  StageArgs sa;
  sa.fl = fl;
  sa.gas = Gas{gamma, gamma - 1.0, 1.0 / (gamma - 1.0)};
  sa.ct_eps = ct_eps;
  sa.cf = coef;
  sa.dt_dev = dt_dev;
  sa.beta = beta;
  sa.bad = bad;
  return sa;
}

hipError_t launch_stage_fused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                              const double* xb, const double* unc, const double* unb, double* outc, double* outb,
                              StageCoef coef, const double* dt_dev, double beta, int nb, int kz, Floors fl, int* bad,
                              double* fm, hipStream_t s) {
  UniformArgs fa;
  fa.g = g;
  fa.sa = make_stage_args(gamma, ct_eps, coef, dt_dev, beta, fl, bad);
  fa.xc = xc; fa.xb = xb; fa.unc = unc; fa.unb = unb; fa.oc = outc; fa.ob = outb;
  fa.fm = fm;
  fa.kz = kz;
  fa.ntx = (g.n1 + TileU::TX - 1) / TileU::TX;
  fa.nty = (g.n2 + TileU::TY - 1) / TileU::TY;
  fa.nseg = (g.n3 + fa.kz - 1) / fa.kz;
  fa.total = (int64_t)fa.ntx * fa.nty * fa.nseg * nb;
  fa.per_xcd = (fa.total + 7) / 8;
  if (recon == 0) return launch_rs<0>(rs, fa, s);
  if (recon == 1) return launch_rs<1>(rs, fa, s);
  return launch_rs<2>(rs, fa, s);
}

int batch_tile_count() { return 4; }

void batch_tile_shape(int shape, int* tx, int* ty) {
  static const int t[4][2] = {{16, 12}, {12, 16}, {14, 14}, {16, 8}};
  *tx = t[shape][0];
  *ty = t[shape][1];
}

int batch_tile_threads(int shape) {
  int tx, ty;
  batch_tile_shape(shape, &tx, &ty);
  return (tx + 2) * (ty + 2);
}

hipError_t launch_stage_batch(int shape, double gamma, int recon, int rs, double ct_eps, const BatchDesc* desc,
                              const WorkItem* items, int nitems, unsigned* queue, const double* xc,
                              const double* xb, const double* unc, const double* unb, double* outc, double* outb,
                              StageCoef coef, const double* dt_dev, double beta, int grid, Floors fl, int* bad,
                              double* fm, hipStream_t s, bool mesh) {
  if (mesh && (fl.on() || fm)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchArgs ba;
  ba.desc = desc;
  ba.items = items;
  ba.nitems = nitems;
  ba.queue = queue;
  ba.sa = make_stage_args(gamma, ct_eps, coef, dt_dev, beta, fl, bad);
  ba.xc = xc; ba.xb = xb; ba.unc = unc; ba.unb = unb; ba.oc = outc; ba.ob = outb;
  ba.fm = fm;
  switch (shape) {
    case 0: return launch_batch_recon<Tile<18, 14>>(recon, rs, ba, grid, s, mesh);
    case 1: return launch_batch_recon<Tile<14, 18>>(recon, rs, ba, grid, s, mesh);
    case 2: return launch_batch_recon<Tile<16, 16>>(recon, rs, ba, grid, s, mesh);
    default: return launch_batch_recon<Tile<18, 10>>(recon, rs, ba, grid, s, mesh);
  }
}

}  // namespace athmhd
