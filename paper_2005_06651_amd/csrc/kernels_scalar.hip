// kernels_scalar.hip -- passive scalars (Sec. 3.2.6, Eq. (passive_scalars)):
// the mass rho C_i of each scalar obeys the continuity equation with the
// specific density C_i carried along.  C_i is reconstructed like the other
// primitives (DC / PLM / PPM, Sec. 3.2.1) and moves with the face mass flux
// F_rho of the stage's Riemann solves, taken from the upwind side.  The fused
// stage kernel stores F_rho on the lower faces of the active cells; one
// HBM-bound kernel then finishes the stage for every scalar.
//
// A workgroup owns a tile of (x1, x2) columns of one scalar (64 x 8 on uniform
// blocks, 16 x 16 on batched blocks, whose edges are 16 to 32 cells) and
// marches along x3 over a segment of planes.
// Each plane of C = (rho C) / rho, with a halo of LA + 1 cells, is computed
// once from the stage input and kept in a ring of 2 LA + 4 planes in LDS, so
// that the lines of the reconstruction along x1, x2 and x3 all come from LDS;
// the ring is one plane longer than the stencil, which lets one barrier per
// plane separate every write of a slot from the reads of its previous plane.
// Each thread then forms the upwinded fluxes through the six faces of its
// cell and writes the 2S update (Eq. (rk-2s)).  A periodic block reads the
// periodic images of its cells; the blocks of a coupled mesh read their ghost
// cells (filled by the mesh exchange) and take the mass flux through an upper
// boundary face from the next block, which owns that face.
#include "common.hpp"
#include "kernels.hpp"
#include "mhd_math.hpp"

namespace athmhd {

namespace {

constexpr int kSX = 64, kSY = 8;  // uniform blocks and coupled meshes
constexpr int kBT = 16;           // batched blocks: kBT x kBT columns

struct ScalarCoef {
  StageCoef cf;
  const double* dt_dev;  // optional device copy of dt: bdt = beta * (*dt_dev)
  double beta;
  Floors fl;
};

struct ScalarArgs {
  Geo g;
  ScalarCoef sc;
  const double* xc;      // stage input: rho, E and rho C_i are read
  const double* unc;     // U^n
  double* oc;            // stage output
  const double* fm;      // face mass fluxes, 3 face arrays per block
  int ntx, nty, nseg, kz;
};

struct ScalarBatchArgs {
  const BatchDesc* desc;
  const WorkItem* items;
  int ns;
  ScalarCoef sc;
  const double* xc;
  const double* unc;
  double* oc;
  const double* fm;  // laid out like bface
};

// Stored index of position idx along a direction with n active cells, for a
// periodic block.  NEAR: every position a stencil of an active cell reaches
// is less than a block past the active range, so one correction step finds
// its periodic image; positions past that (halo columns of a ragged tile,
// never used by an active cell) are only kept inside the array.
template <bool NEAR>
__device__ __forceinline__ int wrap_sc(int idx, int n, int ng) {
  if (!NEAR) return wrap_index(idx, n, ng);
  idx = idx < ng ? idx + n : (idx >= ng + n ? idx - n : idx);
  return (idx < ng || idx >= ng + n) ? ng : idx;
}

// Stored cell index read for position idx (0 .. N-1 with ghosts): the
// periodic image on a self-periodic block, else the entry itself, clamped
// into the array for halo columns of a ragged tile past the block.
template <bool MESH, bool NEAR>
__device__ __forceinline__ int read_sc(int idx, int n, int ng) {
  if (!MESH) return wrap_sc<NEAR>(idx, n, ng);
  const int hi = n + 2 * ng - 1;
  return idx < 0 ? 0 : (idx > hi ? hi : idx);
}

template <int RECON, int SX, int SY>
struct ScalarRing {
  static constexpr int H = RECON + 1;  // halo: the edges of c-1, c, c+1 read c-H .. c+H
  static constexpr int R = 2 * H + 2;  // planes in the ring
  static constexpr int PW = SX + 2 * H, PH = SY + 2 * H, PL = PW * PH;
};

// Scalar v of one tile of block b over the planes [k0, kend).  xb, unb, ob:
// the block's stage input, U^n and output cell arrays; fm: its mass fluxes;
// fm_all: block 0's (coupled meshes read a neighbour's upper boundary faces).
template <int RECON, bool FL, bool NEAR, bool MESH, int SX, int SY>
__device__ __forceinline__ void scalar_tile(const Geo& g, const ScalarCoef& sc, const double* __restrict__ xb,
                                            const double* __restrict__ unb, double* __restrict__ ob,
                                            const double* __restrict__ fm, const double* __restrict__ fm_all,
                                            int b, int tile_x, int tile_y, int k0, int kend, int v,
                                            double* __restrict__ ring) {
  using RG = ScalarRing<RECON, SX, SY>;
  constexpr int H = RG::H, NW = 2 * H + 1, R = RG::R, PW = RG::PW, PL = RG::PL, NT = SX * SY;
  const int x0 = g.ng + tile_x * SX, y0 = g.ng + tile_y * SY;
  const int tid = threadIdx.x, tx = tid % SX, ty = tid / SX;
  const int i = x0 + tx, j = y0 + ty;
  const bool act = i < g.ng + g.n1 && j < g.ng + g.n2;
  const double* __restrict__ sv = xb + (5 + v) * g.cvar;
  const double bdt = sc.dt_dev ? sc.beta * *sc.dt_dev : sc.cf.bdt;
  const double i1 = 1.0 / g.dx1, i2 = 1.0 / g.dx2, i3 = 1.0 / g.dx3;

  // C of plane z (with its halo) into ring slot `slot`
  auto load_plane = [&](int z, int slot) {
    const int kk = read_sc<MESH, NEAR>(z, g.n3, g.ng);
    for (int e = tid; e < PL; e += NT) {
      const int ii = read_sc<MESH, NEAR>(x0 - H + e % PW, g.n1, g.ng);
      const int jj = read_sc<MESH, NEAR>(y0 - H + e / PW, g.n2, g.ng);
      const int q = g.c(ii, jj, kk);
      double rho = xb[q];
      // with floors, C uses the density of the floored primitives
      if (FL && isfinite(rho) && isfinite(xb[4 * g.cvar + q]) && !(rho >= sc.fl.d)) rho = sc.fl.d;
      ring[slot * PL + e] = sv[q] / rho;
    }
  };

#pragma unroll
  for (int z = 0; z < 2 * H; ++z) load_plane(k0 - H + z, z);
  // upper faces: the block's own lower faces, or on the upper boundary the
  // lower boundary face of the next block (the block itself when periodic)
  const int ip = wrap_sc<NEAR>(i + 1, g.n1, g.ng), jp = wrap_sc<NEAR>(j + 1, g.n2, g.ng);
  const double* fm1 = (MESH && i + 1 == g.ng + g.n1) ? fm_all + next_block<0>(g, b) * 3 * g.fvar : fm;
  const double* fm2 = (MESH && j + 1 == g.ng + g.n2) ? fm_all + next_block<1>(g, b) * 3 * g.fvar : fm;
  const double* fm3 = MESH ? fm_all + next_block<2>(g, b) * 3 * g.fvar : fm;
  const int l = (ty + H) * PW + tx + H;
  double f3lo = act ? fm[2 * g.fvar + g.f(i, j, k0)] : 0.0;
  for (int p = k0; p < kend; ++p) {
    const int base = p - k0;  // ring index of plane p - H
    load_plane(p + H, (base + 2 * H) % R);
    __syncthreads();
    if (act) {
      double lx[NW], ly[NW], lz[NW];
      const double* pc = ring + ((base + H) % R) * PL;
#pragma unroll
      for (int o = 0; o < NW; ++o) {
        lx[o] = pc[l + o - H];
        ly[o] = pc[l + (o - H) * PW];
        lz[o] = ring[((base + o) % R) * PL + l];
      }
      const double f1lo = fm[g.f(i, j, p)], f1up = fm1[g.f(ip, j, p)];
      const double f2lo = fm[g.fvar + g.f(i, j, p)], f2up = fm2[g.fvar + g.f(i, jp, p)];
      const double f3up = (p + 1 == g.ng + g.n3 ? fm3 : fm)[2 * g.fvar + g.f(i, j, wrap_sc<NEAR>(p + 1, g.n3, g.ng))];
      const double* lines[3] = {lx, ly, lz};
      const double flo[3] = {f1lo, f2lo, f3lo}, fup[3] = {f1up, f2up, f3up}, inv[3] = {i1, i2, i3};
      double sum = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double lm, rm, l0, r0, lp, rp;
        cell_edges<RECON>(lines[d], lm, rm);      // cell c-1
        cell_edges<RECON>(lines[d] + 1, l0, r0);  // cell c
        cell_edges<RECON>(lines[d] + 2, lp, rp);  // cell c+1
        // face c-1/2: left state rm, right state l0; face c+1/2: r0, lp
        const double flux_lo = flo[d] >= 0.0 ? flo[d] * rm : flo[d] * l0;
        const double flux_up = fup[d] >= 0.0 ? fup[d] * r0 : fup[d] * lp;
        sum += (flux_up - flux_lo) * inv[d];
      }
      const int64_t e = (5 + v) * g.cvar + g.c(i, j, p);
      double out = sc.cf.g1 * unb[e];
      if (sc.cf.g0 != 0.0) out += sc.cf.g0 * xb[e];
      ob[e] = out - bdt * sum;
      f3lo = f3up;
    }
  }
}

template <int RECON, bool FL, bool NEAR, bool MESH>
__global__ void __launch_bounds__(kSX * kSY) k_scalar_stage(ScalarArgs a) {
  __shared__ double ring[ScalarRing<RECON, kSX, kSY>::R * ScalarRing<RECON, kSX, kSY>::PL];
  const Geo& g = a.g;
  int64_t r = blockIdx.x;
  const int tile_x = (int)(r % a.ntx); r /= a.ntx;
  const int tile_y = (int)(r % a.nty); r /= a.nty;
  const int seg = (int)(r % a.nseg); r /= a.nseg;
  const int v = (int)(r % g.ns);
  const int b = (int)(r / g.ns);
  const int k0 = g.ng + seg * a.kz;
  const int kend = min(k0 + a.kz, g.ng + g.n3);
  scalar_tile<RECON, FL, NEAR, MESH, kSX, kSY>(g, a.sc, a.xc + b * g.cblock, a.unc + b * g.cblock,
                                              a.oc + b * g.cblock, a.fm + (int64_t)b * 3 * g.fvar, a.fm, b, tile_x,
                                              tile_y, k0, kend, v, ring);
}

// Batched blocks: one workgroup per (work item, scalar).
template <int RECON, bool FL, bool NEAR>
__global__ void __launch_bounds__(kBT * kBT) k_scalar_batch(ScalarBatchArgs a) {
  __shared__ double ring[ScalarRing<RECON, kBT, kBT>::R * ScalarRing<RECON, kBT, kBT>::PL];
  const WorkItem w = a.items[blockIdx.x / a.ns];
  const int v = blockIdx.x % a.ns;
  const BatchDesc& d = a.desc[w.block];
  scalar_tile<RECON, FL, NEAR, false, kBT, kBT>(d.g, a.sc, a.xc + d.coff, a.unc + d.coff, a.oc + d.coff,
                                                a.fm + d.foff, a.fm, w.block, w.tile_x, w.tile_y, w.k0, w.kend, v,
                                                ring);
}

template <int RECON, bool FL>
void launch_r(const ScalarArgs& sa, bool near, unsigned grid, hipStream_t s) {
  constexpr int NT = kSX * kSY;
  if (sa.g.mesh[0]) hipLaunchKernelGGL((k_scalar_stage<RECON, FL, true, true>), dim3(grid), dim3(NT), 0, s, sa);
  else if (near) hipLaunchKernelGGL((k_scalar_stage<RECON, FL, true, false>), dim3(grid), dim3(NT), 0, s, sa);
  else hipLaunchKernelGGL((k_scalar_stage<RECON, FL, false, false>), dim3(grid), dim3(NT), 0, s, sa);
}

template <int RECON>
void launch_f(const ScalarArgs& sa, bool near, unsigned grid, hipStream_t s) {
  if (sa.sc.fl.on()) launch_r<RECON, true>(sa, near, grid, s);
  else launch_r<RECON, false>(sa, near, grid, s);
}

template <int RECON, bool FL>
void launch_br(const ScalarBatchArgs& ba, bool near, unsigned grid, hipStream_t s) {
  constexpr int NT = kBT * kBT;
  if (near) hipLaunchKernelGGL((k_scalar_batch<RECON, FL, true>), dim3(grid), dim3(NT), 0, s, ba);
  else hipLaunchKernelGGL((k_scalar_batch<RECON, FL, false>), dim3(grid), dim3(NT), 0, s, ba);
}

template <int RECON>
void launch_bf(const ScalarBatchArgs& ba, bool near, unsigned grid, hipStream_t s) {
  if (ba.sc.fl.on()) launch_br<RECON, true>(ba, near, grid, s);
  else launch_br<RECON, false>(ba, near, grid, s);
}

}  // namespace

hipError_t launch_scalar_stage(const Geo& g, int recon, const double* xc, const double* unc, double* outc,
                               const double* fm, StageCoef coef, const double* dt_dev, double beta, int nb, Floors fl,
                               hipStream_t s) {
  if (g.ns <= 0) return hipSuccess;
  ScalarArgs sa{g, ScalarCoef{coef, dt_dev, beta, fl}, xc, unc, outc, fm, 0, 0, 0, 0};
  sa.ntx = (g.n1 + kSX - 1) / kSX;
  sa.nty = (g.n2 + kSY - 1) / kSY;
  // x3 segments: the longest of 32 .. 4 planes that still gives about 1024
  // workgroups (the ring's start-up costs 2 (LA + 1) planes per segment)
  const int64_t cols = (int64_t)sa.ntx * sa.nty * g.ns * nb;
  int kz = 32;
  while (kz > 4 && cols * ((g.n3 + kz - 1) / kz) < 1024) kz /= 2;
  sa.kz = kz < g.n3 ? kz : g.n3;
  sa.nseg = (g.n3 + sa.kz - 1) / sa.kz;
  const int64_t total = cols * sa.nseg;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  // one correction step finds every periodic image a stencil reaches when each
  // direction has more active cells than the halo
  const int h = recon + 1;
  const bool near = g.n1 > h && g.n2 > h && g.n3 > h;
  if (recon == 0) launch_f<0>(sa, near, (unsigned)total, s);
  else if (recon == 1) launch_f<1>(sa, near, (unsigned)total, s);
  else launch_f<2>(sa, near, (unsigned)total, s);
  return hipGetLastError();
}

int scalar_batch_tile() { return kBT; }

hipError_t launch_scalar_stage_batch(const BatchDesc* desc, const WorkItem* items, int nitems, int ns, bool near,
                                     int recon, const double* xc, const double* unc, double* outc, const double* fm,
                                     StageCoef coef, const double* dt_dev, double beta, Floors fl, hipStream_t s) {
  if (ns <= 0 || nitems <= 0) return hipSuccess;
  const int64_t total = (int64_t)nitems * ns;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  ScalarBatchArgs ba{desc, items, ns, ScalarCoef{coef, dt_dev, beta, fl}, xc, unc, outc, fm};
  if (recon == 0) launch_bf<0>(ba, near, (unsigned)total, s);
  else if (recon == 1) launch_bf<1>(ba, near, (unsigned)total, s);
  else launch_bf<2>(ba, near, (unsigned)total, s);
  return hipGetLastError();
}

}  // namespace athmhd
