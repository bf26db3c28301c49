// kernels_basic.hip -- ghost fill, prim->cons, CFL time step and copy kernels.
#include <algorithm>
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"
#include "mhd_math.hpp"

namespace athmhd {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Ghost cells and the periodic image faces (Sec. 2.1.1; a periodic block is
// its own neighbour).  Only the shell of stored entries outside the active box
// is visited: whole ghost planes along x3, then ghost rows along x2 of the
// active planes, then ghost entries along x1 of the active rows.  Every
// source is an active entry, so the three regions are independent.
__host__ __device__ __forceinline__ int ghost_index(int q, int n, int ng) { return q < ng ? q : q + n; }

__global__ void __launch_bounds__(kThreads) k_fill_ghosts(Geo g, double* __restrict__ cons,
                                                         double* __restrict__ bface) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nz = (int64_t)(g.F3 - g.n3) * g.F2 * g.F1;
  const int64_t ny = (int64_t)g.n3 * (g.F2 - g.n2) * g.F1;
  const int64_t nx = (int64_t)g.n3 * g.n2 * (g.F1 - g.n1);
  int i, j, k;
  if (t < nz) {
    i = (int)(t % g.F1);
    const int64_t r = t / g.F1;
    j = (int)(r % g.F2);
    k = ghost_index((int)(r / g.F2), g.n3, g.ng);
  } else if (t < nz + ny) {
    const int64_t u = t - nz;
    i = (int)(u % g.F1);
    const int64_t r = u / g.F1;
    j = ghost_index((int)(r % (g.F2 - g.n2)), g.n2, g.ng);
    k = g.ng + (int)(r / (g.F2 - g.n2));
  } else if (t < nz + ny + nx) {
    const int64_t u = t - nz - ny;
    i = ghost_index((int)(u % (g.F1 - g.n1)), g.n1, g.ng);
    const int64_t r = u / (g.F1 - g.n1);
    j = g.ng + (int)(r % g.n2);
    k = g.ng + (int)(r / g.n2);
  } else {
    return;
  }
  const int ii = wrap_index(i, g.n1, g.ng), jj = wrap_index(j, g.n2, g.ng), kk = wrap_index(k, g.n3, g.ng);
  double* cb = cons + blockIdx.y * g.cblock;
  double* fb = bface + blockIdx.y * g.fblock;
  if (i < g.N1 && j < g.N2 && k < g.N3) {
    const int d = g.c(i, j, k), s = g.c(ii, jj, kk);
#pragma unroll
    for (int v = 0; v < 5; ++v) cb[v * g.cvar + d] = cb[v * g.cvar + s];
    for (int v = 5; v < 5 + g.ns; ++v) cb[v * g.cvar + d] = cb[v * g.cvar + s];  // passive scalars
  }
  const int d = g.f(i, j, k), s = g.f(ii, jj, kk);
#pragma unroll
  for (int c = 0; c < 3; ++c) fb[c * g.fvar + d] = fb[c * g.fvar + s];
}

// Ghost exchange of a coupled mesh (Sec. 2.1.1): every stored entry of block
// b outside its active box (ghost cells, and faces other than the lower faces
// of its active cells) takes the value of the active entry that owns that
// position in the periodic domain tiled by the blocks: an active cell, or the
// lower face of an active cell, of this or a neighbouring block.  The shell
// enumeration is k_fill_ghosts'; sources are active entries only, so every
// destination is written once from data this kernel does not change.  With
// near = 1 (every block has more cells than ghost layers along each
// direction) the owner is at most one block away and is found without
// integer division.  Only the w ghost layers nearest the active box (and the
// faces bounding them) are filled: a stage whose stencil reaches w cells past
// the block needs no more.
__global__ void __launch_bounds__(kThreads) k_mesh_ghosts(Geo g, int w, int near, int open_x1,
                                                         double* __restrict__ cons, double* __restrict__ bface) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  // the filled box: stored indices [ng - w, ng + n + w] (faces), cells below ng + n + w
  const int E1 = g.n1 + 2 * w + 1, E2 = g.n2 + 2 * w + 1, E3 = g.n3 + 2 * w + 1;
  const int lo = g.ng - w;
  const int nz = (E3 - g.n3) * E2 * E1;
  const int ny = g.n3 * (E2 - g.n2) * E1;
  const int nx = g.n3 * g.n2 * (E1 - g.n1);
  int x[3];
  if (t < nz) {
    x[0] = lo + t % E1;
    const int r = t / E1;
    x[1] = lo + r % E2;
    x[2] = lo + ghost_index(r / E2, g.n3, w);
  } else if (t < nz + ny) {
    const int u = t - nz;
    x[0] = lo + u % E1;
    const int r = u / E1;
    x[1] = lo + ghost_index(r % (E2 - g.n2), g.n2, w);
    x[2] = g.ng + r / (E2 - g.n2);
  } else if (t < nz + ny + nx) {
    const int u = t - nz - ny;
    x[0] = lo + ghost_index(u % (E1 - g.n1), g.n1, w);
    const int r = u / (E1 - g.n1);
    x[1] = g.ng + r % g.n2;
    x[2] = g.ng + r / g.n2;
  } else {
    return;
  }
  const int b = blockIdx.y;
  const int m[3] = {g.mesh[0], g.mesh[1], g.mesh[2]};
  const int bc[3] = {b % m[0], (b / m[0]) % m[1], b / (m[0] * m[1])};
  const int n[3] = {g.n1, g.n2, g.n3};
  int sx[3], sb[3];
  // open_x1: entries beyond the mesh along x1 belong to another level and are
  // left alone, except the B1 faces on the mesh's upper x1 boundary plane,
  // which the last blocks along x1 own (copied here from the owner along x2, x3)
  bool plane = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int o = x[d] - g.ng;  // position relative to the block's first active cell
    if (near) {
      const int q = o < 0 ? -1 : (o >= n[d] ? 1 : 0);
      int c = bc[d] + q;
      if (d == 0 && open_x1 && (c < 0 || c >= m[0])) {
        if (c < 0 || o != n[0]) return;
        plane = true;
        sb[0] = bc[0];
        sx[0] = x[0];
        continue;
      }
      c = c < 0 ? c + m[d] : (c >= m[d] ? c - m[d] : c);
      sb[d] = c;
      sx[d] = g.ng + o - q * n[d];
    } else {
      const int len = m[d] * n[d];  // domain cells along d
      int p = bc[d] * n[d] + o;
      if (d == 0 && open_x1 && (p < 0 || p >= len)) {
        if (p != len) return;
        plane = true;
        sb[0] = bc[0];
        sx[0] = x[0];
        continue;
      }
      p = ((p % len) + len) % len;
      sb[d] = p / n[d];
      sx[d] = g.ng + p % n[d];
    }
  }
  const int src = sb[0] + m[0] * (sb[1] + m[1] * sb[2]);
  const double* sc = cons + (int64_t)src * g.cblock;
  const double* sf = bface + (int64_t)src * g.fblock;
  double* dc = cons + (int64_t)b * g.cblock;
  double* df = bface + (int64_t)b * g.fblock;
  if (plane) {  // the block's own plane faces (src == b) are active
    if (src != b) df[g.f(x[0], x[1], x[2])] = sf[g.f(sx[0], sx[1], sx[2])];
    return;
  }
  const int hi = g.ng + w;  // cells stop w layers past the active box, faces one entry further
  if (x[0] < g.n1 + hi && x[1] < g.n2 + hi && x[2] < g.n3 + hi) {
    const int d = g.c(x[0], x[1], x[2]), s = g.c(sx[0], sx[1], sx[2]);
#pragma unroll
    for (int v = 0; v < 5; ++v) dc[v * g.cvar + d] = sc[v * g.cvar + s];
    for (int v = 5; v < 5 + g.ns; ++v) dc[v * g.cvar + d] = sc[v * g.cvar + s];  // passive scalars
  }
  const int d = g.f(x[0], x[1], x[2]), s = g.f(sx[0], sx[1], sx[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) df[c * g.fvar + d] = sf[c * g.fvar + s];
}

inline int64_t ghost_count(const Geo& g) {
  return (int64_t)(g.F3 - g.n3) * g.F2 * g.F1 + (int64_t)g.n3 * (g.F2 - g.n2) * g.F1 +
         (int64_t)g.n3 * g.n2 * (g.F1 - g.n1);
}

// Cell-centred field of active cell (i, j, k) of block b: the mean of its
// lower and upper faces.  An upper face on the block's upper boundary is the
// lower boundary face of the next block along that direction (the block
// itself when it is its own periodic neighbour) and is read there, not from
// the stored image entries, which a step does not refresh.  fb: this block's
// face arrays; all_fb: block 0's (read by coupled meshes only; other callers
// pass fb).  Geometries with mesh[0] < 0 (the blocks of a two-level
// composite, whose ghosts are filled after every step) read the stored upper
// faces.
__device__ __forceinline__ void cell_field(const Geo& g, const double* fb, const double* all_fb, int b, int i, int j,
                                           int k, double& b1, double& b2, double& b3) {
  const int f = g.f(i, j, k);
  if (g.mesh[0] < 0) {  // blocks whose upper boundary faces are stored (filled ghosts)
    b1 = 0.5 * (fb[f] + fb[g.f(i + 1, j, k)]);
    b2 = 0.5 * (fb[g.fvar + f] + fb[g.fvar + g.f(i, j + 1, k)]);
    b3 = 0.5 * (fb[2 * g.fvar + f] + fb[2 * g.fvar + g.f(i, j, k + 1)]);
    return;
  }
  const double* p1 = fb;
  const double* p2 = fb;
  const double* p3 = fb;
  int iu = i + 1, ju = j + 1, ku = k + 1;
  if (iu == g.ng + g.n1) {
    iu = g.ng;
    if (g.mesh[0]) p1 = all_fb + next_block<0>(g, b) * g.fblock;
  }
  if (ju == g.ng + g.n2) {
    ju = g.ng;
    if (g.mesh[0]) p2 = all_fb + next_block<1>(g, b) * g.fblock;
  }
  if (ku == g.ng + g.n3) {
    ku = g.ng;
    if (g.mesh[0]) p3 = all_fb + next_block<2>(g, b) * g.fblock;
  }
  b1 = 0.5 * (fb[f] + p1[g.f(iu, j, k)]);
  b2 = 0.5 * (fb[g.fvar + f] + p2[g.fvar + g.f(i, ju, k)]);
  b3 = 0.5 * (fb[2 * g.fvar + f] + p3[2 * g.fvar + g.f(i, j, ku)]);
}

// Conserved variables from primitives with the cell-centred field (mean of the
// two bounding faces), Eq. (total_energy) with P = (gamma-1) e.
__global__ void __launch_bounds__(kThreads) k_prim2cons(Geo g, double gamma, const double* __restrict__ prim,
                                                       const double* __restrict__ bface,
                                                       double* __restrict__ cons) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= g.cvar) return;
  const int i = (int)(t % g.N1);
  const int r = (int)(t / g.N1);
  const int j = r % g.N2, k = r / g.N2;
  const double* w = prim + blockIdx.y * g.cblock;
  const double* fb = bface + blockIdx.y * g.fblock;
  double* u = cons + blockIdx.y * g.cblock;
  double b1, b2, b3;
  if (i >= g.ng && i < g.ng + g.n1 && j >= g.ng && j < g.ng + g.n2 && k >= g.ng && k < g.ng + g.n3) {
    cell_field(g, fb, bface, blockIdx.y, i, j, k, b1, b2, b3);
  } else {  // ghost cells: their stored faces
    b1 = 0.5 * (fb[g.f(i, j, k)] + fb[g.f(i + 1, j, k)]);
    b2 = 0.5 * (fb[g.fvar + g.f(i, j, k)] + fb[g.fvar + g.f(i, j + 1, k)]);
    b3 = 0.5 * (fb[2 * g.fvar + g.f(i, j, k)] + fb[2 * g.fvar + g.f(i, j, k + 1)]);
  }
  const double rho = w[t], v1 = w[g.cvar + t], v2 = w[2 * g.cvar + t], v3 = w[3 * g.cvar + t];
  const double p = w[4 * g.cvar + t];
  u[t] = rho;
  u[g.cvar + t] = rho * v1;
  u[2 * g.cvar + t] = rho * v2;
  u[3 * g.cvar + t] = rho * v3;
  u[4 * g.cvar + t] = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) + 0.5 * (b1 * b1 + b2 * b2 + b3 * b3);
  // passive scalars: masses rho C_i from the specific densities C_i
  for (int v = 5; v < 5 + g.ns; ++v) u[v * g.cvar + t] = rho * w[v * g.cvar + t];
}

// Smallest dx_d / (|v_d| + c_f,d) over the active cells (Sec. 2.1.7, Sec. 3.2.3).
// Grid-stride loop per thread, wavefront min by cross-lane shuffles, LDS
// across the workgroup, then one atomicMin per workgroup on the bit pattern
// (non-negative doubles order like their bits).
constexpr int kDtBlocks = 1024;

// End of a CFL workgroup: its minimum and non-physical count, either merged
// into the global result word and counter with atomics (PARTS = false) or
// written as the workgroup's partial result parts[wg] (PARTS = true; a later
// reduction reads them, so nothing needs clearing before the launch).
template <bool PARTS>
__device__ __forceinline__ void dt_workgroup_end(double best, int nbad, unsigned long long* dt_bits, int* bad,
                                                 DtPart* parts, int64_t wg) {
  if (!PARTS && nbad) atomicAdd(bad, nbad);
  // wavefront minimum (and count)
  for (int off = 32; off > 0; off >>= 1) {
    best = fmin(best, __shfl_xor(best, off, 64));
    if (PARTS) nbad += __shfl_xor(nbad, off, 64);
  }
  __shared__ double part[kThreads / 64];
  __shared__ int pbad[kThreads / 64];
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = best;
    pbad[threadIdx.x >> 6] = nbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    int nb = pbad[0];
    for (int w = 1; w < kThreads / 64; ++w) {
      m = fmin(m, part[w]);
      nb += pbad[w];
    }
    if (PARTS) {
      parts[wg].m = m;
      parts[wg].nbad = nb;
    } else if (m < DBL_MAX) {
      atomicMin(dt_bits, (unsigned long long)__double_as_longlong(m));
    }
  }
}

template <bool PARTS>
__global__ void __launch_bounds__(kThreads) k_newdt(Geo g, double gamma, Floors fl, const double* __restrict__ cons,
                                                   const double* __restrict__ bface,
                                                   unsigned long long* __restrict__ dt_bits,
                                                   int* __restrict__ bad, DtPart* __restrict__ parts) {
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  const double* u = cons + blockIdx.y * g.cblock;
  const double* fb = bface + blockIdx.y * g.fblock;
  double best = DBL_MAX;
  int nbad = 0;
  // a block holds fewer than 2^31 cells, so the cell index fits 32 bits
  for (int t = blockIdx.x * kThreads + threadIdx.x; t < (int)nact; t += gridDim.x * kThreads) {
    const int i = g.ng + t % g.n1;
    const int r = t / g.n1;
    const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
    const int q = g.c(i, j, k);
    double bc[3];
    cell_field(g, fb, bface, blockIdx.y, i, j, k, bc[0], bc[1], bc[2]);
    const double uc[5] = {u[q], u[g.cvar + q], u[2 * g.cvar + q], u[3 * g.cvar + q], u[4 * g.cvar + q]};
    double d;
    if (cfl_cell(uc, bc, gamma, fl, g.dx1, g.dx2, g.dx3, d)) best = fmin(best, d);
    else ++nbad;
  }
  dt_workgroup_end<PARTS>(best, nbad, dt_bits, bad, parts, (int64_t)blockIdx.y * gridDim.x + blockIdx.x);
}

// The floors on the values of one cell: uc = (rho, M1, M2, M3, E), b its
// cell-centred field; raises rho to the density floor and E so that the
// pressure is the pressure floor.  Bit 0: rho changed, bit 1: E changed.
__device__ __forceinline__ int floor_values(double gm1, const Floors& fl, double* uc, const double* b) {
  int hit = 0;
  if (!(uc[0] >= fl.d)) {
    uc[0] = fl.d;
    hit = 1;
  }
  const double rho = uc[0];
  const double m1 = uc[1], m2 = uc[2], m3 = uc[3];
  const double kin = 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / rho;
  const double mag = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const double p = gm1 * (uc[4] - kin - mag);
  if (!(p >= fl.p)) {
    uc[4] = fl.p / gm1 + kin + mag;
    hit |= 2;
  }
  return hit;
}

// The same reduction as a march along x3: one thread per (i, j) column of a
// 64 x 4 tile of columns, over a segment of kz planes.  A cell's upper B3 is
// the next cell's lower B3, kept in a register, so each face is read from
// memory once: 64 B per cell against the grid-stride loop's re-reads of the
// upper x2 and x3 faces.  The upper faces are found as cell_field finds them.
// FLOOR: apply the floors of k_floor_state to each cell first, writing the
// cells they change, so that the pass that ends a step with floors reads the
// state once for both.
constexpr int kMarchX = 64, kMarchY = kThreads / kMarchX;
template <bool FLOOR>
// Workgroups are numbered (tile, x3 segment, block), tile (x1 first) fastest;
// launch slot s runs number (s mod 8) per_xcd + s / 8, so that neighbouring
// tiles, which share cache lines at their x1 edges, run on one XCD and meet
// in its L2.
__global__ void __launch_bounds__(kThreads) k_newdt_march(Geo g, double gamma, Floors fl, double* __restrict__ cons,
                                                         const double* __restrict__ bface, int ntx, int nty, int nseg,
                                                         int kz, int total, int per_xcd,
                                                         unsigned long long* __restrict__ dt_bits,
                                                         int* __restrict__ bad) {
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;  // the whole workgroup: the padding of the last XCD
  const int ntiles = ntx * nty;
  const int tile = logical % ntiles, seg = (logical / ntiles) % nseg;
  const int b = logical / (ntiles * nseg);
  const int i = g.ng + (tile % ntx) * kMarchX + (int)(threadIdx.x % kMarchX);
  const int j = g.ng + (tile / ntx) * kMarchY + (int)(threadIdx.x / kMarchX);
  const int k0 = g.ng + seg * kz, kend = min(k0 + kz, g.ng + g.n3);
  double* u = cons + (int64_t)b * g.cblock;
  const double* fb = bface + (int64_t)b * g.fblock;
  double best = DBL_MAX;
  int nbad = 0, nfloor = 0;
  if (i < g.ng + g.n1 && j < g.ng + g.n2 && k0 < kend) {
    // this column's upper x1 and x2 faces: the stored ones (a composite's
    // blocks), the periodic image in the block, or the next block of a mesh
    const double* p1 = fb;
    const double* p2 = fb;
    int iu = i + 1, ju = j + 1;
    if (g.mesh[0] >= 0 && iu == g.ng + g.n1) {
      iu = g.ng;
      if (g.mesh[0]) p1 = bface + (int64_t)next_block<0>(g, b) * g.fblock;
    }
    if (g.mesh[0] >= 0 && ju == g.ng + g.n2) {
      ju = g.ng;
      if (g.mesh[0]) p2 = bface + (int64_t)next_block<1>(g, b) * g.fblock;
    }
    double b3lo = fb[2 * g.fvar + g.f(i, j, k0)];
    for (int k = k0; k < kend; ++k) {
      const double* p3 = fb;
      int ku = k + 1;
      if (g.mesh[0] >= 0 && ku == g.ng + g.n3) {
        ku = g.ng;
        if (g.mesh[0]) p3 = bface + (int64_t)next_block<2>(g, b) * g.fblock;
      }
      const int q = g.c(i, j, k), f = g.f(i, j, k);
      double uc[5] = {u[q], u[g.cvar + q], u[2 * g.cvar + q], u[3 * g.cvar + q], u[4 * g.cvar + q]};
      const double b3hi = p3[2 * g.fvar + g.f(i, j, ku)];
      const double bc[3] = {0.5 * (fb[f] + p1[g.f(iu, j, k)]), 0.5 * (fb[g.fvar + f] + p2[g.fvar + g.f(i, ju, k)]),
                            0.5 * (b3lo + b3hi)};
      if (FLOOR) {
        const int hit = floor_values(gamma - 1.0, fl, uc, bc);
        if (hit & 1) u[q] = uc[0];
        if (hit & 2) u[4 * g.cvar + q] = uc[4];
        nfloor += hit != 0;
      }
      double d;
      if (cfl_cell(uc, bc, gamma, fl, g.dx1, g.dx2, g.dx3, d)) best = fmin(best, d);
      else ++nbad;
      b3lo = b3hi;
    }
  }
  if (FLOOR && nfloor) add_floor_count(bad, (unsigned long long)nfloor);
  dt_workgroup_end<false>(best, nbad, dt_bits, bad, nullptr, 0);
}

// Floors on the conserved state after a stage (floors enabled only): density
// below the floor is raised to it, and where the pressure implied by (U, B)
// is below the pressure floor the total energy is raised to give exactly that
// pressure.  The cell-centred field is that of cell_field.  Changed cells are
// counted with add_floor_count.
__device__ __forceinline__ int floor_cell(const Geo& g, double gm1, const Floors& fl, double* u,
                                          const double* fb, const double* all_fb, int b, int i, int j, int k) {
  const int q = g.c(i, j, k);
  double bc[3];
  cell_field(g, fb, all_fb, b, i, j, k, bc[0], bc[1], bc[2]);
  double uc[5] = {u[q], u[g.cvar + q], u[2 * g.cvar + q], u[3 * g.cvar + q], u[4 * g.cvar + q]};
  const int hit = floor_values(gm1, fl, uc, bc);
  if (hit & 1) u[q] = uc[0];
  if (hit & 2) u[4 * g.cvar + q] = uc[4];
  return hit != 0;
}

__global__ void __launch_bounds__(kThreads) k_floor_state(Geo g, double gm1, Floors fl, double* __restrict__ cons,
                                                         const double* __restrict__ bface, int* __restrict__ bad) {
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= nact) return;
  const int i = g.ng + (int)(t % g.n1);
  const int r = (int)(t / g.n1);
  const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
  if (floor_cell(g, gm1, fl, cons + blockIdx.y * g.cblock, bface + blockIdx.y * g.fblock, bface, blockIdx.y, i, j, k))
    add_floor_count(bad, 1ull);
}

__global__ void __launch_bounds__(kThreads) k_floor_state_batch(const BatchDesc* __restrict__ desc, double gm1,
                                                               Floors fl, double* __restrict__ cons,
                                                               const double* __restrict__ bface,
                                                               int* __restrict__ bad) {
  const BatchDesc& d = desc[blockIdx.y];
  const Geo& g = d.g;
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  int hits = 0;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nact; t += (int64_t)gridDim.x * kThreads) {
    const int i = g.ng + (int)(t % g.n1);
    const int r = (int)(t / g.n1);
    const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
    hits += floor_cell(g, gm1, fl, cons + d.coff, bface + d.foff, bface + d.foff, 0, i, j, k);
  }
  if (hits) add_floor_count(bad, (unsigned long long)hits);
}

__global__ void __launch_bounds__(kThreads) k_copy(double* __restrict__ dst, const double* __restrict__ src,
                                                  int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// ---- batched variants: blockIdx.y selects the block, its geometry and the
// offsets of its arrays come from the descriptor table
__global__ void __launch_bounds__(kThreads) k_fill_ghosts_batch(const BatchDesc* __restrict__ desc, double* cons,
                                                               double* bface) {
  const BatchDesc& d = desc[blockIdx.y];
  const Geo& g = d.g;
  const int64_t nshell = g.fvar - (int64_t)g.n1 * g.n2 * g.n3;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < nshell; t += (int64_t)gridDim.x * kThreads) {
    int i, j, k;
    shell_entry(g, t, i, j, k);
    const int ii = wrap_index(i, g.n1, g.ng), jj = wrap_index(j, g.n2, g.ng), kk = wrap_index(k, g.n3, g.ng);
    double* cb = cons + d.coff;
    double* fb = bface + d.foff;
    if (i < g.N1 && j < g.N2 && k < g.N3) {
      const int dd = g.c(i, j, k), ss = g.c(ii, jj, kk);
#pragma unroll
      for (int v = 0; v < 5; ++v) cb[v * g.cvar + dd] = cb[v * g.cvar + ss];
      for (int v = 5; v < 5 + g.ns; ++v) cb[v * g.cvar + dd] = cb[v * g.cvar + ss];  // passive scalars
    }
    const int dd = g.f(i, j, k), ss = g.f(ii, jj, kk);
#pragma unroll
    for (int c = 0; c < 3; ++c) fb[c * g.fvar + dd] = fb[c * g.fvar + ss];
  }
}

// Ghost exchange of batched blocks that tile one periodic domain: shell entry
// t of block b takes its cell and that cell's three lower faces from the
// block owning the same cell of the domain, src[off[b] + t] = (owner, the
// owner's stored position packed as i | j << 10 | k << 20).  Sources are
// active entries and destinations shell entries, so no entry is both read
// and written by a launch.  Workgroup w copies entries [t0, t0 + kXchgChunk)
// of block b, (b, t0) = work[w], kXchgChunk / kThreads per thread.
constexpr int kXchgChunk = 4 * kThreads;
__global__ void __launch_bounds__(kThreads) k_exchange_batch(const BatchDesc* __restrict__ desc,
                                                            const int64_t* __restrict__ off,
                                                            const int2* __restrict__ src,
                                                            const int2* __restrict__ work, double* cons,
                                                            double* bface) {
  const int2 w = work[blockIdx.x];
  const BatchDesc& d = desc[w.x];
  const Geo& g = d.g;
  const int64_t nshell = g.fvar - (int64_t)g.n1 * g.n2 * g.n3;
  const int2* sb = src + off[w.x];
  double* cb = cons + d.coff;
  double* fb = bface + d.foff;
  const int64_t tend = min(nshell, (int64_t)w.y + kXchgChunk);
  for (int64_t t = (int64_t)w.y + threadIdx.x; t < tend; t += kThreads) {
    int i, j, k;
    shell_entry(g, t, i, j, k);
    const int2 e = sb[t];
    const BatchDesc& o = desc[e.x];
    const int si = e.y & 1023, sj = (e.y >> 10) & 1023, sk = (e.y >> 20) & 1023;
    const double* oc = cons + o.coff;
    const double* ofb = bface + o.foff;
    if (i < g.N1 && j < g.N2 && k < g.N3) {
      const int dd = g.c(i, j, k), ss = o.g.c(si, sj, sk);
#pragma unroll
      for (int v = 0; v < 5; ++v) cb[v * g.cvar + dd] = oc[v * o.g.cvar + ss];
      for (int v = 5; v < 5 + g.ns; ++v) cb[v * g.cvar + dd] = oc[v * o.g.cvar + ss];
    }
    const int dd = g.f(i, j, k), ss = o.g.f(si, sj, sk);
#pragma unroll
    for (int c = 0; c < 3; ++c) fb[c * g.fvar + dd] = ofb[c * o.g.fvar + ss];
  }
}

__global__ void __launch_bounds__(kThreads) k_prim2cons_batch(const BatchDesc* __restrict__ desc, double gamma,
                                                             const double* __restrict__ prim,
                                                             const double* __restrict__ bface,
                                                             double* __restrict__ cons) {
  const BatchDesc& d = desc[blockIdx.y];
  const Geo& g = d.g;
  const double* w = prim + d.coff;
  const double* fb = bface + d.foff;
  double* u = cons + d.coff;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < g.cvar; t += (int64_t)gridDim.x * kThreads) {
    const int i = (int)(t % g.N1);
    const int r = (int)(t / g.N1);
    const int j = r % g.N2, k = r / g.N2;
    const double b1 = 0.5 * (fb[g.f(i, j, k)] + fb[g.f(i + 1, j, k)]);
    const double b2 = 0.5 * (fb[g.fvar + g.f(i, j, k)] + fb[g.fvar + g.f(i, j + 1, k)]);
    const double b3 = 0.5 * (fb[2 * g.fvar + g.f(i, j, k)] + fb[2 * g.fvar + g.f(i, j, k + 1)]);
    const double rho = w[t], v1 = w[g.cvar + t], v2 = w[2 * g.cvar + t], v3 = w[3 * g.cvar + t];
    const double p = w[4 * g.cvar + t];
    u[t] = rho;
    u[g.cvar + t] = rho * v1;
    u[2 * g.cvar + t] = rho * v2;
    u[3 * g.cvar + t] = rho * v3;
    u[4 * g.cvar + t] =
        p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) + 0.5 * (b1 * b1 + b2 * b2 + b3 * b3);
    for (int v = 5; v < 5 + g.ns; ++v) u[v * g.cvar + t] = rho * w[v * g.cvar + t];  // passive scalars
  }
}

// a few workgroups per block: their minima of dx_d/(|v_d| + c_f,d), then one
// atomicMin per workgroup (or one partial result, PARTS)
template <bool PARTS>
__global__ void __launch_bounds__(kThreads) k_newdt_batch(const BatchDesc* __restrict__ desc, double gamma,
                                                         Floors fl, const double* __restrict__ cons,
                                                         const double* __restrict__ bface,
                                                         unsigned long long* __restrict__ dt_bits,
                                                         int* __restrict__ bad, DtPart* __restrict__ parts) {
  const BatchDesc& d = desc[blockIdx.y];
  const Geo& g = d.g;
  const double* u = cons + d.coff;
  const double* fb = bface + d.foff;
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  double best = DBL_MAX;
  int nbad = 0;
  for (int t = blockIdx.x * kThreads + threadIdx.x; t < (int)nact; t += gridDim.x * kThreads) {
    const int i = g.ng + t % g.n1;
    const int r = t / g.n1;
    const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
    const int q = g.c(i, j, k);
    double bc[3];
    cell_field(g, fb, fb, 0, i, j, k, bc[0], bc[1], bc[2]);  // batched blocks: their own neighbours
    const double uc[5] = {u[q], u[g.cvar + q], u[2 * g.cvar + q], u[3 * g.cvar + q], u[4 * g.cvar + q]};
    double d;
    if (cfl_cell(uc, bc, gamma, fl, g.dx1, g.dx2, g.dx3, d)) best = fmin(best, d);
    else ++nbad;
  }
  dt_workgroup_end<PARTS>(best, nbad, dt_bits, bad, parts, (int64_t)blockIdx.y * gridDim.x + blockIdx.x);
}

// Reduction of nparts partial CFL results in one workgroup, in a fixed order
// (the result does not depend on the scheduling of the partial launch):
// dt_out = cfl * min (+inf when no cell was physical); nbad_out = the
// partial counts plus step_bad[0] (non-physical cells met by steps since the
// last newdt), and step_bad[0] is cleared.
__global__ void __launch_bounds__(kThreads) k_newdt_finish(const DtPart* __restrict__ parts, int nparts, double cfl,
                                                          int* __restrict__ step_bad, double* __restrict__ dt_out,
                                                          int* __restrict__ nbad_out) {
  double best = DBL_MAX;
  int nbad = 0;
  for (int t = threadIdx.x; t < nparts; t += kThreads) {
    best = fmin(best, parts[t].m);
    nbad += parts[t].nbad;
  }
  for (int off = 32; off > 0; off >>= 1) {
    best = fmin(best, __shfl_xor(best, off, 64));
    nbad += __shfl_xor(nbad, off, 64);
  }
  __shared__ double part[kThreads / 64];
  __shared__ int pbad[kThreads / 64];
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = best;
    pbad[threadIdx.x >> 6] = nbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    int nb = pbad[0];
    for (int w = 1; w < kThreads / 64; ++w) {
      m = fmin(m, part[w]);
      nb += pbad[w];
    }
    nb += step_bad[0];
    step_bad[0] = 0;
    *dt_out = cfl * (m < DBL_MAX ? m : (double)INFINITY);
    *nbad_out = nb;
  }
}

}  // namespace

hipError_t launch_fill_ghosts_batch(const BatchDesc* desc, int nblocks, int64_t max_shell, double* cons,
                                    double* bface, hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(grid_for(max_shell), 64);
  hipLaunchKernelGGL(k_fill_ghosts_batch, dim3(gx, nblocks), dim3(kThreads), 0, s, desc, cons, bface);
  return hipGetLastError();
}

int exchange_chunk() { return kXchgChunk; }

hipError_t launch_exchange_batch(const BatchDesc* desc, const int64_t* off, const int2* src, const int2* work,
                                 int nwork, double* cons, double* bface, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exchange_batch, dim3(nwork), dim3(kThreads), 0, s, desc, off, src, work, cons, bface);
  return hipGetLastError();
}

hipError_t launch_prim2cons_batch(const BatchDesc* desc, int nblocks, int64_t max_cells, double gamma,
                                  const double* prim, const double* bface, double* cons, hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(grid_for(max_cells), 64);
  hipLaunchKernelGGL(k_prim2cons_batch, dim3(gx, nblocks), dim3(kThreads), 0, s, desc, gamma, prim, bface, cons);
  return hipGetLastError();
}

hipError_t launch_newdt_batch(const BatchDesc* desc, int nblocks, int64_t, double gamma, const double* cons,
                              const double* bface, unsigned long long* dt_bits, const Floors& fl, int* bad,
                              hipStream_t s) {
  // a few workgroups per block so that small blocks do not serialise
  hipLaunchKernelGGL(k_newdt_batch<false>, dim3(4, nblocks), dim3(kThreads), 0, s, desc, gamma, fl, cons, bface,
                     dt_bits, bad, nullptr);
  return hipGetLastError();
}

hipError_t launch_newdt_parts_batch(const BatchDesc* desc, int nblocks, double gamma, const double* cons,
                                    const double* bface, const Floors& fl, DtPart* parts, int max_parts, int* nparts,
                                    hipStream_t s) {
  if (nblocks < 1 || nblocks > max_parts) return hipErrorInvalidValue;
  const int gx = std::max(1, std::min(4, max_parts / nblocks));
  *nparts = gx * nblocks;
  hipLaunchKernelGGL(k_newdt_batch<true>, dim3(gx, nblocks), dim3(kThreads), 0, s, desc, gamma, fl, cons, bface,
                     nullptr, nullptr, parts);
  return hipGetLastError();
}

hipError_t launch_newdt_finish(const DtPart* parts, int nparts, double cfl, int* step_bad, double* dt_out,
                               int* nbad_out, hipStream_t s) {
  hipLaunchKernelGGL(k_newdt_finish, dim3(1), dim3(kThreads), 0, s, parts, nparts, cfl, step_bad, dt_out, nbad_out);
  return hipGetLastError();
}

hipError_t launch_floor_state(const Geo& g, double gamma, const Floors& fl, double* cons, const double* bface, int nb,
                              int* bad, hipStream_t s) {
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(k_floor_state, dim3(grid_for(nact), nb), dim3(kThreads), 0, s, g, gamma - 1.0, fl, cons, bface,
                     bad);
  return hipGetLastError();
}

hipError_t launch_floor_state_batch(const BatchDesc* desc, int nblocks, double gamma, const Floors& fl, double* cons,
                                    const double* bface, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_floor_state_batch, dim3(16, nblocks), dim3(kThreads), 0, s, desc, gamma - 1.0, fl, cons,
                     bface, bad);
  return hipGetLastError();
}

hipError_t launch_fill_ghosts(const Geo& g, double* cons, double* bface, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_ghosts, dim3(grid_for(ghost_count(g)), nb), dim3(kThreads), 0, s, g, cons, bface);
  return hipGetLastError();
}

hipError_t launch_mesh_ghosts(const Geo& g, int w, double* cons, double* bface, hipStream_t s, bool open_x1) {
  if (w < 1 || w > g.ng) w = g.ng;
  const int nb = g.mesh[0] * g.mesh[1] * g.mesh[2];
  // the owner of a ghost entry is at most one block away when every block has
  // more cells than the filled layers (the entries reach w + 1 past the block)
  const int near = g.n1 > w && g.n2 > w && g.n3 > w;
  const int64_t E1 = g.n1 + 2 * w + 1, E2 = g.n2 + 2 * w + 1, E3 = g.n3 + 2 * w + 1;
  const int64_t count = (E3 - g.n3) * E2 * E1 + (int64_t)g.n3 * (E2 - g.n2) * E1 + (int64_t)g.n3 * g.n2 * (E1 - g.n1);
  hipLaunchKernelGGL(k_mesh_ghosts, dim3(grid_for(count), nb), dim3(kThreads), 0, s, g, w, near, open_x1 ? 1 : 0,
                     cons, bface);
  return hipGetLastError();
}

hipError_t launch_prim2cons(const Geo& g, double gamma, const double* prim, const double* bface, double* cons,
                            int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_prim2cons, dim3(grid_for(g.cvar), nb), dim3(kThreads), 0, s, g, gamma, prim, bface, cons);
  return hipGetLastError();
}

hipError_t launch_newdt(const Geo& g, double gamma, const double* cons, const double* bface, int nb,
                        unsigned long long* dt_bits, const Floors& fl, int* bad, hipStream_t s, bool floor) {
  // x3 segments: about 2 kDtBlocks workgroups in all (enough to fill the chip,
  // few enough atomics on the one result word), at least 8 planes each
  const int ntx = (g.n1 + kMarchX - 1) / kMarchX, nty = (g.n2 + kMarchY - 1) / kMarchY;
  const int64_t tiles = (int64_t)ntx * nty * std::max(nb, 1);
  const int64_t want = (2 * kDtBlocks + tiles - 1) / tiles;
  const int nseg0 = (int)std::max<int64_t>(1, std::min<int64_t>(want, std::max(1, g.n3 / 8)));
  const int kz = (g.n3 + nseg0 - 1) / nseg0;
  const int nseg = (g.n3 + kz - 1) / kz;
  const int64_t total = tiles * nseg;
  if (total > INT32_MAX / 2) return hipErrorInvalidValue;
  const int per_xcd = (int)((total + 7) / 8);
  const dim3 grid((unsigned)(8 * per_xcd), 1u);
  if (floor)
    hipLaunchKernelGGL(k_newdt_march<true>, grid, dim3(kThreads), 0, s, g, gamma, fl, const_cast<double*>(cons), bface,
                       ntx, nty, nseg, kz, (int)total, per_xcd, dt_bits, bad);
  else
    hipLaunchKernelGGL(k_newdt_march<false>, grid, dim3(kThreads), 0, s, g, gamma, fl, const_cast<double*>(cons),
                       bface, ntx, nty, nseg, kz, (int)total, per_xcd, dt_bits, bad);
  return hipGetLastError();
}

hipError_t launch_newdt_parts(const Geo& g, double gamma, const double* cons, const double* bface, int nb,
                              const Floors& fl, DtPart* parts, int max_parts, int* nparts, hipStream_t s) {
  if (nb < 1 || nb > max_parts) return hipErrorInvalidValue;
  const int64_t nact = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t per_block = std::max<int64_t>(1, std::min<int64_t>(kDtBlocks, max_parts / nb));
  const unsigned blocks = (unsigned)std::min<int64_t>(grid_for(nact), per_block);
  *nparts = (int)blocks * nb;
  hipLaunchKernelGGL(k_newdt<true>, dim3(blocks, nb), dim3(kThreads), 0, s, g, gamma, fl, cons, bface, nullptr,
                     nullptr, parts);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace athmhd
