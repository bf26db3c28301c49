// common.hpp -- block geometry, launch helpers and kernel entry points shared
// by the host ABI and the HIP kernels of libathmhd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace athmhd {

// Geometry of one MeshBlock as stored: n_d active cells, ng ghost layers on
// each side (Sec. 2.1.1), N_d = n_d + 2 ng stored cells, face arrays padded to
// N_d + 1 in every direction.  i (direction 1) is fastest.
struct Geo {
  int n1, n2, n3, ng;
  int ns;          // passive scalars rho C_i, stored as cell arrays after the 5 MHD variables
  int N1, N2, N3;
  int F1, F2, F3;
  int64_t cvar;    // cells per variable (stride between cell arrays)
  int64_t fvar;    // faces per component (stride between face arrays)
  int64_t cblock;  // (5 + ns) * cvar: stride between blocks in cons
  int64_t fblock;  // 3 * fvar: stride between blocks in bface
  double dx1, dx2, dx3;
  // Blocks per direction of a coupled mesh: equal blocks that tile one
  // periodic domain, block b at (b mod m0, (b / m0) mod m1, b / (m0 m1)), each
  // reading its neighbours' cells through its ghost entries (Sec. 2.1.1).
  // All 0: every block is its own periodic neighbour.  mesh[0] = -1: the
  // block's upper boundary faces are stored entries filled from its
  // neighbours (blocks of a two-level composite or of a coupled batch).
  int mesh[3];

  __host__ __device__ __forceinline__ int c(int i, int j, int k) const { return (k * N2 + j) * N1 + i; }
  __host__ __device__ __forceinline__ int f(int i, int j, int k) const { return (k * F2 + j) * F1 + i; }
};

inline Geo make_geo(int n1, int n2, int n3, int ng, double dx1, double dx2, double dx3, int ns = 0) {
  Geo g;
  g.n1 = n1; g.n2 = n2; g.n3 = n3; g.ng = ng;
  g.ns = ns;
  g.N1 = n1 + 2 * ng; g.N2 = n2 + 2 * ng; g.N3 = n3 + 2 * ng;
  g.F1 = g.N1 + 1; g.F2 = g.N2 + 1; g.F3 = g.N3 + 1;
  g.cvar = (int64_t)g.N1 * g.N2 * g.N3;
  g.fvar = (int64_t)g.F1 * g.F2 * g.F3;
  g.cblock = (5 + ns) * g.cvar;
  g.fblock = 3 * g.fvar;
  g.dx1 = dx1; g.dx2 = dx2; g.dx3 = dx3;
  g.mesh[0] = g.mesh[1] = g.mesh[2] = 0;
  return g;
}

// Coefficients of one stage of the 2S scheme (Eq. (rk-2s)):
//   out = g0 * x + g1 * un + beta * dt * L(x)
struct StageCoef {
  double g0, g1, bdt;
};

// Optional density and pressure floors (0 disables each).  The primitives
// taken from a cell or reconstructed on a face are limited from below, and a
// separate pass after each stage raises the stored density and total energy
// of a cell that fell below them; that pass is the only change the floors make
// to the conserved variables.
struct Floors {
  double d, p;
  __host__ __device__ bool on() const { return d > 0.0 || p > 0.0; }
};

// Event counters of a handle, one device array of four ints: [0] counts
// non-physical cells met since the last newdt; ints [2, 4) hold the 64-bit
// count of floor activations, which a long run with floors can take past 2^31.
__device__ __forceinline__ void add_floor_count(int* bad, unsigned long long n) {
  atomicAdd(reinterpret_cast<unsigned long long*>(bad + 2), n);
}

// Periodic image of a stored index along a direction with n active cells.
__host__ __device__ __forceinline__ int wrap_index(int idx, int n, int ng) {
  int r = (idx - ng) % n;
  if (r < 0) r += n;
  return ng + r;
}

// Entry t of a block's shell: the stored positions (i, j, k) of the face box
// (F1 x F2 x F3) outside the block's active cells, t in [0, fvar - n1 n2 n3),
// in the order x3 slabs (all i, j), x2 slabs (active k), x1 slabs (active j,
// k).  A position names a cell (when inside the cell box) and the three lower
// faces of that cell.
__host__ __device__ __forceinline__ void shell_entry(const Geo& g, int64_t t64, int& i, int& j, int& k) {
  // 32-bit unsigned index arithmetic: a block's face box holds fewer than
  // 2^31 entries (checked when the block is created)
  const unsigned t = (unsigned)t64;
  const unsigned F1 = (unsigned)g.F1, F2 = (unsigned)g.F2;
  const unsigned nz = (unsigned)(g.F3 - g.n3) * F2 * F1;
  const unsigned ny = (unsigned)g.n3 * (F2 - (unsigned)g.n2) * F1;
  if (t < nz) {
    i = (int)(t % F1);
    const unsigned r = t / F1;
    j = (int)(r % F2);
    const int q = (int)(r / F2);
    k = q < g.ng ? q : q + g.n3;
  } else if (t < nz + ny) {
    const unsigned u = t - nz;
    i = (int)(u % F1);
    const unsigned r = u / F1, W = F2 - (unsigned)g.n2;
    const int q = (int)(r % W);
    j = q < g.ng ? q : q + g.n2;
    k = g.ng + (int)(r / W);
  } else {
    const unsigned u = t - nz - ny, W = F1 - (unsigned)g.n1;
    const int q = (int)(u % W);
    i = q < g.ng ? q : q + g.n1;
    const unsigned r = u / W;
    j = g.ng + (int)(r % (unsigned)g.n2);
    k = g.ng + (int)(r / (unsigned)g.n2);
  }
}

// The next block (+1) along direction D from block b of a coupled mesh,
// periodic over the mesh; b itself when blocks are their own periodic
// neighbours.
template <int D>
__host__ __device__ __forceinline__ int next_block(const Geo& g, int b) {
  const int m0 = g.mesh[0], m1 = g.mesh[1], m2 = g.mesh[2];
  if (m0 <= 0 || m1 <= 0 || m2 <= 0) return b;
  if (D == 0) return (b % m0 == m0 - 1) ? b - (m0 - 1) : b + 1;
  if (D == 1) return ((b / m0) % m1 == m1 - 1) ? b - (m1 - 1) * m0 : b + m0;
  return (b / (m0 * m1) == m2 - 1) ? b - (m2 - 1) * m0 * m1 : b + m0 * m1;
}

}  // namespace athmhd
