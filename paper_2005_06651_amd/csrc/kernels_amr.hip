// Level operators of block refinement (Sec. 2.1.5) on a box: restriction of
// fine cells [f, f + 2 h) of a fine block onto coarse cells [c, c + h) of a
// coarse block, and prolongation the other way (stored indices, ghost zones
// included).  Both blocks have the same shape (n1 x n2 x n3 active cells, ng
// ghosts, 5 + ns cell arrays); the fine cells are half as wide.  An octant
// (o1, o2, o3) of a coarse parent is the box f = ng, c = ng + o_d n_d / 2,
// h = n / 2; boxes in ghost zones serve the coarse buffers and ghost-zone
// prolongation between levels.  The host checks every box against the
// stored ranges before a launch.
//
// One thread per coarse cell of the box (plus one layer beyond its upper
// side for the faces there).  These run once per refinement or derefinement
// of a block, not per step: plain HBM-bound kernels, rows of threads along x1
// so that the fine reads and writes of neighbouring threads are contiguous.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace athmhd {
namespace {

constexpr int kAmrThreads = 256;

struct OctArgs {
  Geo g;
  int h[3];     // box extent in coarse cells
  int cl[3];    // first coarse cell of the box (stored index)
  int fl[3];    // first fine cell of the box (stored index)
  int per_xcd;  // workgroups per XCD: ceil(workgroups / 8)
  int keep;     // prolongation: bit 2 d + S keeps the fine faces on side S of the box along d
  double gm1;     // gamma - 1
  double pfloor;  // pressure floor of the refined cells (prolongation; 0: off)
  int* bad;       // floor activations counted with add_floor_count
};

// Thread index in the box's point order, XCD-aware: workgroup b runs on
// XCD b mod 8, so logical workgroup (b mod 8) per_xcd + b / 8 gives each XCD
// one contiguous run of rows and planes, and the neighbour rows and planes a
// thread reads sit in that XCD's L2.  Launched with 8 per_xcd workgroups.
__device__ __forceinline__ int oct_thread(const OctArgs& A) {
  const int b = blockIdx.x;
  return ((b % 8) * A.per_xcd + b / 8) * kAmrThreads + threadIdx.x;
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

// flat index of the cell / face at p = (x1, x2, x3)
__device__ __forceinline__ int cidx(const Geo& g, const int p[3]) { return g.c(p[0], p[1], p[2]); }
__device__ __forceinline__ int fidx(const Geo& g, const int p[3]) { return g.f(p[0], p[1], p[2]); }

// Restriction: volume average of the 8 fine cells of each coarse cell (every
// cell array), area average of the 4 fine faces on each coarse face of the
// box, upper faces included.
__global__ void __launch_bounds__(kAmrThreads)
    k_restrict(OctArgs A, const double* __restrict__ fc, const double* __restrict__ fb, double* __restrict__ cc,
               double* __restrict__ cb) {
  const Geo& g = A.g;
  const int e1 = A.h[0] + 1, e2 = A.h[1] + 1, e3 = A.h[2] + 1;
  const int t = oct_thread(A);
  if (t >= e1 * e2 * e3) return;
  const int q[3] = {t % e1, (t / e1) % e2, t / (e1 * e2)};
  const bool cell = q[0] < A.h[0] && q[1] < A.h[1] && q[2] < A.h[2];
  const int C[3] = {A.cl[0] + q[0], A.cl[1] + q[1], A.cl[2] + q[2]};
  const int F[3] = {A.fl[0] + 2 * q[0], A.fl[1] + 2 * q[1], A.fl[2] + 2 * q[2]};
  if (cell) {
    const int nv = 5 + g.ns;
    for (int v = 0; v < nv; ++v) {
      const double* src = fc + v * g.cvar;
      double s = 0.0;
      for (int s3 = 0; s3 < 2; ++s3)
        for (int s2 = 0; s2 < 2; ++s2)
          for (int s1 = 0; s1 < 2; ++s1) s += src[g.c(F[0] + s1, F[1] + s2, F[2] + s3)];
      cc[v * g.cvar + cidx(g, C)] = s / 8.0;
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    if (q[t1] >= A.h[t1] || q[t2] >= A.h[t2]) continue;
    const double* src = fb + d * g.fvar;
    double s = 0.0;
    for (int u = 0; u < 2; ++u)
      for (int w = 0; w < 2; ++w) {
        int p[3];
        p[d] = F[d];
        p[t1] = F[t1] + u;
        p[t2] = F[t2] + w;
        s += src[fidx(g, p)];
      }
    cb[d * g.fvar + fidx(g, C)] = s / 4.0;
  }
}

// The 4 fine values of the coarse face of component d at coarse index C:
// the face value plus the minmod-limited slopes along its two transverse
// directions (t1, t2) = (d + 1, d + 2) times the quarter offsets, out[p][q]
// with p the half along t1, q the half along t2.
__device__ __forceinline__ void split_face(const Geo& g, const double* cb, int d, const int C[3], double out[2][2]) {
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const double* b = cb + d * g.fvar;
  const double B = b[fidx(g, C)];
  double sl[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int t = e == 0 ? t1 : t2;
    int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
    m[t] -= 1;
    p[t] += 1;
    sl[e] = minmod(B - b[fidx(g, m)], b[fidx(g, p)] - B);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) out[p][q] = B + 0.25 * ((2 * p - 1) * sl[0] + (2 * q - 1) * sl[1]);
}

// Prolongation.  Cells: U_C plus the minmod-limited slope along each
// direction times the child's offset +-1/4.  Faces: every coarse face of the
// box split into 4 by split_face; the 12 faces inside each coarse cell in
// closed form.  Those are the one solution of Toth & Roe's conditions (every
// fine cell has the coarse cell's divergence; the curl at each of the 6
// interior edges equals the mean of the tangential differences on the two
// outer faces parallel to it).  Solved once by hand, with O_d[S][p][q] the
// outer fine value of component d on side S in {0, 1} and halves (p, q) along
// (d + 1, d + 2), s(x) = 2 x - 1, and w = 3/16 for r equal to the face's own
// half, 1/16 otherwise:
//   B_d(p, q) = (O_d[0][p][q] + O_d[1][p][q]) / 2
//             + sum_{S,i,r} s(S) s(i) [ w(r, q) O_{d+1}[S][r][i] + w(r, p) O_{d+2}[S][i][r] ]
// (component d + 1 has halves along (d + 2, d), component d + 2 along
// (d, d + 1); i is the half along d).  Each cell thread recomputes the
// splits of its upper faces; only the thread that owns a face as its lower
// face writes it, so every fine face is written once.
// With a pressure floor, every child whose pressure (from its prolonged U and
// the mean of its two bounding fine faces, all in this thread's registers) is
// below it gets E raised to give the floor; rho and M are unchanged.
// PRIM: the cells are prolonged in primitive variables instead -- the coarse
// cell and its 6 neighbours converted to (rho, v, P, C_i) with their own
// cell-centred fields, the primitives prolonged, each child converted back
// with the cell-centred field of its fine faces (no floor then: P itself is
// prolonged, so it stays positive).

// Primitives (rho, v1, v2, v3, P) of coarse cell P from its U and the mean of
// its two stored bounding faces along each direction.
__device__ __forceinline__ void coarse_prim(const Geo& g, double gm1, const double* cc, const double* cb,
                                            const int P[3], double w[5]) {
  const int q = cidx(g, P);
  double b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int up[3] = {P[0], P[1], P[2]};
    up[d] += 1;
    b[d] = 0.5 * (cb[d * g.fvar + fidx(g, P)] + cb[d * g.fvar + fidx(g, up)]);
  }
  const double rho = cc[q];
  const double v1 = cc[g.cvar + q] / rho, v2 = cc[2 * g.cvar + q] / rho, v3 = cc[3 * g.cvar + q] / rho;
  const double kin = 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3);
  const double mag = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  w[0] = rho;
  w[1] = v1;
  w[2] = v2;
  w[3] = v3;
  w[4] = gm1 * (cc[4 * g.cvar + q] - kin - mag);
}

// Cell-centred field of child (s1, s2, s3) from the outer (O) and interior
// (Bi) fine faces of its coarse cell; component d's halves run along
// (d + 1, d + 2).
__device__ __forceinline__ void child_field(const double (&O)[3][2][2][2], const double (&Bi)[3][2][2], int s1,
                                            int s2, int s3, double b[3]) {
  b[0] = 0.5 * ((s1 ? Bi[0][s2][s3] : O[0][0][s2][s3]) + (s1 ? O[0][1][s2][s3] : Bi[0][s2][s3]));
  b[1] = 0.5 * ((s2 ? Bi[1][s3][s1] : O[1][0][s3][s1]) + (s2 ? O[1][1][s3][s1] : Bi[1][s3][s1]));
  b[2] = 0.5 * ((s3 ? Bi[2][s1][s2] : O[2][0][s1][s2]) + (s3 ? O[2][1][s1][s2] : Bi[2][s1][s2]));
}

template <bool FLOOR, bool PRIM>
__global__ void __launch_bounds__(kAmrThreads)
    k_prolong(OctArgs A, const double* __restrict__ cc, const double* __restrict__ cb, double* __restrict__ fc,
              double* __restrict__ fb) {
  const Geo& g = A.g;
  const int e1 = A.h[0] + 1, e2 = A.h[1] + 1, e3 = A.h[2] + 1;
  const int t = oct_thread(A);
  if (t >= e1 * e2 * e3) return;
  const int q[3] = {t % e1, (t / e1) % e2, t / (e1 * e2)};
  const bool cell = q[0] < A.h[0] && q[1] < A.h[1] && q[2] < A.h[2];
  const int C[3] = {A.cl[0] + q[0], A.cl[1] + q[1], A.cl[2] + q[2]};
  const int F[3] = {A.fl[0] + 2 * q[0], A.fl[1] + 2 * q[1], A.fl[2] + 2 * q[2]};

  if (cell && !PRIM) {
    const int nv = 5 + g.ns;
    for (int v = 0; v < nv; ++v) {
      const double* src = cc + v * g.cvar;
      const double u0 = src[cidx(g, C)];
      double sl[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
        m[d] -= 1;
        p[d] += 1;
        sl[d] = minmod(u0 - src[cidx(g, m)], src[cidx(g, p)] - u0);
      }
      double* dst = fc + v * g.cvar;
#pragma unroll
      for (int s3 = 0; s3 < 2; ++s3)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
          for (int s1 = 0; s1 < 2; ++s1)
            dst[g.c(F[0] + s1, F[1] + s2, F[2] + s3)] =
                u0 + 0.25 * ((2 * s1 - 1) * sl[0] + (2 * s2 - 1) * sl[1] + (2 * s3 - 1) * sl[2]);
    }
  }

  // outer faces: O[d][S][p][q]; the lower one (S = 0) is this thread's own.
  // Faces on a kept side of the box are read, never written; all others are
  // split from the coarse face, and only their owner writes them.
  double O[3][2][2][2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    if (q[t1] >= A.h[t1] || q[t2] >= A.h[t2]) continue;
    double* dst = fb + d * g.fvar;
    const bool keep_lo = (q[d] == 0 && ((A.keep >> (2 * d)) & 1)) || (q[d] == A.h[d] && ((A.keep >> (2 * d + 1)) & 1));
    if (keep_lo) {
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          int x[3];
          x[d] = F[d];
          x[t1] = F[t1] + p;
          x[t2] = F[t2] + r;
          O[d][0][p][r] = dst[fidx(g, x)];
        }
    } else {
      split_face(g, cb, d, C, O[d][0]);
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          int x[3];
          x[d] = F[d];
          x[t1] = F[t1] + p;
          x[t2] = F[t2] + r;
          dst[fidx(g, x)] = O[d][0][p][r];
        }
    }
    if (cell) {
      if (q[d] == A.h[d] - 1 && ((A.keep >> (2 * d + 1)) & 1)) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            int x[3];
            x[d] = F[d] + 2;
            x[t1] = F[t1] + p;
            x[t2] = F[t2] + r;
            O[d][1][p][r] = dst[fidx(g, x)];
          }
      } else {
        int Cu[3] = {C[0], C[1], C[2]};
        Cu[d] += 1;
        split_face(g, cb, d, Cu, O[d][1]);
      }
    }
  }
  if (!cell) return;

  double Bi[3][2][2];  // interior faces, halves as for O
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    double* dst = fb + d * g.fvar;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        double v = 0.5 * (O[d][0][p][r] + O[d][1][p][r]);
        double cross = 0.0;
#pragma unroll
        for (int S = 0; S < 2; ++S)
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const double sg = (S == i) ? 1.0 : -1.0;  // s(S) s(i)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const double w1 = (k == r) ? 0.1875 : 0.0625;
              const double w2 = (k == p) ? 0.1875 : 0.0625;
              cross += sg * (w1 * O[d1][S][k][i] + w2 * O[d2][S][i][k]);
            }
          }
        int x[3];
        x[d] = F[d] + 1;
        x[d1] = F[d1] + p;
        x[d2] = F[d2] + r;
        Bi[d][p][r] = v + cross;
        dst[fidx(g, x)] = Bi[d][p][r];
      }
  }
  const int64_t cv = g.cvar;
  if (PRIM) {
    // slopes of the 5 MHD primitives, one direction at a time
    double w0[5], sl[5][3];
    coarse_prim(g, A.gm1, cc, cb, C, w0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
      m[d] -= 1;
      p[d] += 1;
      double wm[5], wp[5];
      coarse_prim(g, A.gm1, cc, cb, m, wm);
      coarse_prim(g, A.gm1, cc, cb, p, wp);
#pragma unroll
      for (int v = 0; v < 5; ++v) sl[v][d] = minmod(w0[v] - wm[v], wp[v] - w0[v]);
    }
    double rho_c[8];
#pragma unroll
    for (int s3 = 0; s3 < 2; ++s3)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1) {
          double w[5];
#pragma unroll
          for (int v = 0; v < 5; ++v)
            w[v] = w0[v] + 0.25 * ((2 * s1 - 1) * sl[v][0] + (2 * s2 - 1) * sl[v][1] + (2 * s3 - 1) * sl[v][2]);
          double b[3];
          child_field(O, Bi, s1, s2, s3, b);
          const int q0 = g.c(F[0] + s1, F[1] + s2, F[2] + s3);
          fc[q0] = w[0];
          fc[cv + q0] = w[0] * w[1];
          fc[2 * cv + q0] = w[0] * w[2];
          fc[3 * cv + q0] = w[0] * w[3];
          fc[4 * cv + q0] = w[4] / A.gm1 + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) +
                            0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
          rho_c[(s3 * 2 + s2) * 2 + s1] = w[0];
        }
    // passive scalars: C = (rho C) / rho prolonged, back as rho_child C
    const int nv = 5 + g.ns;
    const double r0 = cc[cidx(g, C)];
    for (int v = 5; v < nv; ++v) {
      const double* src = cc + v * cv;
      const double c0 = src[cidx(g, C)] / r0;
      double s[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int m[3] = {C[0], C[1], C[2]}, p[3] = {C[0], C[1], C[2]};
        m[d] -= 1;
        p[d] += 1;
        const double cm = src[cidx(g, m)] / cc[cidx(g, m)], cp = src[cidx(g, p)] / cc[cidx(g, p)];
        s[d] = minmod(c0 - cm, cp - c0);
      }
#pragma unroll
      for (int s3 = 0; s3 < 2; ++s3)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
          for (int s1 = 0; s1 < 2; ++s1)
            fc[v * cv + g.c(F[0] + s1, F[1] + s2, F[2] + s3)] =
                rho_c[(s3 * 2 + s2) * 2 + s1] *
                (c0 + 0.25 * ((2 * s1 - 1) * s[0] + (2 * s2 - 1) * s[1] + (2 * s3 - 1) * s[2]));
    }
  }
  if (!FLOOR) return;

  int hits = 0;
#pragma unroll
  for (int s3 = 0; s3 < 2; ++s3)
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
      for (int s1 = 0; s1 < 2; ++s1) {
        double bc[3];
        child_field(O, Bi, s1, s2, s3, bc);
        const double bx = bc[0], by = bc[1], bz = bc[2];
        const int q0 = g.c(F[0] + s1, F[1] + s2, F[2] + s3);
        const double rho = fc[q0], m1 = fc[cv + q0], m2 = fc[2 * cv + q0], m3 = fc[3 * cv + q0];
        const double e = fc[4 * cv + q0];
        const double kin = 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / rho;
        const double mag = 0.5 * (bx * bx + by * by + bz * bz);
        if (!(A.gm1 * (e - kin - mag) >= A.pfloor)) {
          fc[4 * cv + q0] = A.pfloor / A.gm1 + kin + mag;
          ++hits;
        }
      }
  if (hits) add_floor_count(A.bad, (unsigned long long)hits);
}

OctArgs box_args(const Geo& g, const int flo[3], const int clo[3], const int ext[3]) {
  OctArgs A;
  A.g = g;
  A.gm1 = 0.0;
  A.pfloor = 0.0;
  A.bad = nullptr;
  A.keep = 0;
  for (int d = 0; d < 3; ++d) {
    A.h[d] = ext[d];
    A.cl[d] = clo[d];
    A.fl[d] = flo[d];
  }
  const long pts = (long)(A.h[0] + 1) * (A.h[1] + 1) * (A.h[2] + 1);
  const long wgs = (pts + kAmrThreads - 1) / kAmrThreads;
  A.per_xcd = (int)((wgs + 7) / 8);
  return A;
}

int grid_of(const OctArgs& A) { return 8 * A.per_xcd; }

}  // namespace

hipError_t launch_restrict(const Geo& g, const int flo[3], const int clo[3], const int ext[3], const double* fc,
                           const double* fb, double* cc, double* cb, hipStream_t s) {
  const OctArgs A = box_args(g, flo, clo, ext);
  hipLaunchKernelGGL(k_restrict, dim3(grid_of(A)), dim3(kAmrThreads), 0, s, A, fc, fb, cc, cb);
  return hipGetLastError();
}

hipError_t launch_prolong(const Geo& g, const int flo[3], const int clo[3], const int ext[3], const double* cc,
                          const double* cb, double* fc, double* fb, bool primitive, int keep, double gamma, double pfloor,
                          int* bad, hipStream_t s) {
  OctArgs A = box_args(g, flo, clo, ext);
  A.keep = keep;
  A.gm1 = gamma - 1.0;
  if (!primitive && pfloor > 0.0 && bad) {
    A.pfloor = pfloor;
    A.bad = bad;
  }
  const dim3 grid(grid_of(A)), block(kAmrThreads);
  if (primitive)
    hipLaunchKernelGGL((k_prolong<false, true>), grid, block, 0, s, A, cc, cb, fc, fb);
  else if (A.pfloor > 0.0)
    hipLaunchKernelGGL((k_prolong<true, false>), grid, block, 0, s, A, cc, cb, fc, fb);
  else
    hipLaunchKernelGGL((k_prolong<false, false>), grid, block, 0, s, A, cc, cb, fc, fb);
  return hipGetLastError();
}

}  // namespace athmhd
