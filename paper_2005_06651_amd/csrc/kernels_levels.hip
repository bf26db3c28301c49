// kernels_levels.hip -- the two kernels of a stage that couple the levels of
// a two-level composite (block 0 coarse, blocks 1 + a + 2b + 4c fine, the
// fine region below the coarse block along x1, periodic domain) between the
// flux computation and the update of the unfused pipeline:
//   * flux correction (Sec. 2.1.4): the coarse flux through each face of the
//     two coarse-fine interfaces becomes the mean of the four fine fluxes
//     through it (area integral);
//   * EMF correction (Sec. 2.1.4, Eq. emfcorr): each coarse E2, E3 on an
//     interface plane becomes the mean of the two fine EMFs along it (line
//     integral);
// and the update of the interface faces the fine blocks own (x1 = X).
// Plain HBM-bound kernels over the interface planes.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace athmhd {
namespace {

constexpr int kLevelThreads = 256;

// fine block offset (a + 2b + 4c, relative to the first fine block) and
// stored index of global fine index gl along a direction of n cells per block
__device__ __forceinline__ void fine_pos(int gl, int n, int ng, int& blk, int& idx) {
  const int len = 2 * n;
  gl = gl < 0 ? gl + len : (gl >= len ? gl - len : gl);
  blk = gl >= n ? 1 : 0;
  idx = ng + gl - blk * n;
}

// One thread per (side, j, k) with j in [0, n2], k in [0, n3] (relative to the
// first active index): the four fluxes of face (j, k), the E2 edge over cell j
// at x3 face k, and the E3 edge over cell k at x2 face j, as far as they exist.
__global__ void __launch_bounds__(kLevelThreads)
    k_level_correct(Geo g, double* __restrict__ cface0, double* __restrict__ cedge,
                    const double* __restrict__ fface0, const double* __restrict__ fedge) {
  const int t = blockIdx.x * kLevelThreads + threadIdx.x;
  const int nj = g.n2 + 1, nk = g.n3 + 1;
  if (t >= 2 * nj * nk) return;
  const int side = t / (nj * nk);
  const int r = t - side * nj * nk;
  const int jr = r % nj, kr = r / nj;
  const int ng = g.ng;
  const int ci = side == 0 ? ng : ng + g.n1;  // coarse x1 face / edge plane
  const int fi = side == 0 ? ng + g.n1 : ng;  // the same plane in the fine blocks
  const int fa = side == 0 ? 1 : 0;
  const int j = ng + jr, k = ng + kr;
  if (jr < g.n2 && kr < g.n3) {
    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int dk = 0; dk < 2; ++dk)
      for (int dj = 0; dj < 2; ++dj) {
        int bj, jj, bk, kk;
        fine_pos(2 * jr + dj, g.n2, ng, bj, jj);
        fine_pos(2 * kr + dk, g.n3, ng, bk, kk);
        const double* F = fface0 + (int64_t)(fa + 2 * bj + 4 * bk) * 8 * g.fvar;
        const int f = g.f(fi, jj, kk);
#pragma unroll
        for (int v = 0; v < 5; ++v) sum[v] += F[v * g.fvar + f];
      }
#pragma unroll
    for (int v = 0; v < 5; ++v) cface0[v * g.fvar + g.f(ci, j, k)] = 0.25 * sum[v];
  }
  if (jr < g.n2) {  // E2 over coarse cell j at the x3 face k (k up to ng + n3)
    double sum = 0.0;
    for (int dj = 0; dj < 2; ++dj) {
      int bj, jj, bk, kk;
      fine_pos(2 * jr + dj, g.n2, ng, bj, jj);
      fine_pos(2 * kr, g.n3, ng, bk, kk);
      sum += fedge[(int64_t)(fa + 2 * bj + 4 * bk) * 3 * g.fvar + 1 * g.fvar + g.f(fi, jj, kk)];
    }
    cedge[1 * g.fvar + g.f(ci, j, k)] = 0.5 * sum;
  }
  if (kr < g.n3) {  // E3 over coarse cell k at the x2 face j (j up to ng + n2)
    double sum = 0.0;
    for (int dk = 0; dk < 2; ++dk) {
      int bj, jj, bk, kk;
      fine_pos(2 * jr, g.n2, ng, bj, jj);
      fine_pos(2 * kr + dk, g.n3, ng, bk, kk);
      sum += fedge[(int64_t)(fa + 2 * bj + 4 * bk) * 3 * g.fvar + 2 * g.fvar + g.f(fi, jj, kk)];
    }
    cedge[2 * g.fvar + g.f(ci, j, k)] = 0.5 * sum;
  }
}

// One thread per (fine block with a = 1, j, k): the x1 face at i = ng + n1.
__global__ void __launch_bounds__(kLevelThreads)
    k_level_fine_faces(Geo g, StageCoef cf, const double* dt_dev, double beta, const double* __restrict__ xb,
                       const double* unb, double* outb, const double* __restrict__ fedge) {
  const int t = blockIdx.x * kLevelThreads + threadIdx.x;
  const int per = g.n2 * g.n3;
  if (t >= 4 * per) return;
  const int q = 2 * (t / per) + 1;  // fine blocks a = 1: offsets 1, 3, 5, 7
  const int r = t % per;
  const int j = g.ng + r % g.n2, k = g.ng + r / g.n2;
  const int fc = g.f(g.ng + g.n1, j, k);
  const int s2 = g.F1, s3 = g.F1 * g.F2;
  const double* E2 = fedge + (int64_t)q * 3 * g.fvar + g.fvar;
  const double* E3 = E2 + g.fvar;
  const double bdt = dt_dev ? beta * *dt_dev : cf.bdt;
  // dB1 = -[(E3(j+1) - E3(j))/dx2 - (E2(k+1) - E2(k))/dx3]
  const double c1 = (E3[fc + s2] - E3[fc]) * (1.0 / g.dx2) - (E2[fc + s3] - E2[fc]) * (1.0 / g.dx3);
  const int64_t o = (int64_t)q * g.fblock + fc;
  outb[o] = cf.g0 * xb[o] + cf.g1 * unb[o] - bdt * c1;
}

}  // namespace

hipError_t launch_level_correct(const Geo& gc, UnfusedScratch& coarse, const UnfusedScratch& fine, hipStream_t s) {
  const int n = 2 * (gc.n2 + 1) * (gc.n3 + 1);
  hipLaunchKernelGGL(k_level_correct, dim3((n + kLevelThreads - 1) / kLevelThreads), dim3(kLevelThreads), 0, s, gc,
                     coarse.face[0], coarse.edge, fine.face[0], fine.edge);
  return hipGetLastError();
}

hipError_t launch_level_fine_faces(const Geo& gf, const double* xb, const double* unb, double* outb, StageCoef coef,
                                   const double* dt_dev, double beta, const UnfusedScratch& fine, hipStream_t s) {
  const int n = 4 * gf.n2 * gf.n3;
  hipLaunchKernelGGL(k_level_fine_faces, dim3((n + kLevelThreads - 1) / kLevelThreads), dim3(kLevelThreads), 0, s, gf,
                     coef, dt_dev, beta, xb, unb, outb, fine.edge);
  return hipGetLastError();
}

}  // namespace athmhd
