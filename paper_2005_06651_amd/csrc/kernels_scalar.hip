// kernels_scalar.hip -- passive scalars (Sec. 3.3.x, Eq. (passive_scalars)):
// the mass rho C_i of each scalar obeys the continuity equation with the
// specific density C_i carried along.  C_i is reconstructed like the other
// primitives (DC / PLM / PPM, Sec. 3.2.1) and moves with the face mass flux
// F_rho of the stage's Riemann solves, taken from the upwind side.  The fused
// stage kernel stores F_rho on the lower faces of the active cells; two
// HBM-bound kernels then finish the stage for any number of scalars:
//   k_scalar_prim    C_i = (rho C_i) / rho of the stage input on the active
//                    cells, rho floored as in the MHD primitives when floors
//                    are on;
//   k_scalar_update  flux difference of rho C_i and the 2S stage update
//                    (Eq. (rk-2s)), one thread per active cell, x1 fastest so
//                    that lines along x1 are coalesced and the x2 / x3
//                    neighbours come from L2.
#include "common.hpp"
#include "kernels.hpp"
#include "mhd_math.hpp"

namespace athmhd {

namespace {

constexpr int kScThreads = 256;

// Stored index of position idx along a direction of a periodic block with n
// active cells.  NEAR: the stencil reaches less than a block past the active
// range, so one correction step finds the periodic image.
template <bool NEAR>
__device__ __forceinline__ int wrap_sc(int idx, int n, int ng) {
  if (!NEAR) return wrap_index(idx, n, ng);
  return idx < ng ? idx + n : (idx >= ng + n ? idx - n : idx);
}

template <bool FL>
__global__ void __launch_bounds__(kScThreads) k_scalar_prim(Geo g, Floors fl, const double* __restrict__ xc,
                                                            double* __restrict__ cs) {
  const int t = blockIdx.x * kScThreads + threadIdx.x;
  if (t >= g.n1 * g.n2 * g.n3) return;
  const int i = g.ng + t % g.n1, r = t / g.n1, j = g.ng + r % g.n2, k = g.ng + r / g.n2;
  const int q = g.c(i, j, k);
  const double* x = xc + (int64_t)blockIdx.y * g.cblock;
  double* c = cs + (int64_t)blockIdx.y * g.ns * g.cvar;
  double rho = x[q];
  if (FL && isfinite(rho) && isfinite(x[4 * g.cvar + q]) && !(rho >= fl.d)) rho = fl.d;
  for (int v = 0; v < g.ns; ++v) c[v * g.cvar + q] = x[(5 + v) * g.cvar + q] / rho;
}

struct ScalarArgs {
  Geo g;
  StageCoef cf;
  const double* dt_dev;  // optional device copy of dt: bdt = beta * (*dt_dev)
  double beta;
  const double* xc;      // stage input (read where g0 != 0)
  const double* unc;     // U^n
  double* oc;            // stage output
  const double* fm;      // face mass fluxes, 3 face arrays per block
  const double* cs;     // C_i on the active cells, ns cell arrays per block
};

template <int RECON, bool NEAR>
__global__ void __launch_bounds__(kScThreads) k_scalar_update(ScalarArgs a) {
  const Geo& g = a.g;
  constexpr int LA = RECON;       // reconstruction half-width: DC 0, PLM 1, PPM 2
  constexpr int W = 2 * LA + 3;   // cells c-LA-1 .. c+LA+1: the edges of c-1, c, c+1
  const int t = blockIdx.x * kScThreads + threadIdx.x;
  if (t >= g.n1 * g.n2 * g.n3) return;
  const int i = g.ng + t % g.n1, r = t / g.n1, j = g.ng + r % g.n2, k = g.ng + r / g.n2;
  const int64_t b = blockIdx.y;
  const double* __restrict__ fm = a.fm + b * 3 * g.fvar;
  const double* __restrict__ cs = a.cs + b * g.ns * g.cvar;
  const double bdt = a.dt_dev ? a.beta * *a.dt_dev : a.cf.bdt;
  int si[W], sj[W], sk[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    si[o] = wrap_sc<NEAR>(i + o - LA - 1, g.n1, g.ng);
    sj[o] = wrap_sc<NEAR>(j + o - LA - 1, g.n2, g.ng);
    sk[o] = wrap_sc<NEAR>(k + o - LA - 1, g.n3, g.ng);
  }
  // mass fluxes through the lower and upper faces along each direction; the
  // upper face of the last cell is the periodic image of the first lower face
  double flo[3], fup[3];
  flo[0] = fm[g.f(i, j, k)];
  fup[0] = fm[g.f(si[LA + 2], j, k)];
  flo[1] = fm[g.fvar + g.f(i, j, k)];
  fup[1] = fm[g.fvar + g.f(i, sj[LA + 2], k)];
  flo[2] = fm[2 * g.fvar + g.f(i, j, k)];
  fup[2] = fm[2 * g.fvar + g.f(i, j, sk[LA + 2])];
  const double inv[3] = {1.0 / g.dx1, 1.0 / g.dx2, 1.0 / g.dx3};
  const int q = g.c(i, j, k);
  for (int v = 0; v < g.ns; ++v) {
    const double* __restrict__ c = cs + v * g.cvar;
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double line[W];
#pragma unroll
      for (int o = 0; o < W; ++o)
        line[o] = c[d == 0 ? g.c(si[o], j, k) : (d == 1 ? g.c(i, sj[o], k) : g.c(i, j, sk[o]))];
      double lm, rm, l0, r0, lp, rp;
      cell_edges<RECON>(line, lm, rm);      // cell c-1
      cell_edges<RECON>(line + 1, l0, r0);  // cell c
      cell_edges<RECON>(line + 2, lp, rp);  // cell c+1
      // face c-1/2 has left state rm, right state l0; face c+1/2 has r0, lp
      const double flux_lo = flo[d] >= 0.0 ? flo[d] * rm : flo[d] * l0;
      const double flux_up = fup[d] >= 0.0 ? fup[d] * r0 : fup[d] * lp;
      sum += (flux_up - flux_lo) * inv[d];
    }
    const int64_t e = b * g.cblock + (5 + v) * g.cvar + q;
    double out = a.cf.g1 * a.unc[e];
    if (a.cf.g0 != 0.0) out += a.cf.g0 * a.xc[e];
    a.oc[e] = out - bdt * sum;
  }
}

template <int RECON>
void launch_update(const ScalarArgs& sa, bool near, dim3 grid, hipStream_t s) {
  if (near) hipLaunchKernelGGL((k_scalar_update<RECON, true>), grid, dim3(kScThreads), 0, s, sa);
  else hipLaunchKernelGGL((k_scalar_update<RECON, false>), grid, dim3(kScThreads), 0, s, sa);
}

}  // namespace

hipError_t launch_scalar_stage(const Geo& g, int recon, const double* xc, const double* unc, double* outc,
                               const double* fm, double* cs, StageCoef coef, const double* dt_dev, double beta,
                               int nb, Floors fl, hipStream_t s) {
  if (g.ns <= 0) return hipSuccess;
  const int64_t na = (int64_t)g.n1 * g.n2 * g.n3;
  const dim3 grid((unsigned)((na + kScThreads - 1) / kScThreads), (unsigned)nb);
  if (fl.on()) hipLaunchKernelGGL((k_scalar_prim<true>), grid, dim3(kScThreads), 0, s, g, fl, xc, cs);
  else hipLaunchKernelGGL((k_scalar_prim<false>), grid, dim3(kScThreads), 0, s, g, fl, xc, cs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ScalarArgs sa{g, coef, dt_dev, beta, xc, unc, outc, fm, cs};
  // one correction step finds every periodic image when each direction has
  // more active cells than the stencil reaches past the block
  const int reach = recon + 2;
  const bool near = g.n1 >= reach && g.n2 >= reach && g.n3 >= reach;
  if (recon == 0) launch_update<0>(sa, near, grid, s);
  else if (recon == 1) launch_update<1>(sa, near, grid, s);
  else launch_update<2>(sa, near, grid, s);
  return hipGetLastError();
}

}  // namespace athmhd
