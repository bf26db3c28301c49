// abi.hip -- host side of the C ABI declared in include/athmhd.h: argument
// validation (entirely before any HIP call), device buffers, the stage driver
// of the 2S integrators (Eq. (rk-2s), Sec. 3.2.3) and error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/athmhd.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace athmhd;

struct athmhd_s {
  athmhd_config cfg;
  Geo g;
  int nbmax = 0;
  int device = 0;
  double* reg[2] = {nullptr, nullptr};  // two stage registers (cons followed by bface), nbmax blocks each
  UnfusedScratch scr{};
  double* scratch_base = nullptr;
  unsigned long long* d_dt = nullptr;   // running min of dx/(|v|+cf), bit pattern
  int* d_bad = nullptr;                 // non-physical cells met since the last newdt
  void* h_pinned = nullptr;             // 16 bytes of pinned host memory for newdt
  int kz = 0;                           // x3 planes per fused workgroup (0: default)
  int occ = 2;                          // register target of the fused kernel (waves per SIMD)
  bool profiling = false;
  std::vector<hipEvent_t> events;       // (start, stop) pairs around stage kernels
  std::string err;
};

namespace {

thread_local std::string g_create_err;

int fail(athmhd_t h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(athmhd_t h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  else g_create_err = buf;
  return code;
}

int hip_fail(athmhd_t h, hipError_t e, const char* what) {
  return fail(h, ATHMHD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Coefficients of the supported integrators (Sec. 3.2.3).  All have
// delta_s = 0 for s > 0, so the second register u^(1) always equals U^n and
// the caller's buffers serve as it.
struct Scheme {
  int nstage;
  double g0[3], g1[3], beta[3];
};

Scheme scheme_of(int integ) {
  switch (integ) {
    case ATHMHD_RK1: return {1, {0, 0, 0}, {1, 0, 0}, {1.0, 0, 0}};
    case ATHMHD_VL2: return {2, {0, 0, 0}, {1, 1, 0}, {0.5, 1.0, 0}};
    case ATHMHD_RK2: return {2, {0, 0.5, 0}, {1, 0.5, 0}, {1.0, 0.5, 0}};
    default: return {3, {0, 0.25, 2.0 / 3.0}, {1, 0.75, 1.0 / 3.0}, {1.0, 0.25, 2.0 / 3.0}};
  }
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v, int* bad, int clear_bad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *p = v;
    if (clear_bad) *bad = 0;
  }
}

int validate_cfg(const athmhd_config* c) {
  if (!c) return fail(nullptr, ATHMHD_EINVAL, "config is NULL");
  if (c->n1 < 1 || c->n2 < 1 || c->n3 < 1)
    return fail(nullptr, ATHMHD_EINVAL, "block dims must be >= 1 (got %d %d %d)", c->n1, c->n2, c->n3);
  if (c->recon < ATHMHD_RECON_DC || c->recon > ATHMHD_RECON_PPM)
    return fail(nullptr, ATHMHD_EINVAL, "unknown reconstruction %d", c->recon);
  if (c->riemann != ATHMHD_RS_HLLE && c->riemann != ATHMHD_RS_HLLD)
    return fail(nullptr, ATHMHD_EINVAL, "unknown Riemann solver %d", c->riemann);
  if (c->integrator < ATHMHD_RK1 || c->integrator > ATHMHD_RK3)
    return fail(nullptr, ATHMHD_EINVAL, "unknown integrator %d", c->integrator);
  const int need = c->recon == ATHMHD_RECON_PPM ? 3 : 2;
  if (c->nghost < need || c->nghost > 8)
    return fail(nullptr, ATHMHD_EINVAL, "nghost must be in [%d, 8] for this reconstruction (got %d)", need,
                c->nghost);
  if (!(std::isfinite(c->gamma) && c->gamma > 1.0))
    return fail(nullptr, ATHMHD_EINVAL, "gamma must be finite and > 1 (got %g)", c->gamma);
  if (!finite_pos(c->dx1) || !finite_pos(c->dx2) || !finite_pos(c->dx3))
    return fail(nullptr, ATHMHD_EINVAL, "cell widths must be finite and > 0");
  if (!(std::isfinite(c->cfl) && c->cfl > 0.0 && c->cfl <= 1.0))
    return fail(nullptr, ATHMHD_EINVAL, "cfl must be in (0, 1] (got %g)", c->cfl);
  if (!(std::isfinite(c->ct_eps) && c->ct_eps >= 0.0))
    return fail(nullptr, ATHMHD_EINVAL, "ct_eps must be finite and >= 0 (got %g)", c->ct_eps);
  if (c->kernel_path != 0 && c->kernel_path != 1)
    return fail(nullptr, ATHMHD_EINVAL, "kernel_path must be 0 (fused) or 1 (unfused)");
  const double faces = (double)(c->n1 + 2 * c->nghost + 1) * (c->n2 + 2 * c->nghost + 1) * (c->n3 + 2 * c->nghost + 1);
  if (faces >= 2147483647.0) return fail(nullptr, ATHMHD_EINVAL, "block too large for 32-bit in-array indices");
  return ATHMHD_OK;
}

int check_call(athmhd_t h, const void* a, const void* b, int nb) {
  if (!h) return ATHMHD_EINVAL;
  if (!a || !b) return fail(h, ATHMHD_EINVAL, "NULL array argument");
  if (nb < 1 || nb > h->nbmax) return fail(h, ATHMHD_EINVAL, "nblocks %d outside [1, %d]", nb, h->nbmax);
  return ATHMHD_OK;
}

void drop_events(athmhd_t h) {
  for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
  h->events.clear();
}

// record one event of a (start, stop) pair when profiling
hipError_t mark(athmhd_t h, hipStream_t s) {
  if (!h->profiling) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreate(&ev);
  if (e != hipSuccess) return e;
  h->events.push_back(ev);
  return hipEventRecord(ev, s);
}

void free_all(athmhd_t h) {
  if (!h) return;
  drop_events(h);
  for (int r = 0; r < 2; ++r)
    if (h->reg[r]) (void)hipFree(h->reg[r]);
  if (h->scratch_base) (void)hipFree(h->scratch_base);
  if (h->d_dt) (void)hipFree(h->d_dt);
  if (h->d_bad) (void)hipFree(h->d_bad);
  if (h->h_pinned) (void)hipHostFree(h->h_pinned);
}

}  // namespace

extern "C" {

int athmhd_version(void) { return 100; }

int athmhd_create(const athmhd_config* cfg, int nblocks_max, athmhd_t* out) {
  if (!out) return fail(nullptr, ATHMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_cfg(cfg);
  if (rc != ATHMHD_OK) return rc;
  if (nblocks_max < 1) return fail(nullptr, ATHMHD_EINVAL, "nblocks_max must be >= 1");
  athmhd_t h = new (std::nothrow) athmhd_s();
  if (!h) return fail(nullptr, ATHMHD_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->g = make_geo(cfg->n1, cfg->n2, cfg->n3, cfg->nghost, cfg->dx1, cfg->dx2, cfg->dx3);
  h->nbmax = nblocks_max;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    rc = fail(nullptr, ATHMHD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    delete h;
    return rc;
  }
  const int64_t state = (h->g.cblock + h->g.fblock) * (int64_t)nblocks_max;
  const int64_t nscr =
      cfg->kernel_path == 1 ? (8 * h->g.cvar + 24 * h->g.fvar + 3 * h->g.fvar) * (int64_t)nblocks_max : 1;
  bool ok = hipMalloc(&h->reg[0], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->reg[1], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->scratch_base, nscr * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->d_dt, sizeof(unsigned long long)) == hipSuccess &&
            hipMalloc(&h->d_bad, sizeof(int)) == hipSuccess &&
            hipHostMalloc(&h->h_pinned, 16, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_ENOMEM, "device allocation of %.3f GB failed",
                (2.0 * state + nscr) * 8.0 / 1e9);
  }
  double* p = h->scratch_base;
  h->scr.w = p;
  p += 8 * h->g.cvar * nblocks_max;
  for (int d = 0; d < 3; ++d) {
    h->scr.face[d] = p;
    p += 8 * h->g.fvar * nblocks_max;
  }
  h->scr.edge = p;
  if (const char* kz = getenv("ATHMHD_KZ")) h->kz = atoi(kz);
  if (const char* oc = getenv("ATHMHD_OCC")) h->occ = atoi(oc) == 1 ? 1 : 2;
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, nullptr, h->d_dt, 0ull, h->d_bad, 1);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_EHIP, "initialisation: %s", hipGetErrorString(e));
  }
  *out = h;
  return ATHMHD_OK;
}

void athmhd_destroy(athmhd_t h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
}

const char* athmhd_last_error(athmhd_t h) { return h ? h->err.c_str() : g_create_err.c_str(); }

int athmhd_fill_ghosts(athmhd_t h, double* cons, double* bface, int nblocks, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  hipError_t e = launch_fill_ghosts(h->g, cons, bface, nblocks, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "fill_ghosts launch");
}

int athmhd_prim2cons(athmhd_t h, const double* prim, const double* bface, double* cons, int nblocks,
                     void* stream) {
  int rc = check_call(h, prim, bface, nblocks);
  if (rc) return rc;
  if (!cons) return fail(h, ATHMHD_EINVAL, "NULL cons");
  hipError_t e = launch_prim2cons(h->g, h->cfg.gamma, prim, bface, cons, nblocks, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "prim2cons launch");
}

int athmhd_step(athmhd_t h, double* cons, double* bface, double dt, int nblocks, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(h, ATHMHD_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->g;
  const Scheme sc = scheme_of(h->cfg.integrator);
  const int64_t coff = g.cblock * h->nbmax;  // bface of a register follows its cons
  const double* xc = cons;
  const double* xb = bface;
  hipError_t e;
  for (int st = 0; st < sc.nstage; ++st) {
    // ghosts of the stage input (the caller's U^n, or a register)
    if ((e = launch_fill_ghosts(g, const_cast<double*>(xc), const_cast<double*>(xb), nblocks, s)) != hipSuccess)
      return hip_fail(h, e, "fill_ghosts launch");
    const bool last = st == sc.nstage - 1;
    double* oc;
    double* ob;
    if (last && xc != cons) {
      oc = cons;
      ob = bface;
    } else {
      double* r = h->reg[st % 2];
      oc = r;
      ob = r + coff;
    }
    // the VL2 predictor always uses donor-cell fluxes (Sec. 3.2.3)
    const int recon = (h->cfg.integrator == ATHMHD_VL2 && st == 0) ? ATHMHD_RECON_DC : h->cfg.recon;
    StageCoef cf{sc.g0[st], sc.g1[st], sc.beta[st] * dt};
    if ((e = mark(h, s)) != hipSuccess) return hip_fail(h, e, "profiling event");
    if (h->cfg.kernel_path == 0)
      e = launch_stage_fused(g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc, xb, cons, bface, oc, ob, cf,
                             nblocks, h->kz, h->occ, h->d_bad, s);
    else
      e = launch_stage_unfused(g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc, xb, cons, bface, oc, ob,
                               cf, nblocks, h->scr, h->d_bad, s);
    if (e != hipSuccess) return hip_fail(h, e, "stage launch");
    if ((e = mark(h, s)) != hipSuccess) return hip_fail(h, e, "profiling event");
    xc = oc;
    xb = ob;
  }
  if (xc != cons) {  // single-stage scheme: result sits in a register
    for (int b = 0; b < nblocks; ++b) {
      if ((e = launch_copy(cons + b * g.cblock, xc + b * g.cblock, g.cblock, s)) != hipSuccess)
        return hip_fail(h, e, "copy launch");
      if ((e = launch_copy(bface + b * g.fblock, xb + b * g.fblock, g.fblock, s)) != hipSuccess)
        return hip_fail(h, e, "copy launch");
    }
  }
  if ((e = launch_fill_ghosts(g, cons, bface, nblocks, s)) != hipSuccess) return hip_fail(h, e, "fill_ghosts launch");
  return ATHMHD_OK;
}

int athmhd_newdt(athmhd_t h, const double* cons, const double* bface, int nblocks, double* dt_host, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (!dt_host) return fail(h, ATHMHD_EINVAL, "NULL dt_host");
  hipStream_t s = (hipStream_t)stream;
  const double inf = INFINITY;
  unsigned long long inf_bits;
  std::memcpy(&inf_bits, &inf, 8);
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dt, inf_bits, h->d_bad, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "newdt init launch");
  if ((e = launch_newdt(h->g, h->cfg.gamma, cons, bface, nblocks, h->d_dt, h->d_bad, s)) != hipSuccess)
    return hip_fail(h, e, "newdt launch");
  char* hp = (char*)h->h_pinned;
  if ((e = hipMemcpyAsync(hp, h->d_dt, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(hp + 8, h->d_bad, 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(h, e, "newdt copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "newdt synchronise");
  unsigned long long bits;
  int bad;
  std::memcpy(&bits, hp, 8);
  std::memcpy(&bad, hp + 8, 4);
  double m;
  std::memcpy(&m, &bits, 8);
  *dt_host = h->cfg.cfl * m;
  if (bad != 0) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dt, bits, h->d_bad, 1);
    (void)hipStreamSynchronize(s);
    return fail(h, ATHMHD_ENONPHYS, "%d non-physical cell evaluations (rho <= 0, P <= 0 or not finite)", bad);
  }
  return ATHMHD_OK;
}

int athmhd_profile(athmhd_t h, int enable, double* total_ms, int* launches) {
  if (!h) return ATHMHD_EINVAL;
  if (enable) {
    drop_events(h);
    h->profiling = true;
    return ATHMHD_OK;
  }
  h->profiling = false;
  double sum = 0.0;
  int n = 0;
  for (size_t q = 0; q + 1 < h->events.size(); q += 2) {
    hipError_t e = hipEventSynchronize(h->events[q + 1]);
    if (e != hipSuccess) return hip_fail(h, e, "profiling event synchronise");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, h->events[q], h->events[q + 1]);
    if (e != hipSuccess) return hip_fail(h, e, "profiling elapsed time");
    sum += ms;
    ++n;
  }
  drop_events(h);
  if (total_ms) *total_ms = sum;
  if (launches) *launches = n;
  return ATHMHD_OK;
}

}  // extern "C"
