// abi.hip -- host side of the C ABI declared in include/athmhd.h: argument
// validation (entirely before any HIP call), device buffers, the stage driver
// of the 2S integrators (Eq. (rk-2s), Sec. 3.2.3), batched blocks of uneven
// sizes (work items, tile autotuner), optional hipGraph replay of a step, and
// error reporting.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/athmhd.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace athmhd;

struct athmhd_s {
  athmhd_config cfg;
  int device = 0;
  // uniform handle: nbmax identical blocks of geometry g
  Geo g;
  int nbmax = 0;
  // coupled mesh (athmhd_create_mesh): the nbmax blocks tile one periodic
  // domain as g.mesh[0] x g.mesh[1] x g.mesh[2]
  bool mesh = false;
  // the unfused pipeline runs the stages (kernel_path 1, or characteristic
  // reconstruction, which only that pipeline implements)
  bool unfused = false;
  // two-level composite (athmhd_create_levels): block 0 coarse (geometry g,
  // with mesh[0] = -1), blocks 1..8 fine (geometry gf, widths dx / 2)
  bool levels = false;
  Geo gf{};
  // batched handle: blocks of their own sizes, concatenated in the arrays
  bool batch = false;
  int nbatch = 0;
  std::vector<BatchDesc> desc;
  int64_t ctot = 0, ftot = 0;            // doubles of cons / bface over all blocks
  int64_t max_shell = 0, max_cells = 0;  // per-block maxima (ghost shell, stored cells)
  BatchDesc* d_desc = nullptr;
  WorkItem* d_items = nullptr;
  int nitems = 0, items_cap = 0;
  unsigned* d_queue = nullptr;
  int shape = 0, split = 0, grid = 0;   // batch tile candidate, x3 split, persistent grid
  // coupled batch (athmhd_batch_couple): the blocks tile one periodic domain
  // and exchange their shell entries by table (k_exchange_batch)
  bool coupled = false;
  int64_t* d_xoff = nullptr;  // per block: first table entry of its shell
  int2* d_xsrc = nullptr;     // per shell entry: owner block, packed stored position
  int2* d_xwork = nullptr;    // per exchange workgroup: block, first shell entry
  int nxwork = 0;
  // state registers and scratch
  double* reg[2] = {nullptr, nullptr};  // two stage registers (cons followed by bface)
  int64_t reg_coff = 0;                  // offset of bface inside a register
  UnfusedScratch scr{};
  double* scratch_base = nullptr;
  // passive scalars (g.ns > 0): face mass fluxes of a stage, 3 face arrays per block
  double* d_fm = nullptr;
  WorkItem* d_sitems = nullptr;  // batched blocks: the scalar kernel's work items
  int nsitems = 0;
  int min_edge = 0;  // batched blocks: fewest active cells along any direction of any block
  unsigned long long* d_dtmin = nullptr;  // running min of dx/(|v|+cf), bit pattern
  int* d_bad = nullptr;                   // counters of add_floor_count: [0] non-physical cells, [2, 4) floors (64-bit)
  Floors floors{0.0, 0.0};                // optional primitive floors (off by default)
  double* d_dtval = nullptr;              // dt of the step on the device (graph replay)
  void* h_pinned = nullptr;               // 16 bytes of pinned host memory for newdt
  int kz = 0;                             // x3 planes per fused workgroup (0: default)
  int cus = 0;                            // compute units of the device
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> events;  // (start, stop) pairs around stage kernels
  // hipGraph replay of a step
  bool use_graph = false;
  hipGraph_t graph = nullptr;  // kept alive: its dt node is updated in the executable graph
  hipGraphExec_t gexec = nullptr;
  hipGraphNode_t dt_node = nullptr;
  const void* gkey[3] = {nullptr, nullptr, nullptr};
  int gkey_nb = 0;
  // reverse mode (allocated by the first athmhd_step_vjp)
  double* adj_base = nullptr;
  double* adj_state[2] = {nullptr, nullptr};  // recomputed stage inputs X_1, X_2
  double* adj_scr = nullptr;                  // per-block scratch of the stage VJP
  double* adj_cot[3] = {nullptr, nullptr, nullptr};  // cotangent sets A, A', Z
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

// clear_bad: bit 0 clears the non-physical counter, bit 1 the floor counter
__global__ void k_set_u64(unsigned long long* p, unsigned long long v, int* bad, int clear_bad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *p = v;
    if (clear_bad & 1) bad[0] = 0;
    if (clear_bad & 2) *reinterpret_cast<unsigned long long*>(bad + 2) = 0ull;
  }
}

// End of a chained step: the next step's dt from the CFL minimum (cfl times
// +inf when no cell gave a limit), and the non-physical count handed over and
// cleared when the caller asked for it.
__global__ void k_chain_finish(const unsigned long long* bits, double cfl, int* bad, double* dt_dev,
                               int32_t* nbad_dev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *dt_dev = cfl * __longlong_as_double((long long)*bits);
    if (nbad_dev) {
      *nbad_dev = bad[0];
      bad[0] = 0;
    }
  }
}

// first node of a replayed step: puts this step's dt on the device
__global__ void k_set_dt(double* p, double dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = dt;
}

int validate_common(const athmhd_config* c) {
  if (!c) return fail(nullptr, ATHMHD_EINVAL, "config is NULL");
  if (c->recon < ATHMHD_RECON_DC || c->recon > ATHMHD_RECON_PPM)
    return fail(nullptr, ATHMHD_EINVAL, "unknown reconstruction %d", c->recon);
  if (c->riemann != ATHMHD_RS_HLLE && c->riemann != ATHMHD_RS_HLLD && c->riemann != ATHMHD_RS_ROE)
    return fail(nullptr, ATHMHD_EINVAL, "unknown Riemann solver %d", c->riemann);
  if (c->integrator < ATHMHD_RK1 || c->integrator > ATHMHD_RK3)
    return fail(nullptr, ATHMHD_EINVAL, "unknown integrator %d", c->integrator);
  const int need = c->recon == ATHMHD_RECON_PPM ? 3 : 2;
  if (c->nghost < need || c->nghost > 8)
    return fail(nullptr, ATHMHD_EINVAL, "nghost must be in [%d, 8] for this reconstruction (got %d)", need,
                c->nghost);
  if (!(std::isfinite(c->gamma) && c->gamma > 1.0))
    return fail(nullptr, ATHMHD_EINVAL, "gamma must be finite and > 1 (got %g)", c->gamma);
  if (!(std::isfinite(c->cfl) && c->cfl > 0.0 && c->cfl <= 1.0))
    return fail(nullptr, ATHMHD_EINVAL, "cfl must be in (0, 1] (got %g)", c->cfl);
  if (!(std::isfinite(c->ct_eps) && c->ct_eps >= 0.0))
    return fail(nullptr, ATHMHD_EINVAL, "ct_eps must be finite and >= 0 (got %g)", c->ct_eps);
  if (c->kernel_path != 0 && c->kernel_path != 1)
    return fail(nullptr, ATHMHD_EINVAL, "kernel_path must be 0 (fused) or 1 (unfused)");
  if (c->nscalars < 0 || c->nscalars > 64)
    return fail(nullptr, ATHMHD_EINVAL, "nscalars must be in [0, 64] (got %d)", c->nscalars);
  if (c->charac != 0 && c->charac != 1) return fail(nullptr, ATHMHD_EINVAL, "charac must be 0 or 1");
  return ATHMHD_OK;
}

int validate_block(int n1, int n2, int n3, int ng, double dx1, double dx2, double dx3) {
  if (n1 < 1 || n2 < 1 || n3 < 1)
    return fail(nullptr, ATHMHD_EINVAL, "block dims must be >= 1 (got %d %d %d)", n1, n2, n3);
  if (!finite_pos(dx1) || !finite_pos(dx2) || !finite_pos(dx3))
    return fail(nullptr, ATHMHD_EINVAL, "cell widths must be finite and > 0");
  const double faces = (double)(n1 + 2 * ng + 1) * (n2 + 2 * ng + 1) * (n3 + 2 * ng + 1);
  if (faces >= 2147483647.0) return fail(nullptr, ATHMHD_EINVAL, "block too large for 32-bit in-array indices");
  return ATHMHD_OK;
}

int check_call(athmhd_t h, const void* a, const void* b, int nb) {
  if (!h) return ATHMHD_EINVAL;
  if (!a || !b) return fail(h, ATHMHD_EINVAL, "NULL array argument");
  if (h->levels) {
    if (nb != 9) return fail(h, ATHMHD_EINVAL, "a two-level composite has 9 blocks (got %d)", nb);
  } else if (h->batch) {
    if (nb != h->nbatch)
      return fail(h, ATHMHD_EINVAL, "nblocks must equal the batch size %d (got %d)", h->nbatch, nb);
  } else if (h->mesh) {
    if (nb != h->nbmax)
      return fail(h, ATHMHD_EINVAL, "nblocks must equal the mesh's block count %d (got %d)", h->nbmax, nb);
  } else if (nb < 1 || nb > h->nbmax) {
    return fail(h, ATHMHD_EINVAL, "nblocks %d outside [1, %d]", nb, h->nbmax);
  }
  return ATHMHD_OK;
}

void drop_events(athmhd_t h) {
  for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
  h->events.clear();
}

void drop_graph(athmhd_t h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->dt_node = nullptr;
  h->gkey[0] = h->gkey[1] = h->gkey[2] = nullptr;
  h->gkey_nb = 0;
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
  drop_graph(h);
  for (int r = 0; r < 2; ++r)
    if (h->reg[r]) (void)hipFree(h->reg[r]);
  if (h->scratch_base) (void)hipFree(h->scratch_base);
  if (h->d_fm) (void)hipFree(h->d_fm);
  if (h->d_sitems) (void)hipFree(h->d_sitems);
  if (h->d_dtmin) (void)hipFree(h->d_dtmin);
  if (h->d_bad) (void)hipFree(h->d_bad);
  if (h->d_dtval) (void)hipFree(h->d_dtval);
  if (h->d_desc) (void)hipFree(h->d_desc);
  if (h->d_items) (void)hipFree(h->d_items);
  if (h->d_queue) (void)hipFree(h->d_queue);
  if (h->d_xoff) (void)hipFree(h->d_xoff);
  if (h->d_xsrc) (void)hipFree(h->d_xsrc);
  if (h->d_xwork) (void)hipFree(h->d_xwork);
  if (h->h_pinned) (void)hipHostFree(h->h_pinned);
  if (h->adj_base) (void)hipFree(h->adj_base);
}

// Small device buffers every handle has.
bool alloc_common(athmhd_t h) {
  return hipMalloc(&h->d_dtmin, sizeof(unsigned long long)) == hipSuccess &&
         hipMalloc(&h->d_bad, 4 * sizeof(int)) == hipSuccess && hipMalloc(&h->d_dtval, sizeof(double)) == hipSuccess &&
         hipHostMalloc(&h->h_pinned, 16, hipHostMallocDefault) == hipSuccess;
}

void read_env(athmhd_t h) {
  if (const char* kz = getenv("ATHMHD_KZ")) h->kz = atoi(kz);
}

// ---- batched blocks: work items of one tile candidate ---------------------
int build_items(athmhd_t h, int shape, int split) {
  int TX, TY;
  batch_tile_shape(shape, &TX, &TY);
  std::vector<WorkItem> items;
  for (int b = 0; b < h->nbatch; ++b) {
    const Geo& g = h->desc[b].g;
    const int ntx = (g.n1 + TX - 1) / TX, nty = (g.n2 + TY - 1) / TY;
    const int kz = split ? (g.n3 + 1) / 2 : g.n3;
    for (int k0 = g.ng; k0 < g.ng + g.n3; k0 += kz)
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) items.push_back({b, tx, ty, k0, std::min(k0 + kz, g.ng + g.n3)});
  }
  // longest items first, so the short ones fill the tail of the persistent grid
  std::stable_sort(items.begin(), items.end(),
                   [](const WorkItem& a, const WorkItem& b) { return (a.kend - a.k0) > (b.kend - b.k0); });
  if ((int)items.size() > h->items_cap) {
    if (h->d_items) (void)hipFree(h->d_items);
    h->d_items = nullptr;
    if (hipMalloc(&h->d_items, items.size() * sizeof(WorkItem)) != hipSuccess)
      return fail(h, ATHMHD_ENOMEM, "work item table");
    h->items_cap = (int)items.size();
  }
  hipError_t e = hipMemcpy(h->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "work item upload");
  h->nitems = (int)items.size();
  h->shape = shape;
  h->split = split;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, h->device);
  if (e != hipSuccess) return hip_fail(h, e, "device properties");
  // persistent grid: enough workgroups to fill every CU at the kernels' LDS and
  // register occupancy (at most 3 per CU), never more than there are items
  h->grid = std::max(1, std::min(h->nitems, prop.multiProcessorCount * 3));
  drop_graph(h);
  return ATHMHD_OK;
}

// ---- two-level composite ----------------------------------------------------
// Unfused scratch of the fine blocks (the coarse block's is h->scr itself).
UnfusedScratch fine_scratch(athmhd_t h) {
  UnfusedScratch f = h->scr;
  f.w += 8 * h->g.cvar;
  for (int d = 0; d < 3; ++d) f.face[d] += 8 * h->g.fvar;
  f.edge += 3 * h->g.fvar;
  return f;
}

// Ghosts of the composite (Sec. 2.1.3): the fine blocks' same-level exchange
// (a 2 x 2 x 2 mesh, open along x1); the coarse block's periodic images, then
// its x1 ghost slabs and x1 boundary faces restricted from the fine blocks
// (Sec. 2.1.5), in boxes split where the fine block or the periodic image
// changes; the fine blocks' x1 ghost slabs beyond the fine region
// prolongated from the coarse block, keeping the fine interface faces.
hipError_t levels_ghosts(athmhd_t h, double* cons, double* bface, hipStream_t s) {
  const Geo& g = h->g;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3, ng = g.ng;
  double* fc = cons + g.cblock;
  double* fb = bface + g.fblock;
  Geo gm = h->gf;
  gm.mesh[0] = gm.mesh[1] = gm.mesh[2] = 2;
  hipError_t e = launch_mesh_ghosts(gm, 0, fc, fb, s, true);
  if (e == hipSuccess) e = launch_fill_ghosts(g, cons, bface, 1, s);
  // (first coarse stored index, extent, fine block along the direction, first fine stored index)
  struct Seg {
    int c, h, fb, f;
  };
  const Seg sj[4] = {{0, ng, 1, n2 - ng}, {ng, n2 / 2, 0, ng}, {ng + n2 / 2, n2 / 2, 1, ng}, {ng + n2, ng, 0, ng}};
  const Seg sk[4] = {{0, ng, 1, n3 - ng}, {ng, n3 / 2, 0, ng}, {ng + n3 / 2, n3 / 2, 1, ng}, {ng + n3, ng, 0, ng}};
  for (int side = 0; side < 2 && e == hipSuccess; ++side)
    for (int a = 0; a < 4 && e == hipSuccess; ++a)
      for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        const int fa = side == 0 ? 1 : 0;
        const int flo[3] = {side == 0 ? n1 - ng : ng, sj[a].f, sk[c].f};
        const int clo[3] = {side == 0 ? 0 : ng + n1, sj[a].c, sk[c].c};
        const int ext[3] = {ng, sj[a].h, sk[c].h};
        const int q = fa + 2 * sj[a].fb + 4 * sk[c].fb;
        e = launch_restrict(g, flo, clo, ext, fc + q * g.cblock, fb + q * g.fblock, cons, bface, s);
      }
  for (int q = 0; q < 8 && e == hipSuccess; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const int flo[3] = {a == 1 ? ng + n1 : 0, 0, 0};
    const int clo[3] = {a == 1 ? ng : ng + n1 - ng / 2, ng + b * n2 / 2 - ng / 2, ng + c * n3 / 2 - ng / 2};
    const int ext[3] = {ng / 2, g.N2 / 2, g.N3 / 2};
    e = launch_prolong(g, flo, clo, ext, cons, bface, fc + q * g.cblock, fb + q * g.fblock, false, a == 1 ? 1 : 2,
                       h->cfg.gamma, h->floors.p, h->d_bad, s);
  }
  return e;
}

// One stage of the composite: fluxes and EMFs of both levels, flux and EMF
// correction (Sec. 2.1.4), the updates, and the fine-owned interface faces.
hipError_t levels_stage(athmhd_t h, int recon, const double* xc, const double* xb, const double* unc,
                        const double* unb, double* oc, double* ob, StageCoef cf, double beta, const double* dt_dev,
                        hipStream_t s) {
  const Geo& g = h->g;
  UnfusedScratch fs = fine_scratch(h);
  const bool ch = h->cfg.charac != 0;
  hipError_t e = launch_fluxes_unfused(g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc, xb, 1, h->scr,
                                       h->floors, h->d_bad, ch, s);
  if (e == hipSuccess)
    e = launch_fluxes_unfused(h->gf, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc + g.cblock, xb + g.fblock,
                              8, fs, h->floors, h->d_bad, ch, s);
  if (e == hipSuccess) e = launch_level_correct(g, h->scr, fs, s);
  // the coarse x1 boundary faces are the fine blocks' (restricted at each fill)
  if (e == hipSuccess) e = launch_update_unfused(g, xc, xb, unc, unb, oc, ob, cf, dt_dev, beta, 1, h->scr, s, true);
  if (e == hipSuccess)
    e = launch_update_unfused(h->gf, xc + g.cblock, xb + g.fblock, unc + g.cblock, unb + g.fblock, oc + g.cblock,
                              ob + g.fblock, cf, dt_dev, beta, 8, fs, s);
  if (e == hipSuccess)
    e = launch_level_fine_faces(h->gf, xb + g.fblock, unb + g.fblock, ob + g.fblock, cf, dt_dev, beta, fs, s);
  return e;
}

// The CFL minimum of a state folded into bits (atomic minimum of the bit
// patterns of non-negative doubles).  floor: the floors of the last stage
// are applied in the same pass (uniform and mesh handles).
hipError_t launch_cfl(athmhd_t h, const double* cons, const double* bface, int nblocks, unsigned long long* bits,
                      hipStream_t s, bool floor = false) {
  if (h->levels) {
    hipError_t e = launch_newdt(h->g, h->cfg.gamma, cons, bface, 1, bits, h->floors, h->d_bad, s);
    if (e != hipSuccess) return e;
    return launch_newdt(h->gf, h->cfg.gamma, cons + h->g.cblock, bface + h->g.fblock, 8, bits, h->floors,
                        h->d_bad, s);
  }
  if (h->batch) return launch_newdt_batch(h->d_desc, h->nbatch, 0, h->cfg.gamma, cons, bface, bits, h->floors,
                                          h->d_bad, s);
  return launch_newdt(h->g, h->cfg.gamma, cons, bface, nblocks, bits, h->floors, h->d_bad, s, floor);
}

// x3 planes per workgroup of the fused stage kernel on nblocks uniform blocks
int stage_kz(athmhd_t h, int nblocks) { return h->kz > 0 ? h->kz : fused_default_kz(h->g, nblocks, h->cus); }

// One stage: uniform or batched, fused or unfused.
hipError_t launch_stage(athmhd_t h, int recon, const double* xc, const double* xb, const double* unc,
                        const double* unb, double* oc, double* ob, StageCoef cf, double beta, const double* dt_dev,
                        int nblocks, hipStream_t s) {
  if (h->levels) return levels_stage(h, recon, xc, xb, unc, unb, oc, ob, cf, beta, dt_dev, s);
  if (h->batch)
    return launch_stage_batch(h->shape, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, h->d_desc, h->d_items,
                              h->nitems, h->d_queue, xc, xb, unc, unb, oc, ob, cf, dt_dev, beta, h->grid, h->floors,
                              h->d_bad, h->g.ns > 0 ? h->d_fm : nullptr, s, h->coupled);
  if (!h->unfused)
    return launch_stage_fused(h->g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc, xb, unc, unb, oc, ob, cf,
                              dt_dev, beta, nblocks, stage_kz(h, nblocks), h->floors, h->d_bad,
                              h->g.ns > 0 ? h->d_fm : nullptr, s);
  return launch_stage_unfused(h->g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc, xb, unc, unb, oc, ob,
                              cf, dt_dev, beta, nblocks, h->scr, h->floors, h->d_bad, h->cfg.charac != 0, s);
}

// depth: ghost layers a mesh exchange fills (0: all); other handles fill all
hipError_t fill_ghosts(athmhd_t h, double* cons, double* bface, int nblocks, hipStream_t s, int depth = 0) {
  if (h->levels) return levels_ghosts(h, cons, bface, s);
  if (h->batch && h->coupled)
    return launch_exchange_batch(h->d_desc, h->d_xoff, h->d_xsrc, h->d_xwork, h->nxwork, cons, bface, s);
  if (h->batch) return launch_fill_ghosts_batch(h->d_desc, h->nbatch, h->max_shell, cons, bface, s);
  if (h->mesh) return launch_mesh_ghosts(h->g, depth, cons, bface, s);
  return launch_fill_ghosts(h->g, cons, bface, nblocks, s);
}

// The launches of one full step (everything asynchronous on s).  With
// dt_dev != NULL the stage kernels read dt from the device.
// stages != NULL (uniform handles): the inputs of stages 1..S-1 are written
// there (S-1 states, each all blocks' cons then all blocks' bface) instead of
// the library's registers.  dt_bits != NULL: the CFL minimum of the new
// state is folded into it after the step.
int enqueue_step(athmhd_t h, double* cons, double* bface, double dt, const double* dt_dev, int nblocks,
                 hipStream_t s, double* stages = nullptr, unsigned long long* dt_bits = nullptr) {
  // a chained step with floors on a uniform or mesh handle floors its last
  // stage's output in the CFL pass, which reads the whole state anyway
  const bool floor_in_cfl = dt_bits && h->floors.on() && !h->batch && !h->levels;
  const Scheme sc = scheme_of(h->cfg.integrator);
  const double* xc = cons;
  const double* xb = bface;
  hipError_t e;
  // the fused kernels read periodic images directly; the unfused pipeline
  // and the blocks of a coupled mesh or batch read ghost entries, which are
  // filled (exchanged between the blocks) before each stage
  const bool ghosts = (h->unfused && !h->batch) || h->mesh || h->coupled;
  const int64_t ncell = h->batch ? h->ctot : h->g.cblock * nblocks;
  const int64_t nface = h->batch ? h->ftot : h->g.fblock * nblocks;
  if (sc.nstage == 1) {
    // a single-stage scheme cannot update in place: its stage writes the
    // active entries of a register, which is copied back whole afterwards;
    // seed the register with the input so that the copy leaves ghost cells
    // and periodic-image faces as they were (they are not part of a step)
    if ((e = launch_copy(h->reg[0], cons, ncell, s)) != hipSuccess) return hip_fail(h, e, "copy launch");
    if ((e = launch_copy(h->reg[0] + h->reg_coff, bface, nface, s)) != hipSuccess)
      return hip_fail(h, e, "copy launch");
  }
  for (int st = 0; st < sc.nstage; ++st) {
    // the VL2 predictor always uses donor-cell fluxes (Sec. 3.2.3)
    const int recon = (h->cfg.integrator == ATHMHD_VL2 && st == 0) ? ATHMHD_RECON_DC : h->cfg.recon;
    // the fused stage reads recon + 1 cells past the block (the reconstruction
    // stencil of the ring faces); the unfused pipeline reads every ghost layer
    const int depth = h->unfused ? 0 : recon + 1;
    // a chained step on a coupled batch takes its input's shell entries as
    // current: every step ends with an exchange of its output
    const bool current = h->coupled && dt_bits && st == 0;
    if (ghosts && !current &&
        (e = fill_ghosts(h, const_cast<double*>(xc), const_cast<double*>(xb), nblocks, s, depth)) != hipSuccess)
      return hip_fail(h, e, "fill_ghosts launch");
    const bool last = st == sc.nstage - 1;
    double* oc;
    double* ob;
    if (last && xc != cons) {
      oc = cons;
      ob = bface;
    } else if (stages && !last) {
      oc = stages + (h->g.cblock + h->g.fblock) * (int64_t)nblocks * st;
      ob = oc + h->g.cblock * (int64_t)nblocks;
    } else {
      double* r = h->reg[st % 2];
      oc = r;
      ob = r + h->reg_coff;
    }
    StageCoef cf{sc.g0[st], sc.g1[st], sc.beta[st] * dt};
    if ((e = mark(h, s)) != hipSuccess) return hip_fail(h, e, "profiling event");
    e = launch_stage(h, recon, xc, xb, cons, bface, oc, ob, cf, sc.beta[st], dt_dev, nblocks, s);
    if (e != hipSuccess) return hip_fail(h, e, "stage launch");
    if ((e = mark(h, s)) != hipSuccess) return hip_fail(h, e, "profiling event");
    // passive scalars, carried by the mass fluxes the stage kernel stored
    if (h->g.ns > 0) {
      // one correction step finds the periodic images when every block has
      // more active cells per direction than the stencil's halo
      e = h->batch ? launch_scalar_stage_batch(h->d_desc, h->d_sitems, h->nsitems, h->g.ns, h->min_edge > recon + 1,
                                               recon, xc, cons, oc, h->d_fm, cf, dt_dev, sc.beta[st], h->floors, s)
                   : launch_scalar_stage(h->g, recon, xc, cons, oc, h->d_fm, cf, dt_dev, sc.beta[st], nblocks,
                                         h->floors, s);
      if (e != hipSuccess) return hip_fail(h, e, "scalar stage launch");
    }
    if (h->floors.on() && !(last && floor_in_cfl)) {
      e = h->batch ? launch_floor_state_batch(h->d_desc, h->nbatch, h->cfg.gamma, h->floors, oc, ob, h->d_bad, s)
                   : launch_floor_state(h->g, h->cfg.gamma, h->floors, oc, ob, nblocks, h->d_bad, s);
      if (e != hipSuccess) return hip_fail(h, e, "floor launch");
    }
    xc = oc;
    xb = ob;
  }
  if (xc != cons) {  // single-stage scheme: the result sits in a register
    if ((e = launch_copy(cons, xc, ncell, s)) != hipSuccess) return hip_fail(h, e, "copy launch");
    if ((e = launch_copy(bface, xb, nface, s)) != hipSuccess) return hip_fail(h, e, "copy launch");
  }
  // a composite leaves its ghosts and restricted coarse faces filled, which
  // its newdt reads; so does a coupled batch, whose blocks read their upper
  // faces (written by the neighbour that owns them) from their own shell
  if (h->levels && (e = levels_ghosts(h, cons, bface, s)) != hipSuccess) return hip_fail(h, e, "level ghost launch");
  if (h->coupled && (e = fill_ghosts(h, cons, bface, nblocks, s)) != hipSuccess)
    return hip_fail(h, e, "batch exchange launch");
  if (dt_bits && (e = launch_cfl(h, cons, bface, nblocks, dt_bits, s, floor_in_cfl)) != hipSuccess)
    return hip_fail(h, e, "newdt launch");
  return ATHMHD_OK;
}

// Capture one step into a graph whose first node writes dt to the device.
int capture_step(athmhd_t h, double* cons, double* bface, int nblocks, hipStream_t s) {
  drop_graph(h);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(h, e, "begin graph capture");
  hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, s, h->d_dtval, 0.0);
  int rc = enqueue_step(h, cons, bface, 0.0, h->d_dtval, nblocks, s);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (rc != ATHMHD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(h, e, "end graph capture");
  // the dt node is the only root of the captured graph
  size_t nroot = 0;
  e = hipGraphGetRootNodes(graph, nullptr, &nroot);
  if (e != hipSuccess || nroot != 1) {
    (void)hipGraphDestroy(graph);
    return fail(h, ATHMHD_EHIP, "captured step graph has %zu roots", nroot);
  }
  e = hipGraphGetRootNodes(graph, &h->dt_node, &nroot);
  if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    h->gexec = nullptr;
    h->dt_node = nullptr;
    return hip_fail(h, e, "graph instantiate");
  }
  h->graph = graph;
  h->gkey[0] = cons;
  h->gkey[1] = bface;
  h->gkey[2] = s;
  h->gkey_nb = nblocks;
  return ATHMHD_OK;
}

int replay_step(athmhd_t h, double dt, hipStream_t s) {
  hipKernelNodeParams p{};
  hipError_t e = hipGraphKernelNodeGetParams(h->dt_node, &p);
  if (e != hipSuccess) return hip_fail(h, e, "graph dt node");
  double* dst = h->d_dtval;
  void* args[2] = {&dst, &dt};
  p.kernelParams = args;
  p.extra = nullptr;
  e = hipGraphExecKernelNodeSetParams(h->gexec, h->dt_node, &p);
  if (e != hipSuccess) return hip_fail(h, e, "graph dt update");
  e = hipGraphLaunch(h->gexec, s);
  if (e != hipSuccess) return hip_fail(h, e, "graph launch");
  return ATHMHD_OK;
}

// Reverse-mode buffers of a uniform handle: stage states beyond the first,
// the stage-VJP scratch and three cotangent sets, for nbmax blocks.
int alloc_adjoint(athmhd_t h) {
  if (h->adj_base) return ATHMHD_OK;
  const Geo& g = h->g;
  const int64_t state = g.cblock + g.fblock;
  const int64_t nc = (int64_t)g.n1 * g.n2 * g.n3;
  const int nst = scheme_of(h->cfg.integrator).nstage;
  const int64_t nb = h->nbmax;
  const int64_t total = ((nst - 1) * state + adj_scratch_per_block(g) + 3 * 8 * nc) * nb;
  if (hipMalloc(&h->adj_base, total * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    h->adj_base = nullptr;
    return fail(h, ATHMHD_ENOMEM, "reverse-mode scratch of %.3f GB", total * 8.0 / 1e9);
  }
  double* p = h->adj_base;
  for (int st = 0; st < nst - 1; ++st) {
    h->adj_state[st] = p;
    p += state * nb;
  }
  h->adj_scr = p;
  p += adj_scratch_per_block(g) * nb;
  for (int q = 0; q < 3; ++q) {
    h->adj_cot[q] = p;
    p += 8 * nc * nb;
  }
  return ATHMHD_OK;
}

// ---- allocation-free CFL reduction (athmhd_newdt_noalloc) -----------------
// One partial result per workgroup of the reduction, in a fixed array of the
// library: each GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` is only a stand-in for the symbol; its device
// address on each device is found once, with that device current, and only
// that address is passed to kernels.
static __device__ __align__(256) DtPart scratch[ATHMHD_NOALLOC_MAX_BLOCKS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
DtPart* g_scratch_ptr[kMaxDevices] = {};

// Device address of scratch on device dev, which must be current.
int noalloc_scratch(athmhd_t h, int dev, DtPart** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(h, ATHMHD_EUNSUP, "device %d: the library keeps scratch addresses for devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(h, e, "address of the newdt scratch array");
    if (!p) return fail(h, ATHMHD_EHIP, "address of the newdt scratch array is NULL");
    g_scratch_ptr[dev] = static_cast<DtPart*>(p);
  }
  *out = g_scratch_ptr[dev];
  return ATHMHD_OK;
}

}  // namespace

extern "C" {

int athmhd_version(void) { return 112; }

int athmhd_create(const athmhd_config* cfg, int nblocks_max, athmhd_t* out) {
  if (!out) return fail(nullptr, ATHMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_common(cfg);
  if (rc != ATHMHD_OK) return rc;
  rc = validate_block(cfg->n1, cfg->n2, cfg->n3, cfg->nghost, cfg->dx1, cfg->dx2, cfg->dx3);
  if (rc != ATHMHD_OK) return rc;
  if (nblocks_max < 1) return fail(nullptr, ATHMHD_EINVAL, "nblocks_max must be >= 1");
  if (cfg->nscalars > 0 && (cfg->kernel_path != 0 || cfg->charac))
    return fail(nullptr, ATHMHD_EUNSUP, "passive scalars run with the fused kernels only");
  athmhd_t h = new (std::nothrow) athmhd_s();
  if (!h) return fail(nullptr, ATHMHD_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->g = make_geo(cfg->n1, cfg->n2, cfg->n3, cfg->nghost, cfg->dx1, cfg->dx2, cfg->dx3, cfg->nscalars);
  h->nbmax = nblocks_max;
  h->unfused = cfg->kernel_path == 1 || cfg->charac;
  read_env(h);
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device);
  if (e != hipSuccess) {
    rc = fail(nullptr, ATHMHD_EHIP, "device query: %s", hipGetErrorString(e));
    delete h;
    return rc;
  }
  h->reg_coff = h->g.cblock * (int64_t)nblocks_max;
  const int64_t state = (h->g.cblock + h->g.fblock) * (int64_t)nblocks_max;
  const int64_t nscr =
      h->unfused ? (8 * h->g.cvar + 24 * h->g.fvar + 3 * h->g.fvar) * (int64_t)nblocks_max : 1;
  const int64_t nfm = h->g.ns > 0 ? 3 * h->g.fvar * (int64_t)nblocks_max : 0;
  bool ok = hipMalloc(&h->reg[0], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->reg[1], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->scratch_base, nscr * sizeof(double)) == hipSuccess && alloc_common(h) &&
            (nfm == 0 || hipMalloc(&h->d_fm, nfm * sizeof(double)) == hipSuccess);
  if (!ok) {
    (void)hipGetLastError();
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_ENOMEM, "device allocation of %.3f GB failed",
                (2.0 * state + nscr + nfm) * 8.0 / 1e9);
  }
  double* p = h->scratch_base;
  h->scr.w = p;
  p += 8 * h->g.cvar * nblocks_max;
  for (int d = 0; d < 3; ++d) {
    h->scr.face[d] = p;
    p += 8 * h->g.fvar * nblocks_max;
  }
  h->scr.edge = p;
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, nullptr, h->d_dtmin, 0ull, h->d_bad, 3);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_EHIP, "initialisation: %s", hipGetErrorString(e));
  }
  *out = h;
  return ATHMHD_OK;
}

int athmhd_create_mesh(const athmhd_config* cfg, int nbx, int nby, int nbz, athmhd_t* out) {
  if (!out) return fail(nullptr, ATHMHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (nbx < 1 || nby < 1 || nbz < 1)
    return fail(nullptr, ATHMHD_EINVAL, "blocks per direction must be >= 1 (got %d %d %d)", nbx, nby, nbz);
  const double nb = (double)nbx * nby * nbz;
  if (nb > 1048576.0) return fail(nullptr, ATHMHD_EINVAL, "more than 2^20 blocks");
  if (cfg && (cfg->kernel_path != 0 || cfg->charac))
    return fail(nullptr, ATHMHD_EUNSUP, "a coupled mesh runs the fused kernels only");
  int rc = athmhd_create(cfg, (int)nb, out);
  if (rc != ATHMHD_OK) return rc;
  athmhd_t h = *out;
  h->mesh = true;
  h->g.mesh[0] = nbx;
  h->g.mesh[1] = nby;
  h->g.mesh[2] = nbz;
  return ATHMHD_OK;
}

int athmhd_create_levels(const athmhd_config* cfg, athmhd_t* out) {
  if (!out) return fail(nullptr, ATHMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_common(cfg);
  if (rc != ATHMHD_OK) return rc;
  if (cfg->nscalars != 0) return fail(nullptr, ATHMHD_EUNSUP, "a two-level composite carries no passive scalars");
  if (cfg->nghost % 2 != 0)
    return fail(nullptr, ATHMHD_EINVAL, "a two-level composite needs an even nghost (got %d)", cfg->nghost);
  const int n[3] = {cfg->n1, cfg->n2, cfg->n3};
  for (int d = 0; d < 3; ++d)
    if (n[d] % 2 != 0 || n[d] < 2 * cfg->nghost)
      return fail(nullptr, ATHMHD_EINVAL, "block sizes must be even and >= 2 nghost (got %d x %d x %d, nghost %d)",
                  cfg->n1, cfg->n2, cfg->n3, cfg->nghost);
  const double lo = std::min(cfg->dx1, std::min(cfg->dx2, cfg->dx3)), hi = std::max(cfg->dx1, std::max(cfg->dx2, cfg->dx3));
  if (!(hi - lo <= 1e-12 * hi)) return fail(nullptr, ATHMHD_EUNSUP, "face prolongation needs cubic cells (dx1 = dx2 = dx3)");
  athmhd_config c = *cfg;
  c.kernel_path = 1;  // the levels are coupled between flux computation and update
  rc = athmhd_create(&c, 9, out);
  if (rc != ATHMHD_OK) return rc;
  athmhd_t h = *out;
  h->levels = true;
  h->g.mesh[0] = -1;  // the stored upper faces are current after a step
  h->gf = make_geo(cfg->n1, cfg->n2, cfg->n3, cfg->nghost, 0.5 * cfg->dx1, 0.5 * cfg->dx2, 0.5 * cfg->dx3);
  h->gf.mesh[0] = -1;
  return ATHMHD_OK;
}

int athmhd_create_batch(const athmhd_config* base, const int32_t* dims, const double* dx, int nblocks,
                        athmhd_t* out) {
  if (!out) return fail(nullptr, ATHMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_common(base);
  if (rc != ATHMHD_OK) return rc;
  if (base->kernel_path != 0 || base->charac)
    return fail(nullptr, ATHMHD_EUNSUP, "batched blocks run on the fused kernel only");
  if (base->riemann == ATHMHD_RS_ROE)
    return fail(nullptr, ATHMHD_EUNSUP, "batched blocks take HLLE or HLLD");
  if (!dims || !dx) return fail(nullptr, ATHMHD_EINVAL, "NULL dims or dx");
  if (nblocks < 1 || nblocks > 65535) return fail(nullptr, ATHMHD_EINVAL, "nblocks must be in [1, 65535]");
  for (int b = 0; b < nblocks; ++b) {
    rc = validate_block(dims[3 * b], dims[3 * b + 1], dims[3 * b + 2], base->nghost, dx[3 * b], dx[3 * b + 1],
                        dx[3 * b + 2]);
    if (rc != ATHMHD_OK) {
      const std::string msg = g_create_err;
      return fail(nullptr, rc, "block %d: %s", b, msg.c_str());
    }
  }
  athmhd_t h = new (std::nothrow) athmhd_s();
  if (!h) return fail(nullptr, ATHMHD_ENOMEM, "host allocation failed");
  h->cfg = *base;
  h->batch = true;
  h->nbatch = nblocks;
  h->desc.resize(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    BatchDesc& d = h->desc[b];
    d.g = make_geo(dims[3 * b], dims[3 * b + 1], dims[3 * b + 2], base->nghost, dx[3 * b], dx[3 * b + 1],
                   dx[3 * b + 2], base->nscalars);
    d.coff = h->ctot;
    d.foff = h->ftot;
    h->ctot += d.g.cblock;
    h->ftot += d.g.fblock;
    const Geo& g = d.g;
    h->max_shell = std::max<int64_t>(h->max_shell, g.fvar - (int64_t)g.n1 * g.n2 * g.n3);
    h->max_cells = std::max<int64_t>(h->max_cells, g.cvar);
    const int edge = std::min(g.n1, std::min(g.n2, g.n3));
    h->min_edge = b == 0 ? edge : std::min(h->min_edge, edge);
  }
  h->g = h->desc[0].g;
  h->nbmax = nblocks;
  read_env(h);
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    rc = fail(nullptr, ATHMHD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    delete h;
    return rc;
  }
  h->reg_coff = h->ctot;
  const int64_t state = h->ctot + h->ftot;
  bool ok = hipMalloc(&h->reg[0], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->reg[1], state * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->d_desc, nblocks * sizeof(BatchDesc)) == hipSuccess &&
            hipMalloc(&h->d_queue, sizeof(unsigned)) == hipSuccess && alloc_common(h) &&
            (base->nscalars == 0 || hipMalloc(&h->d_fm, h->ftot * sizeof(double)) == hipSuccess);
  if (!ok) {
    (void)hipGetLastError();
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_ENOMEM, "device allocation of %.3f GB failed", 2.0 * state * 8.0 / 1e9);
  }
  if (base->nscalars > 0) {
    // work items of the scalar kernel: tiles of T x T columns, x3 segments of
    // at most 32 planes
    const int T = scalar_batch_tile();
    std::vector<WorkItem> si;
    for (int b = 0; b < nblocks; ++b) {
      const Geo& g = h->desc[b].g;
      for (int k0 = g.ng; k0 < g.ng + g.n3; k0 += 32)
        for (int ty = 0; ty < (g.n2 + T - 1) / T; ++ty)
          for (int tx = 0; tx < (g.n1 + T - 1) / T; ++tx) si.push_back({b, tx, ty, k0, std::min(k0 + 32, g.ng + g.n3)});
    }
    h->nsitems = (int)si.size();
    e = hipMalloc(&h->d_sitems, si.size() * sizeof(WorkItem));
    if (e == hipSuccess) e = hipMemcpy(h->d_sitems, si.data(), si.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      free_all(h);
      delete h;
      return fail(nullptr, ATHMHD_ENOMEM, "scalar work items: %s", hipGetErrorString(e));
    }
  }
  e = hipMemcpy(h->d_desc, h->desc.data(), nblocks * sizeof(BatchDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  }
  rc = build_items(h, 0, 0);
  if (rc != ATHMHD_OK) {
    const std::string msg = h->err;
    free_all(h);
    delete h;
    return fail(nullptr, rc, "%s", msg.c_str());
  }
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, nullptr, h->d_dtmin, 0ull, h->d_bad, 3);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, ATHMHD_EHIP, "initialisation: %s", hipGetErrorString(e));
  }
  *out = h;
  return ATHMHD_OK;
}

int athmhd_batch_info(athmhd_t h, int64_t* cons_len, int64_t* bface_len, int64_t* offsets) {
  if (!h) return ATHMHD_EINVAL;
  if (!h->batch) return fail(h, ATHMHD_EINVAL, "not a batched handle");
  if (cons_len) *cons_len = h->ctot;
  if (bface_len) *bface_len = h->ftot;
  if (offsets)
    for (int b = 0; b < h->nbatch; ++b) {
      offsets[2 * b] = h->desc[b].coff;
      offsets[2 * b + 1] = h->desc[b].foff;
    }
  return ATHMHD_OK;
}

int athmhd_batch_couple(athmhd_t h, const int32_t* origin, const int32_t* domain) {
  if (!h) return ATHMHD_EINVAL;
  if (!h->batch) return fail(h, ATHMHD_EINVAL, "not a batched handle");
  if (h->coupled) return fail(h, ATHMHD_EINVAL, "the batch is already coupled");
  if (!origin || !domain) return fail(h, ATHMHD_EINVAL, "NULL origin or domain");
  if (h->g.ns > 0) return fail(h, ATHMHD_EUNSUP, "a coupled batch carries no passive scalars");
  if (h->floors.on()) return fail(h, ATHMHD_EUNSUP, "a coupled batch takes no floors");
  const int64_t D[3] = {domain[0], domain[1], domain[2]};
  if (D[0] < 1 || D[1] < 1 || D[2] < 1 || D[0] * D[1] * D[2] > (int64_t)INT32_MAX)
    return fail(h, ATHMHD_EINVAL, "domain %lld x %lld x %lld cells out of range", (long long)D[0], (long long)D[1],
                (long long)D[2]);
  const int nb = h->nbatch;
  const Geo& g0 = h->desc[0].g;
  for (int b = 0; b < nb; ++b) {
    const Geo& g = h->desc[b].g;
    if (g.dx1 != g0.dx1 || g.dx2 != g0.dx2 || g.dx3 != g0.dx3)
      return fail(h, ATHMHD_EINVAL, "block %d: the blocks of a coupled batch share one cell width", b);
    if (g.F1 > 1024 || g.F2 > 1024 || g.F3 > 1024)
      return fail(h, ATHMHD_EINVAL, "block %d: stored extents above 1023 cells", b);
    const int n[3] = {g.n1, g.n2, g.n3};
    for (int d = 0; d < 3; ++d)
      if (origin[3 * b + d] < 0 || origin[3 * b + d] + n[d] > D[d])
        return fail(h, ATHMHD_EINVAL, "block %d lies outside the domain along x%d", b, d + 1);
  }
  // owner of every cell of the domain: each covered by exactly one block
  std::vector<int32_t> owner((size_t)(D[0] * D[1] * D[2]), -1);
  for (int b = 0; b < nb; ++b) {
    const Geo& g = h->desc[b].g;
    const int32_t* o = origin + 3 * b;
    for (int k = 0; k < g.n3; ++k)
      for (int j = 0; j < g.n2; ++j)
        for (int i = 0; i < g.n1; ++i) {
          int32_t& w = owner[(size_t)(((o[2] + k) * D[1] + o[1] + j) * D[0] + o[0] + i)];
          if (w >= 0) return fail(h, ATHMHD_EINVAL, "blocks %d and %d overlap", w, b);
          w = b;
        }
  }
  for (size_t c = 0; c < owner.size(); ++c)
    if (owner[c] < 0)
      return fail(h, ATHMHD_EINVAL, "cell %zu of the domain (x1 fastest) belongs to no block", c);
  // per block, its shell entries in the order of shell_entry
  std::vector<int64_t> off(nb);
  int64_t total = 0;
  for (int b = 0; b < nb; ++b) {
    const Geo& g = h->desc[b].g;
    off[b] = total;
    total += g.fvar - (int64_t)g.n1 * g.n2 * g.n3;
  }
  std::vector<int2> src((size_t)total);
  for (int b = 0; b < nb; ++b) {
    const Geo& g = h->desc[b].g;
    const int64_t ns = g.fvar - (int64_t)g.n1 * g.n2 * g.n3;
    for (int64_t t = 0; t < ns; ++t) {
      int x[3];
      shell_entry(g, t, x[0], x[1], x[2]);
      int64_t X[3];
      for (int d = 0; d < 3; ++d) {
        X[d] = ((int64_t)origin[3 * b + d] + x[d] - g.ng) % D[d];
        if (X[d] < 0) X[d] += D[d];
      }
      const int w = owner[(size_t)((X[2] * D[1] + X[1]) * D[0] + X[0])];
      const int ng = h->desc[w].g.ng;
      const int li = (int)(X[0] - origin[3 * w]) + ng, lj = (int)(X[1] - origin[3 * w + 1]) + ng,
                lk = (int)(X[2] - origin[3 * w + 2]) + ng;
      src[(size_t)(off[b] + t)] = make_int2(w, li | (lj << 10) | (lk << 20));
    }
  }
  // workgroups of the exchange: chunks of exchange_chunk() entries of one block
  std::vector<int2> work;
  for (int b = 0; b < nb; ++b) {
    const Geo& g = h->desc[b].g;
    const int64_t ns = g.fvar - (int64_t)g.n1 * g.n2 * g.n3;
    for (int64_t t0 = 0; t0 < ns; t0 += exchange_chunk()) work.push_back(make_int2(b, (int)t0));
  }
  if (work.size() > (size_t)INT32_MAX) return fail(h, ATHMHD_EINVAL, "exchange of %zu chunks", work.size());
  hipError_t e = hipMalloc(&h->d_xoff, nb * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&h->d_xsrc, (size_t)total * sizeof(int2));
  if (e == hipSuccess) e = hipMalloc(&h->d_xwork, work.size() * sizeof(int2));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (h->d_xoff) (void)hipFree(h->d_xoff);
    if (h->d_xsrc) (void)hipFree(h->d_xsrc);
    h->d_xoff = nullptr;
    h->d_xsrc = nullptr;
    h->d_xwork = nullptr;
    return fail(h, ATHMHD_ENOMEM, "exchange table of %.3f GB", (double)total * sizeof(int2) / 1e9);
  }
  // the blocks' upper boundary faces are stored (exchanged) entries from now
  // on: newdt and prim2cons read them there (cell_field)
  std::vector<BatchDesc> desc = h->desc;
  for (BatchDesc& d : desc) d.g.mesh[0] = -1;
  e = hipMemcpy(h->d_xoff, off.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_xsrc, src.data(), (size_t)total * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_xwork, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_desc, desc.data(), nb * sizeof(BatchDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipMemcpy(h->d_desc, h->desc.data(), nb * sizeof(BatchDesc), hipMemcpyHostToDevice);
    (void)hipFree(h->d_xoff);
    (void)hipFree(h->d_xsrc);
    (void)hipFree(h->d_xwork);
    h->d_xoff = nullptr;
    h->d_xsrc = nullptr;
    h->d_xwork = nullptr;
    return hip_fail(h, e, "exchange table upload");
  }
  h->nxwork = (int)work.size();
  h->desc = desc;
  h->g = h->desc[0].g;
  h->coupled = true;
  drop_graph(h);
  return ATHMHD_OK;
}

int athmhd_batch_set_tile(athmhd_t h, int shape, int split) {
  if (!h) return ATHMHD_EINVAL;
  if (!h->batch) return fail(h, ATHMHD_EINVAL, "not a batched handle");
  if (shape < 0 || shape >= batch_tile_count() || (split != 0 && split != 1))
    return fail(h, ATHMHD_EINVAL, "tile candidate %d / split %d out of range", shape, split);
  return build_items(h, shape, split);
}

int athmhd_batch_tune(athmhd_t h, const double* cons, const double* bface, void* stream, int* best_shape,
                      int* best_split, double* best_ms) {
  if (!h) return ATHMHD_EINVAL;
  if (!h->batch) return fail(h, ATHMHD_EINVAL, "not a batched handle");
  int rc = check_call(h, cons, bface, h->nbatch);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  // the stage reads the caller's arrays and writes register 0 only
  hipError_t e = hipSuccess;
  const double* xc = cons;
  const double* xb = bface;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(h, e, "tune events");
  }
  double best = 1e300;
  int bs = 0, bsp = 0;
  for (int shape = 0; shape < batch_tile_count() && rc == ATHMHD_OK; ++shape)
    for (int split = 0; split < 2 && rc == ATHMHD_OK; ++split) {
      if ((rc = build_items(h, shape, split)) != ATHMHD_OK) break;
      const StageCoef cf{0.0, 1.0, 1e-6};
      // one warm-up launch, then three timed launches of the configured stage
      for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        if (rep == 1) e = hipEventRecord(e0, s);
        if (e == hipSuccess)
          e = launch_stage(h, h->cfg.recon, xc, xb, xc, xb, h->reg[0], h->reg[0] + h->reg_coff, cf, 1.0, nullptr,
                           h->nbatch, s);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rc = hip_fail(h, e, "tune launch");
        break;
      }
      if (ms / 3.0 < best) {
        best = ms / 3.0;
        bs = shape;
        bsp = split;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the tuning launches may have counted non-physical cells of the scratch output
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dtmin, 0ull, h->d_bad, 3);
  if (rc != ATHMHD_OK) return rc;
  if ((rc = build_items(h, bs, bsp)) != ATHMHD_OK) return rc;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "tune synchronise");
  if (best_shape) *best_shape = bs;
  if (best_split) *best_split = bsp;
  if (best_ms) *best_ms = best;
  return ATHMHD_OK;
}

int athmhd_set_floors(athmhd_t h, double dfloor, double pfloor) {
  if (!h) return ATHMHD_EINVAL;
  if (!(std::isfinite(dfloor) && dfloor >= 0.0 && std::isfinite(pfloor) && pfloor >= 0.0))
    return fail(h, ATHMHD_EINVAL, "floors must be finite and >= 0 (got %g, %g)", dfloor, pfloor);
  if (h->coupled && (dfloor > 0.0 || pfloor > 0.0))
    return fail(h, ATHMHD_EUNSUP, "a coupled batch takes no floors");
  h->floors = Floors{dfloor, pfloor};
  drop_graph(h);  // captured launches carry the floors as arguments
  return ATHMHD_OK;
}

int athmhd_floor_count(athmhd_t h, long long* count, void* stream) {
  if (!h) return ATHMHD_EINVAL;
  if (!count) return fail(h, ATHMHD_EINVAL, "NULL count");
  hipStream_t s = (hipStream_t)stream;
  char* hp = (char*)h->h_pinned;
  hipError_t e = hipMemcpyAsync(hp, h->d_bad + 2, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dtmin, 0ull, h->d_bad, 2);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(h, e, "floor count");
  unsigned long long n;
  std::memcpy(&n, hp, 8);
  *count = (long long)n;
  return ATHMHD_OK;
}

int athmhd_set_graph(athmhd_t h, int enable) {
  if (!h) return ATHMHD_EINVAL;
  drop_graph(h);
  h->use_graph = enable != 0;
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
  hipError_t e = fill_ghosts(h, cons, bface, nblocks, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "fill_ghosts launch");
}

int athmhd_prim2cons(athmhd_t h, const double* prim, const double* bface, double* cons, int nblocks,
                     void* stream) {
  int rc = check_call(h, prim, bface, nblocks);
  if (rc) return rc;
  if (!cons) return fail(h, ATHMHD_EINVAL, "NULL cons");
  hipError_t e = h->batch ? launch_prim2cons_batch(h->d_desc, h->nbatch, h->max_cells, h->cfg.gamma, prim, bface,
                                                   cons, (hipStream_t)stream)
                          : launch_prim2cons(h->g, h->cfg.gamma, prim, bface, cons, nblocks, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "prim2cons launch");
}

int athmhd_step(athmhd_t h, double* cons, double* bface, double dt, int nblocks, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (h->levels && h->floors.on()) return fail(h, ATHMHD_EUNSUP, "a two-level composite runs without floors");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(h, ATHMHD_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  hipStream_t s = (hipStream_t)stream;
  if (!h->use_graph || h->profiling) return enqueue_step(h, cons, bface, dt, nullptr, nblocks, s);
  if (!s) return fail(h, ATHMHD_EINVAL, "graph replay needs a non-default stream");
  if (!(h->gexec && h->gkey[0] == cons && h->gkey[1] == bface && h->gkey[2] == s && h->gkey_nb == nblocks)) {
    rc = capture_step(h, cons, bface, nblocks, s);
    if (rc != ATHMHD_OK) return rc;
  }
  return replay_step(h, dt, s);
}

int athmhd_step_chain(athmhd_t h, double* cons, double* bface, int nblocks, double* dt_dev, int32_t* nbad_dev,
                      void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (h->levels && h->floors.on()) return fail(h, ATHMHD_EUNSUP, "a two-level composite runs without floors");
  if (!dt_dev) return fail(h, ATHMHD_EINVAL, "NULL dt_dev");
  hipStream_t s = (hipStream_t)stream;
  const double inf = INFINITY;
  unsigned long long inf_bits;
  std::memcpy(&inf_bits, &inf, 8);
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dtmin, inf_bits, h->d_bad, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "chain init launch");
  if ((rc = enqueue_step(h, cons, bface, 0.0, dt_dev, nblocks, s, nullptr, h->d_dtmin)) != ATHMHD_OK) return rc;
  hipLaunchKernelGGL(k_chain_finish, dim3(1), dim3(64), 0, s, h->d_dtmin, h->cfg.cfl, h->d_bad, dt_dev, nbad_dev);
  e = hipGetLastError();
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "chain finish launch");
}

int athmhd_step_vjp(athmhd_t h, const double* cons_n, const double* bface_n, double dt, const double* stages,
                    const double* g_cons_np1, const double* g_bface_np1, double* g_cons_n, double* g_bface_n,
                    int nblocks, void* stream) {
  int rc = check_call(h, cons_n, bface_n, nblocks);
  if (rc) return rc;
  if (h->batch || h->mesh || h->levels)
    return fail(h, ATHMHD_EUNSUP, "reverse mode is available for uniform handles only");
  if (h->floors.on()) return fail(h, ATHMHD_EUNSUP, "reverse mode is not available with floors");
  if (h->g.ns > 0) return fail(h, ATHMHD_EUNSUP, "reverse mode is not available with passive scalars");
  if (h->cfg.charac) return fail(h, ATHMHD_EUNSUP, "reverse mode is not available with characteristic reconstruction");
  if (h->cfg.riemann == ATHMHD_RS_ROE) return fail(h, ATHMHD_EUNSUP, "reverse mode takes HLLE or HLLD");
  if (!g_cons_np1 || !g_bface_np1 || !g_cons_n || !g_bface_n) return fail(h, ATHMHD_EINVAL, "NULL cotangent array");
  if (g_cons_n == cons_n || g_bface_n == bface_n || g_cons_n == (const double*)bface_n ||
      g_bface_n == (const double*)cons_n)
    return fail(h, ATHMHD_EINVAL, "cotangent outputs must not alias the state");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(h, ATHMHD_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  const Scheme sc = scheme_of(h->cfg.integrator);
  for (int st = 0; st < sc.nstage; ++st) {
    const int recon = (h->cfg.integrator == ATHMHD_VL2 && st == 0) ? ATHMHD_RECON_DC : h->cfg.recon;
    if (recon == ATHMHD_RECON_PPM) return fail(h, ATHMHD_EUNSUP, "reverse mode supports DC and PLM only");
  }
  if ((rc = alloc_adjoint(h)) != ATHMHD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->g;
  hipError_t e = hipSuccess;
  // forward: stage inputs X_0 = (cons_n, bface_n), X_1, ..., X_{S-1}
  const double* xc[3] = {cons_n, nullptr, nullptr};
  const double* xb[3] = {bface_n, nullptr, nullptr};
  if (stages) {  // stage inputs recorded by athmhd_step_stages
    for (int st = 0; st + 1 < sc.nstage; ++st) {
      xc[st + 1] = stages + (g.cblock + g.fblock) * (int64_t)nblocks * st;
      xb[st + 1] = xc[st + 1] + g.cblock * (int64_t)nblocks;
    }
  }
  for (int st = 0; !stages && st + 1 < sc.nstage; ++st) {
    double* oc = h->adj_state[st];
    double* ob = oc + g.cblock * (int64_t)nblocks;
    const int recon = (h->cfg.integrator == ATHMHD_VL2 && st == 0) ? ATHMHD_RECON_DC : h->cfg.recon;
    const StageCoef cf{sc.g0[st], sc.g1[st], sc.beta[st] * dt};
    e = launch_stage_fused(g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc[st], xb[st], cons_n, bface_n,
                           oc, ob, cf, nullptr, sc.beta[st], nblocks, stage_kz(h, nblocks), h->floors, h->d_bad,
                           nullptr, s);
    if (e != hipSuccess) return hip_fail(h, e, "vjp forward stage launch");
    xc[st + 1] = oc;
    xb[st + 1] = ob;
  }
  // reverse: with A the cotangent of X_{s+1},
  //   cotangent of X_s  = g0_s A + beta_s dt J_L(X_s)^T A,   and X_0 also
  //   collects g1_s A from every stage (its U^n term).
  double* A = h->adj_cot[0];
  double* An = h->adj_cot[1];
  double* Z = h->adj_cot[2];
  if ((e = launch_adj_gather(g, g_cons_np1, g_bface_np1, A, nblocks, s)) != hipSuccess)
    return hip_fail(h, e, "vjp set-up launch");
  for (int st = sc.nstage - 1; st >= 0; --st) {
    const int recon = (h->cfg.integrator == ATHMHD_VL2 && st == 0) ? ATHMHD_RECON_DC : h->cfg.recon;
    e = launch_stage_vjp(g, h->cfg.gamma, recon, h->cfg.riemann, h->cfg.ct_eps, xc[st], xb[st], A, An, sc.g0[st],
                         sc.beta[st] * dt, Z, sc.g1[st], st == sc.nstage - 1, h->adj_scr, nblocks, s);
    if (e != hipSuccess) return hip_fail(h, e, "stage vjp launch");
    std::swap(A, An);
  }
  e = launch_adj_scatter(g, A, Z, g_cons_np1, g_bface_np1, g_cons_n, g_bface_n, nblocks, s);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "vjp scatter launch");
}

namespace {

// Shared checks of the level operators: a uniform handle, four distinct
// arrays, and (prolongation) cubic cells.
int check_level_arrays(athmhd_t h, const void* a, const void* b, const void* c, const void* d, bool cubic) {
  if (!h) return ATHMHD_EINVAL;
  if (h->batch || h->mesh || h->levels) return fail(h, ATHMHD_EUNSUP, "level operators act on athmhd_create handles");
  if (!a || !b || !c || !d) return fail(h, ATHMHD_EINVAL, "NULL array argument");
  const void* p[4] = {a, b, c, d};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (p[i] == p[j]) return fail(h, ATHMHD_EINVAL, "the four arrays must be distinct");
  if (cubic) {
    const Geo& g = h->g;
    const double lo = std::min(g.dx1, std::min(g.dx2, g.dx3)), hi = std::max(g.dx1, std::max(g.dx2, g.dx3));
    if (hi - lo > 1e-12 * hi) return fail(h, ATHMHD_EUNSUP, "face prolongation needs cubic cells (dx1 = dx2 = dx3)");
  }
  return ATHMHD_OK;
}

// Every index a box operator touches lies in the stored arrays: fine cells
// [flo, flo + 2 ext) and their faces up to flo + 2 ext; coarse cells
// [clo, clo + ext) and faces up to clo + ext, and for prolongation one more
// cell (with its upper faces) on each side.
int check_level_box(athmhd_t h, const int* flo, const int* clo, const int* ext, bool prolong) {
  if (!flo || !clo || !ext) return fail(h, ATHMHD_EINVAL, "NULL box argument");
  const Geo& g = h->g;
  const int N[3] = {g.N1, g.N2, g.N3};
  for (int d = 0; d < 3; ++d) {
    if (ext[d] < 1) return fail(h, ATHMHD_EINVAL, "box extent must be >= 1 (got %d along x%d)", ext[d], d + 1);
    if (flo[d] < 0 || (long)flo[d] + 2L * ext[d] > N[d])
      return fail(h, ATHMHD_EINVAL, "fine box [%d, %ld) outside the %d stored cells along x%d", flo[d],
                  (long)flo[d] + 2L * ext[d], N[d], d + 1);
    const int lo = prolong ? 1 : 0, hi = prolong ? N[d] - 1 : N[d];
    if (clo[d] < lo || (long)clo[d] + ext[d] > hi)
      return fail(h, ATHMHD_EINVAL, "coarse box [%d, %ld) along x%d needs [%d, %d]%s", clo[d], (long)clo[d] + ext[d],
                  d + 1, lo, hi, prolong ? " (prolongation reads one neighbour on each side)" : "");
  }
  return ATHMHD_OK;
}

// The box of octant oct: fine active cells onto coarse active cells
// [ng + o_d n_d / 2, ng + (o_d + 1) n_d / 2).
int octant_box(athmhd_t h, const int oct[3], int flo[3], int clo[3], int ext[3]) {
  const Geo& g = h->g;
  if (g.n1 % 2 || g.n2 % 2 || g.n3 % 2)
    return fail(h, ATHMHD_EINVAL, "block sizes must be even (got %d x %d x %d)", g.n1, g.n2, g.n3);
  const int n[3] = {g.n1, g.n2, g.n3};
  for (int k = 0; k < 3; ++k) {
    if (oct[k] != 0 && oct[k] != 1) return fail(h, ATHMHD_EINVAL, "octant flags must be 0 or 1 (got %d)", oct[k]);
    ext[k] = n[k] / 2;
    flo[k] = g.ng;
    clo[k] = g.ng + oct[k] * ext[k];
  }
  return ATHMHD_OK;
}

int restrict_box(athmhd_t h, const double* fc, const double* fb, double* cc, double* cb, const int* flo,
                 const int* clo, const int* ext, void* stream) {
  int rc = check_level_box(h, flo, clo, ext, false);
  if (rc) return rc;
  hipError_t e = launch_restrict(h->g, flo, clo, ext, fc, fb, cc, cb, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "restrict launch");
}

int prolong_box(athmhd_t h, const double* cc, const double* cb, double* fc, double* fb, const int* flo,
                const int* clo, const int* ext, int primitive, int keep, void* stream) {
  if (primitive != 0 && primitive != 1) return fail(h, ATHMHD_EINVAL, "primitive must be 0 or 1 (got %d)", primitive);
  if (keep < 0 || keep > 63) return fail(h, ATHMHD_EINVAL, "keep must be a 6-bit mask (got %d)", keep);
  int rc = check_level_box(h, flo, clo, ext, true);
  if (rc) return rc;
  hipError_t e = launch_prolong(h->g, flo, clo, ext, cc, cb, fc, fb, primitive == 1, keep, h->cfg.gamma, h->floors.p,
                                h->d_bad, (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "prolong launch");
}

}  // namespace

int athmhd_restrict(athmhd_t h, const double* fine_cons, const double* fine_bface, double* coarse_cons,
                    double* coarse_bface, int o1, int o2, int o3, void* stream) {
  int rc = check_level_arrays(h, fine_cons, fine_bface, coarse_cons, coarse_bface, false);
  if (rc) return rc;
  const int oct[3] = {o1, o2, o3};
  int flo[3], clo[3], ext[3];
  rc = octant_box(h, oct, flo, clo, ext);
  if (rc) return rc;
  return restrict_box(h, fine_cons, fine_bface, coarse_cons, coarse_bface, flo, clo, ext, stream);
}

int athmhd_prolong(athmhd_t h, const double* coarse_cons, const double* coarse_bface, double* fine_cons,
                   double* fine_bface, int o1, int o2, int o3, int primitive, void* stream) {
  int rc = check_level_arrays(h, coarse_cons, coarse_bface, fine_cons, fine_bface, true);
  if (rc) return rc;
  const int oct[3] = {o1, o2, o3};
  int flo[3], clo[3], ext[3];
  rc = octant_box(h, oct, flo, clo, ext);
  if (rc) return rc;
  return prolong_box(h, coarse_cons, coarse_bface, fine_cons, fine_bface, flo, clo, ext, primitive, 0, stream);
}

int athmhd_restrict_box(athmhd_t h, const double* fine_cons, const double* fine_bface, double* coarse_cons,
                        double* coarse_bface, const int* fine_lo, const int* coarse_lo, const int* extent,
                        void* stream) {
  int rc = check_level_arrays(h, fine_cons, fine_bface, coarse_cons, coarse_bface, false);
  if (rc) return rc;
  return restrict_box(h, fine_cons, fine_bface, coarse_cons, coarse_bface, fine_lo, coarse_lo, extent, stream);
}

int athmhd_prolong_box(athmhd_t h, const double* coarse_cons, const double* coarse_bface, double* fine_cons,
                       double* fine_bface, const int* fine_lo, const int* coarse_lo, const int* extent, int primitive,
                       int keep, void* stream) {
  int rc = check_level_arrays(h, coarse_cons, coarse_bface, fine_cons, fine_bface, true);
  if (rc) return rc;
  return prolong_box(h, coarse_cons, coarse_bface, fine_cons, fine_bface, fine_lo, coarse_lo, extent, primitive,
                     keep, stream);
}

int athmhd_prim2cons_vjp(athmhd_t h, const double* prim, const double* bface, const double* g_cons, double* g_prim,
                         double* g_bface, int nblocks, void* stream) {
  int rc = check_call(h, prim, bface, nblocks);
  if (rc) return rc;
  if (h->batch || h->mesh || h->levels)
    return fail(h, ATHMHD_EUNSUP, "reverse mode is available for uniform handles only");
  if (h->g.ns > 0) return fail(h, ATHMHD_EUNSUP, "reverse mode is not available with passive scalars");
  if (!g_cons || !g_prim || !g_bface) return fail(h, ATHMHD_EINVAL, "NULL cotangent array");
  if (g_prim == g_cons || g_prim == prim) return fail(h, ATHMHD_EINVAL, "g_prim must not alias g_cons or prim");
  hipError_t e = launch_prim2cons_vjp(h->g, h->cfg.gamma, prim, bface, g_cons, g_prim, g_bface, nblocks,
                                      (hipStream_t)stream);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "prim2cons vjp launch");
}

int athmhd_step_stages(athmhd_t h, double* cons, double* bface, double dt, double* stages, int nblocks,
                       void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (h->batch || h->mesh || h->levels)
    return fail(h, ATHMHD_EUNSUP, "stage recording is available for uniform handles only");
  if (!stages) return fail(h, ATHMHD_EINVAL, "NULL stages");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(h, ATHMHD_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  return enqueue_step(h, cons, bface, dt, nullptr, nblocks, (hipStream_t)stream, stages);
}

int athmhd_newdt(athmhd_t h, const double* cons, const double* bface, int nblocks, double* dt_host, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (!dt_host) return fail(h, ATHMHD_EINVAL, "NULL dt_host");
  hipStream_t s = (hipStream_t)stream;
  const double inf = INFINITY;
  unsigned long long inf_bits;
  std::memcpy(&inf_bits, &inf, 8);
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dtmin, inf_bits, h->d_bad, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "newdt init launch");
  if (h->levels) {
    e = launch_newdt(h->g, h->cfg.gamma, cons, bface, 1, h->d_dtmin, h->floors, h->d_bad, s);
    if (e == hipSuccess)
      e = launch_newdt(h->gf, h->cfg.gamma, cons + h->g.cblock, bface + h->g.fblock, 8, h->d_dtmin, h->floors,
                       h->d_bad, s);
  } else {
    e = h->batch ? launch_newdt_batch(h->d_desc, h->nbatch, 0, h->cfg.gamma, cons, bface, h->d_dtmin, h->floors,
                                      h->d_bad, s)
                 : launch_newdt(h->g, h->cfg.gamma, cons, bface, nblocks, h->d_dtmin, h->floors, h->d_bad, s);
  }
  if (e != hipSuccess) return hip_fail(h, e, "newdt launch");
  char* hp = (char*)h->h_pinned;
  if ((e = hipMemcpyAsync(hp, h->d_dtmin, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
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
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, h->d_dtmin, bits, h->d_bad, 1);
    (void)hipStreamSynchronize(s);
    return fail(h, ATHMHD_ENONPHYS, "%d non-physical cell evaluations (rho <= 0, P <= 0 or not finite)", bad);
  }
  return ATHMHD_OK;
}

int athmhd_newdt_noalloc(athmhd_t h, const double* cons, const double* bface, int nblocks, double* dt_dev,
                         int32_t* nbad_dev, void* stream) {
  int rc = check_call(h, cons, bface, nblocks);
  if (rc) return rc;
  if (!dt_dev || !nbad_dev) return fail(h, ATHMHD_EINVAL, "NULL dt_dev or nbad_dev");
  if (h->levels) return fail(h, ATHMHD_EUNSUP, "athmhd_newdt_noalloc takes uniform, mesh and batched handles");
  if (nblocks > ATHMHD_NOALLOC_MAX_BLOCKS)
    return fail(h, ATHMHD_EINVAL, "athmhd_newdt_noalloc takes at most %d blocks per call (got %d)",
                ATHMHD_NOALLOC_MAX_BLOCKS, nblocks);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
  if (dev != h->device) return fail(h, ATHMHD_EINVAL, "current device %d is not the handle's device %d", dev, h->device);
  DtPart* parts = nullptr;
  if ((rc = noalloc_scratch(h, dev, &parts)) != ATHMHD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  int nparts = 0;
  e = h->batch ? launch_newdt_parts_batch(h->d_desc, h->nbatch, h->cfg.gamma, cons, bface, h->floors, parts,
                                          ATHMHD_NOALLOC_MAX_BLOCKS, &nparts, s)
               : launch_newdt_parts(h->g, h->cfg.gamma, cons, bface, nblocks, h->floors, parts,
                                    ATHMHD_NOALLOC_MAX_BLOCKS, &nparts, s);
  if (e != hipSuccess) return hip_fail(h, e, "newdt launch");
  e = launch_newdt_finish(parts, nparts, h->cfg.cfl, h->d_bad, dt_dev, nbad_dev, s);
  return e == hipSuccess ? ATHMHD_OK : hip_fail(h, e, "newdt reduction launch");
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
