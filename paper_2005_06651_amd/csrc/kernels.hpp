// kernels.hpp -- host-side launchers of the HIP kernels (defined in the .hip
// files).  All launchers are asynchronous on `s` and return the launch status.
#pragma once

#include "common.hpp"

namespace athmhd {

struct Gas;
struct BatchDesc;

// Scratch of the unfused pipeline for nb blocks: cell primitives (8 arrays:
// rho, v1, v2, v3, p, B1cc, B2cc, B3cc), per-direction face data (8 arrays:
// 5 fluxes, EMF of component t1, EMF of component t2, upwind weight) and the
// three corner-EMF arrays.
struct UnfusedScratch {
  double* w;       // nb * 8 * cvar
  double* face[3]; // nb * 8 * fvar each
  double* edge;    // nb * 3 * fvar
};

hipError_t launch_fill_ghosts(const Geo& g, double* cons, double* bface, int nb, hipStream_t s);
// ghost exchange of the coupled mesh g.mesh[0] x g.mesh[1] x g.mesh[2]: the w
// ghost layers nearest each block's active box (w outside [1, ng]: all ng)
hipError_t launch_mesh_ghosts(const Geo& g, int w, double* cons, double* bface, hipStream_t s, bool open_x1 = false);
// (open_x1: the mesh is not periodic along x1; entries whose owner along x1
// lies beyond the mesh are left as they are, except the B1 faces on the
// mesh's upper x1 boundary plane, owned by the last blocks along x1)
// Level operators of block refinement on a box: fine cells [flo, flo + 2 ext)
// <-> coarse cells [clo, clo + ext) (stored indices, checked by the caller).
hipError_t launch_restrict(const Geo& g, const int flo[3], const int clo[3], const int ext[3], const double* fc,
                           const double* fb, double* cc, double* cb, hipStream_t s);
// primitive: prolong (rho, v, P, C_i) instead of U; otherwise pfloor > 0
// applies the pressure floor to the refined cells, activations counted in bad.
// keep: bit 2 d + S keeps the fine faces already on side S of the box along d.
hipError_t launch_prolong(const Geo& g, const int flo[3], const int clo[3], const int ext[3], const double* cc,
                          const double* cb, double* fc, double* fb, bool primitive, int keep, double gamma,
                          double pfloor, int* bad, hipStream_t s);
hipError_t launch_prim2cons(const Geo& g, double gamma, const double* prim, const double* bface, double* cons,
                            int nb, hipStream_t s);
// dt_bits: device uint64 holding the bit pattern of the running minimum of
// dx_d/(|v_d| + c_f) (initialise to +inf bits); bad: device int counter
hipError_t launch_newdt(const Geo& g, double gamma, const double* cons, const double* bface, int nb,
                        unsigned long long* dt_bits, const Floors& fl, int* bad, hipStream_t s, bool floor = false);
// (floor: apply the floors of launch_floor_state to cons first, in the same
// pass; floors must be on)

// The same CFL reduction in two launches that use no atomics and need no
// cleared memory: one partial result per workgroup (minimum of
// dx_d/(|v_d| + c_f,d), DBL_MAX if the workgroup met no physical cell, and
// its count of non-physical cells), then one workgroup that reduces them.
struct DtPart {
  double m;
  int nbad, pad;
};
// At most max_parts partials are written (one launch over every block;
// *nparts receives the count); hipErrorInvalidValue when nb > max_parts.
hipError_t launch_newdt_parts(const Geo& g, double gamma, const double* cons, const double* bface, int nb,
                              const Floors& fl, DtPart* parts, int max_parts, int* nparts, hipStream_t s);
hipError_t launch_newdt_parts_batch(const BatchDesc* desc, int nblocks, double gamma, const double* cons,
                                    const double* bface, const Floors& fl, DtPart* parts, int max_parts, int* nparts,
                                    hipStream_t s);
// dt_out = cfl * min of the partials (+inf if none is finite); nbad_out = their
// counts plus *step_bad, which is then cleared.
hipError_t launch_newdt_finish(const DtPart* parts, int nparts, double cfl, int* step_bad, double* dt_out,
                               int* nbad_out, hipStream_t s);

// One stage of the unfused pipeline: out = g0*x + g1*un + bdt * L(x), where
// x must have filled ghosts.  out must not alias x; un may alias out.
// dt_dev, if not NULL, supplies dt on the device (bdt = beta * dt).
hipError_t launch_stage_unfused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                                const double* xb, const double* unc, const double* unb, double* outc,
                                double* outb, StageCoef coef, const double* dt_dev, double beta, int nb,
                                UnfusedScratch& scr, const Floors& fl, int* bad,
                                bool charac, hipStream_t s);  // charac: PLM on characteristic variables

// The two halves of launch_stage_unfused: primitives, face fluxes and corner
// EMFs into scr; then the 2S update from them (between the two, a caller may
// correct the fluxes and EMFs in scr).
hipError_t launch_fluxes_unfused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                                 const double* xb, int nb, UnfusedScratch& scr, const Floors& fl, int* bad,
                                 bool charac, hipStream_t s);
hipError_t launch_update_unfused(const Geo& g, const double* xc, const double* xb, const double* unc,
                                 const double* unb, double* outc, double* outb, StageCoef coef, const double* dt_dev,
                                 double beta, int nb, const UnfusedScratch& scr, hipStream_t s,
                                 bool keep_x1_lower = false);

// Two-level composite (block 0 coarse, blocks 1..8 fine; the unfused scratch
// of the coarse block and of the first fine block): flux correction of the
// coarse x1 boundary faces from the mean of the four fine fluxes, and EMF
// correction of the coarse E2, E3 on the two interface planes from the mean
// of the two fine EMFs along them.  gc: the coarse geometry (n, ng).
hipError_t launch_level_correct(const Geo& gc, UnfusedScratch& coarse, const UnfusedScratch& fine, hipStream_t s);
// The x1 faces on the interface x1 = X, owned by the fine blocks with a = 1:
// out = g0 x + g1 un + bdt (-curl E) from the fine blocks' corner EMFs.
hipError_t launch_level_fine_faces(const Geo& gf, const double* xb, const double* unb, double* outb, StageCoef coef,
                                   const double* dt_dev, double beta, const UnfusedScratch& fine, hipStream_t s);

// One stage in a single fused kernel (same contract as launch_stage_unfused);
// kz = x3 planes per workgroup segment (0: default for the block size).
// dt_dev, if not NULL, supplies dt on the device (bdt = beta * dt).
// bad[0] counts threads that met a non-physical cell; floor activations go to
// the 64-bit counter of add_floor_count.
hipError_t launch_stage_fused(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                              const double* xb, const double* unc, const double* unb, double* outc, double* outb,
                              StageCoef coef, const double* dt_dev, double beta, int nb, int kz, Floors fl, int* bad,
                              double* fm, hipStream_t s);  // kz > 0: x3 planes per workgroup
// fm: NULL, or the output of the mass flux through the lower face of every
// active cell along each direction (3 face arrays per block), for the passive
// scalars.
int fused_default_kz(const Geo& g, int nb, int cus);

// Passive scalars of one stage (rows 5 .. 5+ns-1 of the cell arrays), after
// the fused stage that stored the face mass fluxes fm:
//   out_i = g0 * x_i + g1 * un_i + bdt * L_i,
// L_i the difference of the mass fluxes times C_i = (rho C_i)/rho of the
// stage input x, reconstructed (recon) on the upwind side.  Blocks of a
// coupled mesh read their exchanged ghost cells, and the mass flux through an
// upper boundary face from the next block; out may alias un, not x.
hipError_t launch_scalar_stage(const Geo& g, int recon, const double* xc, const double* unc, double* outc,
                               const double* fm, StageCoef coef, const double* dt_dev, double beta, int nb,
                               Floors fl, hipStream_t s);

// Batched blocks of uneven sizes.  One block descriptor per block: its
// geometry and the offsets (in doubles) of its cons and bface in the
// concatenated arrays.  One work item per (block, tile, x3 segment).
struct BatchDesc {
  Geo g;
  int64_t coff, foff;
};
struct WorkItem {
  int block, tile_x, tile_y, k0, kend;
};
int batch_tile_count();                             // candidate thread tiles
void batch_tile_shape(int shape, int* tx, int* ty);  // active columns of a candidate
int batch_tile_threads(int shape);
// One stage of all blocks in one persistent launch of `grid` workgroups that
// drain the item queue.  dt_dev, if not NULL, supplies dt on the device
// (bdt = beta * dt); otherwise coef.bdt is used.
// mesh: the blocks tile one domain and read their (exchanged) ghost entries
// instead of their own periodic images (then without floors and fm).
hipError_t launch_stage_batch(int shape, double gamma, int recon, int rs, double ct_eps, const BatchDesc* desc,
                              const WorkItem* items, int nitems, unsigned* queue, const double* xc,
                              const double* xb, const double* unc, const double* unb, double* outc, double* outb,
                              StageCoef coef, const double* dt_dev, double beta, int grid, Floors fl, int* bad,
                              double* fm, hipStream_t s,  // fm: NULL, or mass-flux output laid out like bface
                              bool mesh = false);
// Passive scalars of one stage of batched blocks (same contract as
// launch_scalar_stage; fm laid out like bface).  items: one per (block, tile of
// scalar_batch_tile() x scalar_batch_tile() columns, x3 segment).
int scalar_batch_tile();
hipError_t launch_scalar_stage_batch(const BatchDesc* desc, const WorkItem* items, int nitems, int ns, bool near,
                                     int recon, const double* xc, const double* unc, double* outc, const double* fm,
                                     StageCoef coef, const double* dt_dev, double beta, Floors fl, hipStream_t s);
// Ghost fill, prim->cons and the CFL reduction over all blocks of a batch.
hipError_t launch_fill_ghosts_batch(const BatchDesc* desc, int nblocks, int64_t max_shell, double* cons,
                                    double* bface, hipStream_t s);
// Blocks that tile one periodic domain: every shell entry of block b (in the
// order of shell_entry) is copied from src[off[b] + t] = (owning block, its
// stored position of the same domain cell packed as i | j << 10 | k << 20).
// work: nwork chunks (block, first entry) of exchange_chunk() entries each,
// covering every block's shell.
int exchange_chunk();
hipError_t launch_exchange_batch(const BatchDesc* desc, const int64_t* off, const int2* src, const int2* work,
                                 int nwork, double* cons, double* bface, hipStream_t s);
hipError_t launch_prim2cons_batch(const BatchDesc* desc, int nblocks, int64_t max_cells, double gamma,
                                  const double* prim, const double* bface, double* cons, hipStream_t s);
hipError_t launch_newdt_batch(const BatchDesc* desc, int nblocks, int64_t max_active, double gamma,
                              const double* cons, const double* bface, unsigned long long* dt_bits,
                              const Floors& fl, int* bad, hipStream_t s);

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);

// Floors on the conserved state of the active cells after a stage: rho raised
// to fl.d, and E raised where the pressure implied by (U, B) is below fl.p
// (face fields are read with periodic wrap).  Changed cells are counted in bad.
hipError_t launch_floor_state(const Geo& g, double gamma, const Floors& fl, double* cons, const double* bface, int nb,
                              int* bad, hipStream_t s);
hipError_t launch_floor_state_batch(const BatchDesc* desc, int nblocks, double gamma, const Floors& fl, double* cons,
                                    const double* bface, int* bad, hipStream_t s);

// ---- reverse mode (periodic uniform blocks) ---------------------------------
// Cotangent sets are 8 active-only arrays per block (5 conserved variables,
// then the lower face of each active cell for B1, B2, B3), x1 fastest, block
// stride 8 * n1 * n2 * n3 doubles.
// Scratch doubles per block needed by launch_stage_vjp.
int64_t adj_scratch_per_block(const Geo& g);
// One stage of the reverse sweep for the spatial operator L of a stage
// (recon DC or PLM, HLLE or HLLD, CT weight eps), X in the padded layout:
//   O = g0 V + scale J_L(X)^T V,  and if Z != NULL:  Z = (zfirst ? 0 : Z) + g1 V.
// O must not alias V or Z.
hipError_t launch_stage_vjp(const Geo& g, double gamma, int recon, int rs, double ct_eps, const double* xc,
                            const double* xb, const double* V, double* O, double g0, double scale, double* Z,
                            double g1, int zfirst, double* scr, int nb, hipStream_t s);
hipError_t launch_adj_fill(double* p, double v, int64_t n, hipStream_t s);
// out = xc * x + yc * y (elementwise; out may alias x or y)
hipError_t launch_adj_axpby(double* out, double xc, const double* x, double yc, const double* y, int64_t n,
                            hipStream_t s);
// reverse of prim -> cons on every stored cell: gprim <- J^T gcons,
// gbface += (dcons/dbface)^T gcons
hipError_t launch_prim2cons_vjp(const Geo& g, double gamma, const double* prim, const double* bface,
                                const double* gcons, double* gprim, double* gbface, int nb, hipStream_t s);
// active entries of padded (cons, bface) arrays -> cotangent set
hipError_t launch_adj_gather(const Geo& g, const double* gc, const double* gb, double* V, int nb, hipStream_t s);
// padded outputs: active entries X + Y, all other entries copied from the inputs
hipError_t launch_adj_scatter(const Geo& g, const double* X, const double* Y, const double* gc_in,
                              const double* gb_in, double* gc_out, double* gb_out, int nb, hipStream_t s);

}  // namespace athmhd
