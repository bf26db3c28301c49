/*
 * athmhd.h -- C ABI of libathmhd.so, an MI355X (gfx950) implementation of the
 * unsplit finite-volume ideal-MHD update of Stone, Tomida, White & Felker
 * (2020), Section 3: primitive reconstruction (DC / PLM / PPM, Sec. 3.2.1),
 * HLLE / HLLD fluxes (Sec. 3.2.2), upwind constrained-transport corner EMFs
 * (Sec. 3.1), and the conservative plus face-field update inside the 2S
 * Runge-Kutta / VL2 integrators (Sec. 3.2.3, Eq. (rk-2s)), all in FP64.
 *
 * Problem solved by one step (Sec. 3.1, Eqs. (cons) and (total_energy) with
 * Pi = eta = eta_AD = Q = 0 and mu = 1): given volume-averaged conserved
 * variables U = (rho, rho v, E) with E = P/(gamma-1) + rho v^2/2 + B^2/2 and
 * face-area-averaged B on a uniform Cartesian MeshBlock, advance the ideal-MHD
 * conservation laws by dt so that the totals of U are conserved on a periodic
 * block and the discrete div B is unchanged.
 *
 * Memory layout (all arrays FP64, device memory, owned by the caller):
 *   N_d = n_d + 2*nghost (ghost layers on both sides, Sec. 2.1.1).
 *   cons  : [b][v][k][j][i], v in (rho, M1, M2, M3, E); shape per block
 *           5 x N3 x N2 x N1, i fastest.  Blocks are contiguous.
 *   bface : [b][c][k][j][i], shape per block 3 x (N3+1) x (N2+1) x (N1+1);
 *           component c at index (k,j,i) is the face on the lower side of cell
 *           (k,j,i) along direction c (B1 at x1-faces, B2 at x2-faces, B3 at
 *           x3-faces, padded to a common shape).
 *   prim  : same shape as cons, v in (rho, v1, v2, v3, P).
 * With nscalars = S > 0 passive scalars, cons holds 5 + S cell arrays per
 * block, the masses rho C_1 .. rho C_S after E, and prim the specific
 * densities C_1 .. C_S after P (see "Passive scalars" below).
 * Every block of an athmhd_create handle is its own periodic neighbour: ghost
 * cells and the boundary faces n_d+nghost are periodic images, filled by the
 * library.  The blocks of a coupled mesh (athmhd_create_mesh) or coupled batch
 * (athmhd_batch_couple) exchange these entries with their neighbours instead.
 *
 * Streams: every call that takes `stream` (a hipStream_t, NULL = default
 * stream) is asynchronous on it unless stated otherwise.
 *
 * Errors: every function returns ATHMHD_OK (0) or a negative code.  Argument
 * errors are detected on the host before any HIP call.  Asynchronous HIP errors
 * and non-physical cells met by a step (rho <= 0, P <= 0 or not finite, unless
 * floors are enabled with athmhd_set_floors) surface at the next athmhd_newdt.
 * athmhd_last_error returns a text description of the last failure of a
 * handle.
 */
#ifndef ATHMHD_H
#define ATHMHD_H

#include <stdint.h>

#if defined(__GNUC__)
#define ATHMHD_API __attribute__((visibility("default")))
#else
#define ATHMHD_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct athmhd_s* athmhd_t;

enum athmhd_status {
  ATHMHD_OK = 0,
  ATHMHD_EINVAL = -1,   /* bad argument or configuration                      */
  ATHMHD_ENOMEM = -2,   /* device allocation failed                            */
  ATHMHD_EHIP = -3,     /* a HIP runtime call failed                           */
  ATHMHD_ENONPHYS = -4, /* a step met rho <= 0, P <= 0 or a non-finite value   */
  ATHMHD_EUNSUP = -5    /* valid but not supported combination                 */
};

/* Reconstruction (Sec. 3.2.1).  The VL2 predictor always uses DC. */
enum { ATHMHD_RECON_DC = 0, ATHMHD_RECON_PLM = 1, ATHMHD_RECON_PPM = 2 };
/* Riemann solver (Sec. 3.2.2).  Roe's linearised solver uses the Roe matrix
 * built from exact jump identities with s-weighted velocity and enthalpy
 * averages and a swapped-weight transverse field average (see roe() in the
 * library source); no entropy fix.  athmhd_create_batch and athmhd_step_vjp
 * return ATHMHD_EUNSUP for it. */
enum { ATHMHD_RS_HLLE = 0, ATHMHD_RS_HLLD = 1, ATHMHD_RS_ROE = 2 };
/* Time integrator (Sec. 3.2.3). */
enum { ATHMHD_RK1 = 0, ATHMHD_VL2 = 1, ATHMHD_RK2 = 2, ATHMHD_RK3 = 3 };

typedef struct {
  int32_t n1, n2, n3;      /* active cells per block, >= 2 each                    */
  int32_t nghost;          /* >= 2 for DC/PLM, >= 3 for PPM (Sec. 2.1.1)           */
  double gamma;            /* adiabatic index, > 1 (Sec. 3.1)                      */
  double dx1, dx2, dx3;    /* uniform Cartesian cell widths, > 0                   */
  int32_t recon;           /* ATHMHD_RECON_*                                       */
  int32_t riemann;         /* ATHMHD_RS_*                                          */
  int32_t integrator;      /* ATHMHD_RK1 / VL2 / RK2 / RK3                         */
  int32_t kernel_path;     /* 0: one fused kernel per stage (default);             */
                           /* 1: unfused pipeline of simple kernels (reference)    */
  double cfl;              /* Courant number C0 for athmhd_newdt, in (0, 1]        */
  double ct_eps;           /* 0: CT upwinding by the sign of the face mass flux    */
                           /* (Gardiner & Stone 2005); > 0: continuous weight      */
                           /* clamp(1/2 + (F_rho/rho_bar)/(2 ct_eps c_max), 0, 1)  */
  int32_t nscalars;        /* passive scalars, in [0, 64] (Sec. 3.2.6, Eq.          */
                           /* (passive_scalars)); see "Passive scalars" below      */
  int32_t charac;          /* 0 or 1: PLM / PPM on characteristic variables C = LW  */
                           /* (Sec. 3.2.1); see "Characteristic reconstruction"    */
} athmhd_config;

/* Passive scalars (Sec. 3.2.6 "Additional Physics", Eq. (passive_scalars)):
 * each scalar obeys d(rho C)/dt + div(rho v C) = 0.  C is reconstructed with
 * the configured method (DC in the VL2 predictor) like the other primitives,
 * and the flux of rho C through a face is the face mass flux of the stage's
 * Riemann solve times C on the upwind side (left state where the mass flux is
 * >= 0).  With floors on, C = (rho C) / rho uses the floored density; the
 * floor pass after a stage leaves rho C unchanged.  Available with
 * kernel_path 0 on athmhd_create, athmhd_create_mesh (the mesh exchange then
 * also fills the scalars' ghost cells) and athmhd_create_batch handles (each
 * block holds 5 + nscalars cell arrays): athmhd_create with kernel_path 1
 * returns ATHMHD_EUNSUP for nscalars != 0, and so do athmhd_step_vjp and
 * athmhd_prim2cons_vjp on a handle with scalars.  The MHD state of a step does not depend on the
 * scalars. */

/* Characteristic reconstruction (Sec. 3.2.1, C = L W): with charac = 1 the
 * PLM or PPM states at each face are formed on the characteristic variables
 * of the primitive system in the face frame: for each cell the differences
 * of (rho, vn, vt1, vt2, P, Bt1, Bt2) across its stencil are projected with
 * the left eigenvectors of that cell's state (normal field: the cell-centred
 * one), reconstructed per wave family (van Leer slope, or the limited PPM
 * parabola) and projected back with the right eigenvectors (normalised after
 * Roe & Balsara 1996).  DC (the VL2 predictor) is unchanged.  Such a handle
 * runs the stages on the unfused kernel pipeline whatever kernel_path says.
 * ATHMHD_EUNSUP with passive scalars, on athmhd_create_mesh and
 * athmhd_create_batch, and from athmhd_step_vjp. */

/* Version of this ABI (major*100 + minor). */
ATHMHD_API int athmhd_version(void);

/* Validate `cfg` on the host, then allocate the stage registers and scratch of
 * one block on the current device.  nblocks_max identical blocks may later be
 * advanced together (each periodic on its own).  On success *out receives a
 * handle owned by the caller (free with athmhd_destroy).  The fused stage
 * kernel marches each workgroup over a segment of x3 planes whose length is
 * chosen per launch from the block size and the device's CU count; a positive
 * integer in the environment variable ATHMHD_KZ, read here, fixes it instead. */
ATHMHD_API int athmhd_create(const athmhd_config* cfg, int nblocks_max, athmhd_t* out);

/* One full time step of nblocks (<= nblocks_max) blocks, in place:
 * (cons, bface) hold U^n on entry and U^{n+1} on return on the active cells
 * and faces.  Ghost entries are neither read nor written by the fused kernels
 * (each block is its own periodic neighbour and reads its periodic images
 * directly); call athmhd_fill_ghosts when the ghost entries are wanted.
 * dt > 0 and finite.  Asynchronous on `stream`. */
ATHMHD_API int athmhd_step(athmhd_t h, double* cons, double* bface, double dt, int nblocks, void* stream);

/* One full time step (as athmhd_step) whose dt comes from the device and
 * which also yields the next one (Sec. 2.1.7: the time step of the next cycle
 * is the CFL limit of the state the cycle leaves).  *dt_dev (device memory,
 * owned by the caller) holds this step's dt on entry; in stream order after
 * the step it holds cfl * min over the new state's active cells of
 * dx_d / (|v_d| + c_f,d), the value athmhd_newdt would return for it (+inf
 * when no cell gives a finite limit), computed by the CFL reduction of
 * athmhd_newdt queued after the step.  nbad_dev (device int, or NULL): the
 * number of non-physical cells met by the step and the reduction, after which
 * the handle's counter is cleared; with NULL the count stays in the handle
 * and the next athmhd_newdt reports it.  No host synchronisation: a run of
 * steps is queued without waiting.  Graph mode (athmhd_set_graph) does not
 * apply.  Asynchronous on `stream`. */
ATHMHD_API int athmhd_step_chain(athmhd_t h, double* cons, double* bface, int nblocks, double* dt_dev,
                                 int32_t* nbad_dev, void* stream);

/* Global time step dt = cfl * min over active cells and directions of
 * dx_d / (|v_d| + c_f,d) (Sec. 2.1.7, Sec. 3.2.3), written to *dt_host.
 * Synchronises `stream`.  Returns ATHMHD_ENONPHYS if this state or any step
 * since the previous call met a non-physical cell (the flag is then cleared),
 * ATHMHD_EHIP if an asynchronous HIP error is pending. */
ATHMHD_API int athmhd_newdt(athmhd_t h, const double* cons, const double* bface, int nblocks, double* dt_host,
                 void* stream);

/* Two-level composite (Sec. 2.1.3 communication between levels, Sec. 2.1.4
 * flux and EMF correction, Sec. 2.1.5 restriction and prolongation): nine
 * blocks of the shape of cfg (n1 x n2 x n3 active cells, nghost ghosts) on a
 * periodic box [0, 2X) x [0, Y) x [0, Z), X = n1 dx1, Y = n2 dx2, Z = n3 dx3.
 * Block 0 is coarse (widths dx of cfg) and covers [X, 2X) x [0, Y) x [0, Z);
 * block 1 + a + 2b + 4c (a, b, c in {0, 1}) is fine (widths dx / 2) and
 * covers the octant (a, b, c) of [0, X) x [0, Y) x [0, Z).  cons and bface
 * hold the nine blocks one after the other in the layout above (nblocks = 9
 * in every call).  Each stage exchanges ghosts within the fine level, fills
 * the coarse block's x1 ghost slabs and x1 boundary faces by restriction of
 * the fine blocks, prolongates the fine blocks' x1 ghost slabs beyond the
 * fine region from the coarse block, computes fluxes and corner EMFs on both
 * levels, replaces the coarse fluxes through the two interfaces by the mean
 * of the four fine fluxes and the coarse E2, E3 on the interface planes by
 * the mean of the two fine EMFs along them, and updates.  The interface
 * faces belong to the fine blocks.  Unlike other handles, a step ends with
 * this ghost fill, so the ghost entries of cons and bface are current after
 * it.  Needs an even nghost, even n_d >= 2 nghost, cubic cells and no
 * passive scalars; runs the unfused kernels (kernel_path is ignored).
 * ATHMHD_EUNSUP from athmhd_step with floors, and from the reverse-mode,
 * stage-recording, level-operator and allocation-free calls. */
ATHMHD_API int athmhd_create_levels(const athmhd_config* cfg, athmhd_t* out);

/* Most blocks one call of athmhd_newdt_noalloc accepts. */
#define ATHMHD_NOALLOC_MAX_BLOCKS 65536

/* Allocation-free athmhd_newdt, for callers that cannot allocate device or
 * pinned host memory or synchronise: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same reduction over the
 * same cells, with its results left in caller-owned device memory instead of
 * host memory:
 *   dt_dev[0]   = cfl * min over active cells and directions of
 *                 dx_d / (|v_d| + c_f,d), the value athmhd_newdt returns
 *                 (+inf when no cell is physical; the minimum over the
 *                 physical cells otherwise);
 *   nbad_dev[0] = non-physical cells met by this reduction plus those met by
 *                 steps since the previous newdt call; the handle's counter
 *                 is then cleared, as athmhd_newdt clears it.  A caller
 *                 checks nbad_dev[0] == 0 where athmhd_newdt would return
 *                 ATHMHD_ENONPHYS.
 * The call allocates nothing, copies nothing to the host and never
 * synchronises; it only enqueues two kernels on `stream`.  Its partial results
 * (one per workgroup, at most ATHMHD_NOALLOC_MAX_BLOCKS of 16 bytes, 1 MiB)
 * live in a fixed device array of the library, one per GPU, kept until the
 * process ends and fully rewritten by every call, so nothing needs clearing.
 * Calls that overlap on one GPU (several streams, or host threads) share that
 * array and race: serialise them.  The handle's device must be current.
 * ATHMHD_EINVAL for NULL outputs or nblocks > ATHMHD_NOALLOC_MAX_BLOCKS, and
 * as athmhd_newdt for the other arguments. */
ATHMHD_API int athmhd_newdt_noalloc(athmhd_t h, const double* cons, const double* bface, int nblocks, double* dt_dev,
                                    int32_t* nbad_dev, void* stream);

/* cons <- conserved variables of (prim, bface) on every stored cell, using the
 * cell-centred field (mean of the two bounding faces).  Asynchronous. */
ATHMHD_API int athmhd_prim2cons(athmhd_t h, const double* prim, const double* bface, double* cons, int nblocks,
                     void* stream);

/* Fill the ghost cells and periodic image faces of (cons, bface). */
ATHMHD_API int athmhd_fill_ghosts(athmhd_t h, double* cons, double* bface, int nblocks, void* stream);

/* Reverse mode of one step (vector-Jacobian product).  The step is the map
 * S: (U^n, B^n) -> (U^{n+1}, B^{n+1}) that athmhd_step computes with this
 * handle's configuration and the given dt, on each of nblocks periodic
 * blocks (Sec. 3.2: reconstruction, Riemann fluxes, upwind CT and the 2S
 * stages of Eq. (rk-2s)).  Given the state (cons_n, bface_n) at the start of
 * the step and cotangents (g_cons_np1, g_bface_np1) of the step's output,
 * writes (g_cons_n, g_bface_n) = J_S^T (g_cons_np1, g_bface_np1), the
 * gradient of <g_np1, S(x)> with respect to x = (cons_n, bface_n).
 *   - Layouts as cons / bface.  The independent entries are the active cells
 *     and, per component, the lower face of each active cell.  Every other
 *     entry (ghost cells, the periodic-image faces n_d + nghost, padding) is
 *     left unchanged by a step, so its cotangent passes through: g_n equals
 *     g_np1 there.
 *   - g_cons_n / g_bface_n may alias g_cons_np1 / g_bface_np1; they must not
 *     alias cons_n / bface_n.
 *   - stages: NULL, or the stage inputs recorded by athmhd_step_stages for
 *     this step (cons_n, bface_n, dt); with NULL they are recomputed from
 *     (cons_n, bface_n).  The library allocates its reverse-mode scratch on
 *     the first call (about 95 doubles per active cell and block, plus one
 *     state per stage beyond the first).
 *   - Supported: DC and PLM reconstruction, HLLE and HLLD, all integrators.
 *     The derivative of the CT weight is taken for ct_eps > 0; with ct_eps = 0
 *     the weight is piecewise constant and contributes nothing.  PPM and
 *     batched handles return ATHMHD_EUNSUP.
 * Asynchronous on `stream`. */
ATHMHD_API int athmhd_step_vjp(athmhd_t h, const double* cons_n, const double* bface_n, double dt,
                               const double* stages, const double* g_cons_np1, const double* g_bface_np1,
                               double* g_cons_n, double* g_bface_n, int nblocks, void* stream);

/* One step exactly as athmhd_step, that also keeps the inputs of stages
 * 1..S-1 of the 2S scheme (S = 1, 2, 2, 3 for RK1, VL2, RK2, RK3): they are
 * written to `stages`, caller-owned device memory of (S-1) states, each the
 * nblocks cons arrays followed by the nblocks bface arrays (only active cells
 * and lower faces are defined).  Passing the same buffer as `stages` to
 * athmhd_step_vjp for this step skips its recomputation of those states.
 * Uniform handles only.  Asynchronous on `stream`. */
ATHMHD_API int athmhd_step_stages(athmhd_t h, double* cons, double* bface, double dt, double* stages, int nblocks,
                                  void* stream);

/* Reverse mode of athmhd_prim2cons on every stored cell: with U = prim2cons(W, B),
 * writes g_prim = (dU/dW)^T g_cons and adds (dU/dB)^T g_cons to g_bface (the
 * energy depends on the cell-centred field, the mean of the two bounding
 * faces, Sec. 3.1).  g_prim must not alias g_cons or prim.  Uniform handles
 * only (batched: ATHMHD_EUNSUP).  Asynchronous on `stream`. */
ATHMHD_API int athmhd_prim2cons_vjp(athmhd_t h, const double* prim, const double* bface, const double* g_cons,
                                    double* g_prim, double* g_bface, int nblocks, void* stream);

/* Coupled mesh: nbx x nby x nbz equal blocks (the block shape of `cfg`)
 * tiling one periodic domain of (nbx n1) x (nby n2) x (nbz n3) cells (Sec. 2.1:
 * a Mesh of MeshBlocks; Sec. 2.1.1: neighbouring blocks exchange ghost cells
 * and faces).  Block b = bx + nbx (by + nby bz) sits at (bx, by, bz); cons and
 * bface hold the nbx nby nbz blocks one after the other as for athmhd_create,
 * and nblocks in later calls must equal that count.
 *   - Before every stage the library fills each block's ghost cells and every
 *     face entry other than the lower faces of its active cells from the
 *     block that owns that position (device kernel); each face is therefore
 *     updated by exactly one block, and shared faces cannot drift apart.
 *     athmhd_step thus writes the ghost entries of its input; after it they
 *     hold the last stage's input (athmhd_fill_ghosts refreshes them).
 *   - athmhd_newdt, athmhd_prim2cons and the floors read the upper faces of a
 *     block's boundary cells from the neighbouring block, so they do not
 *     depend on ghost entries.
 *   - With one block per direction the result equals athmhd_create's
 *     periodic block; split into several blocks it equals the single block
 *     covering the whole domain.
 * Fused kernel path only (kernel_path 0; else ATHMHD_EUNSUP).  Reverse mode and
 * athmhd_step_stages return ATHMHD_EUNSUP on a mesh handle. */
ATHMHD_API int athmhd_create_mesh(const athmhd_config* cfg, int nbx, int nby, int nbz, athmhd_t* out);

/* Batched MeshBlocks of uneven sizes (Sec. 2.1: a Mesh of MeshBlocks, each
 * with its own cell count here, advanced with one global dt, Sec. 2.1.7).
 * `base` gives everything but the block shape (its n1..n3 and dx1..dx3 are
 * ignored); dims[3b..3b+2] and dx[3b..3b+2] give block b.  cons and bface of
 * a batched handle are the concatenations of the per-block arrays (block b's
 * cons at offsets[2b], its bface at offsets[2b+1], see athmhd_batch_info);
 * nblocks in later calls must equal the batch size.  Every block is its own
 * periodic neighbour unless athmhd_batch_couple makes the blocks one periodic
 * mesh.  Each stage runs as one persistent launch whose
 * workgroups pull (block, tile, x3 segment) items from a device queue; ghost
 * fill, prim2cons and newdt run over all blocks from a descriptor table.
 * Only the fused kernel path is supported (kernel_path must be 0). */
ATHMHD_API int athmhd_create_batch(const athmhd_config* base, const int32_t* dims, const double* dx, int nblocks,
                                   athmhd_t* out);

/* Sizes (in doubles) of the concatenated cons and bface arrays of a batched
 * handle and, if offsets is not NULL, the per-block offsets (2 per block). */
ATHMHD_API int athmhd_batch_info(athmhd_t h, int64_t* cons_len, int64_t* bface_len, int64_t* offsets);

/* Couple a batch into one periodic mesh of blocks of uneven sizes and a
 * single cell width (Sec. 2.1: a Mesh of MeshBlocks; Sec. 2.1.1: neighbouring
 * blocks exchange ghost cells and faces).  origin[3b..3b+2] is the position,
 * in cells of the domain, of block b's first active cell (x1 first); the
 * blocks must tile the domain[0] x domain[1] x domain[2] cells exactly, each
 * inside it, with equal dx1..dx3 (else ATHMHD_EINVAL).  Neighbours may
 * differ in size: a block's ghost entries can come from several blocks.
 *   - The library builds, on the host, a table naming for every shell entry
 *     of every block (ghost cells, and every face entry other than the lower
 *     faces of its active cells) the block that owns the same cell of the
 *     domain, and uploads it (8 bytes per entry; the handle owns it).  While
 *     it does, it holds a 4-byte owner for every cell of the domain in host
 *     memory (57 MB for 192 x 192 x 384 cells); the call synchronises.
 *   - athmhd_step then exchanges the shell entries by that table before
 *     every stage (a device gather kernel) and once more after the last, so
 *     every face is updated by exactly one block and the stored state is
 *     whole after a step; athmhd_newdt and athmhd_prim2cons read a block's
 *     upper faces from its own shell.  athmhd_fill_ghosts runs the same
 *     exchange.
 *   - athmhd_step_chain does the same but for the exchange before its first
 *     stage: it takes the shell entries of its input as current, as a step
 *     or athmhd_fill_ghosts leaves them (call athmhd_fill_ghosts after
 *     changing the active entries between chained steps).
 *   - Split into blocks, the result equals one periodic block covering the
 *     whole domain.
 * Not with passive scalars or floors (ATHMHD_EUNSUP; athmhd_set_floors on a
 * coupled batch likewise); calling it twice is ATHMHD_EINVAL. */
ATHMHD_API int athmhd_batch_couple(athmhd_t h, const int32_t* origin, const int32_t* domain);

/* Choose the thread tile of the batched stage kernel: shape indexes the
 * candidate tiles (0: 16x12, 1: 12x16, 2: 14x14, 3: 16x8 active columns) and
 * split = 1 halves the x3 extent of each work item. */
ATHMHD_API int athmhd_batch_set_tile(athmhd_t h, int shape, int split);

/* Autotuner: time the configured stage on (cons, bface) for every candidate
 * tile and split (the caller's arrays are not modified), keep the fastest and
 * report it (any output may be NULL).  Synchronises `stream`. */
ATHMHD_API int athmhd_batch_tune(athmhd_t h, const double* cons, const double* bface, void* stream, int* best_shape,
                                 int* best_split, double* best_ms);

/* Optional density and pressure floors (both 0, the default, disables them).
 * With dfloor or pfloor > 0:
 *   - after every stage, a cell whose density is below dfloor gets
 *     rho = dfloor, and a cell whose pressure (from U and the cell-centred
 *     field) is below pfloor gets its total energy raised so that P = pfloor;
 *     kinetic and magnetic energy are unchanged.  Mass and energy are then
 *     conserved up to what the floors add;
 *   - every conversion to primitives and every reconstructed face state uses
 *     rho_W = max(rho, dfloor), v = M / rho_W, P_W = max(P, pfloor).
 * Non-physical cells then no longer stop a run (only non-finite values are
 * reported by athmhd_newdt); every activation is counted instead.  The paper
 * names floors only for prolongation (Sec. 2.1.5); they are needed here by
 * strong blasts in low-beta gas, whose pressure otherwise falls below zero.
 * dfloor and pfloor must be finite and >= 0.  Reverse mode is unavailable with
 * floors. */
ATHMHD_API int athmhd_set_floors(athmhd_t h, double dfloor, double pfloor);

/* Number of floor activations (cells and face states) since the previous
 * call, which clears the counter.  Synchronises `stream`. */
ATHMHD_API int athmhd_floor_count(athmhd_t h, long long* count, void* stream);

/* enable = 1: athmhd_step records its launches once into a hipGraph (for the
 * given arrays, block count and stream, which must not be the default stream)
 * and replays the graph afterwards, updating only dt; any change of those
 * arguments recaptures.  Ignored while profiling is enabled. */
ATHMHD_API int athmhd_set_graph(athmhd_t h, int enable);

/* Kernel timing for measurement.  enable = 1 starts recording a pair of HIP
 * events around every launch of the stage kernel (the kernel that does
 * reconstruction, Riemann fluxes, CT and the update of one stage) on the stream
 * it is launched on, and clears the totals.  enable = 0 stops recording,
 * synchronises the recorded events and writes the summed duration in
 * milliseconds and the number of launches to *total_ms and *launches (either
 * may be NULL). */
ATHMHD_API int athmhd_profile(athmhd_t h, int enable, double* total_ms, int* launches);

/* Level operators of block refinement (Sec. 2.1.5), between a coarse block
 * and the fine block that refines its octant (o1, o2, o3) (each 0 or 1: the
 * lower or upper half of the active cells along that direction).  Both are
 * single blocks of this handle's shape (athmhd_create handles only, else
 * ATHMHD_EUNSUP; n1, n2, n3 even, else ATHMHD_EINVAL), laid out as for
 * athmhd_step, device arrays, all four distinct; the fine block's cells are
 * half as wide.  Every cell array (5 + nscalars) is treated alike; for new
 * blocks these are the conserved variables, as the method prescribes.
 *
 * athmhd_restrict: writes the octant's active coarse cells with the volume
 * average of their 8 fine cells, and every coarse face of the octant (its
 * upper boundary faces included) with the area average of its 4 fine faces.
 * Nothing else of the coarse block is touched; ghost entries of the fine
 * block are not read.
 *
 * athmhd_prolong: writes every active fine cell and face (upper boundary
 * faces included); fine ghost entries are not touched.  Reads the octant's
 * coarse cells and faces and one layer of their neighbours, ghosts included,
 * so fill the coarse block's ghosts first.  Cells: the coarse value plus the
 * minmod-limited slope along each direction times the child's offset of
 * 1/4 coarse cell.  Faces (Toth & Roe 2002): each coarse face split into 4 by
 * its 2D minmod-limited linear profile, then the 12 faces inside each coarse
 * cell such that every fine cell has the coarse cell's divergence and the
 * curl at each interior edge equals the mean tangential difference over the
 * two outer faces parallel to it.  The fine field of a divergence-free coarse
 * field is then divergence-free, and linear fields are reproduced exactly.
 * primitive = 0 (new blocks: conserved variables, as the method prescribes):
 * the cell arrays themselves are prolonged; with a pressure floor set
 * (athmhd_set_floors, pfloor > 0), a refined cell whose pressure (from its U
 * and the mean of its two bounding fine faces) is below pfloor gets E raised
 * to give pfloor, with rho and M unchanged (mass and momentum stay
 * conserved); activations count in athmhd_floor_count.
 * primitive = 1 (ghost zones between levels, where the method prolongs
 * primitives): the coarse cells read are converted to (rho, v, P, C_i) with
 * their cell-centred fields (mean of the two stored bounding faces), those
 * are prolonged as above, and each fine cell is converted back with the
 * cell-centred field of the prolonged fine faces; no floor is applied (P is
 * prolonged directly).  Other values: ATHMHD_EINVAL.
 * Needs cubic cells (dx1 = dx2 = dx3, else ATHMHD_EUNSUP).
 *
 * Asynchronous on `stream`. */
ATHMHD_API int athmhd_restrict(athmhd_t h, const double* fine_cons, const double* fine_bface, double* coarse_cons,
                               double* coarse_bface, int o1, int o2, int o3, void* stream);
ATHMHD_API int athmhd_prolong(athmhd_t h, const double* coarse_cons, const double* coarse_bface, double* fine_cons,
                              double* fine_bface, int o1, int o2, int o3, int primitive, void* stream);

/* The same operators on a box, for the coarse buffers and ghost zones of
 * blocks at different levels (Sec. 2.1.2, 2.1.5).  fine_lo, coarse_lo and
 * extent are host arrays of 3 ints (x1, x2, x3): fine cells
 * [fine_lo, fine_lo + 2 extent) correspond to coarse cells
 * [coarse_lo, coarse_lo + extent), in stored indices with the ghost zones
 * included (index ng is the first active cell).  athmhd_restrict_box writes
 * those coarse cells and the coarse faces of the box (upper ones included);
 * athmhd_prolong_box writes those fine cells and their faces (upper ones
 * included) and reads the coarse box plus one cell on each side.  Everything
 * touched must lie in the stored arrays, else ATHMHD_EINVAL: extent >= 1,
 * 0 <= fine_lo, fine_lo + 2 extent <= N_d (N_d = n_d + 2 nghost); for
 * restriction 0 <= coarse_lo, coarse_lo + extent <= N_d; for prolongation
 * 1 <= coarse_lo, coarse_lo + extent <= N_d - 1.  Block sizes need not be
 * even.  The octant calls above are the box fine_lo = nghost,
 * coarse_lo = nghost + o_d n_d / 2, extent = n_d / 2.  keep (prolongation;
 * 0 to 63, else ATHMHD_EINVAL): bit 2 d + S set (d = 0, 1, 2 for x1, x2, x3;
 * S = 0 lower, 1 upper side) means the fine faces of component d on that side
 * of the box already hold fine-level values, as where the fine block shares
 * the face with a fine neighbour; they are read, not overwritten, and the
 * faces inside the box are solved with them (Sec. 2.1.5), so a fine field
 * whose kept faces restrict to the coarse faces keeps the coarse divergence.
 * Other rules (handles, distinct arrays, cubic cells for prolongation,
 * primitive, the pressure floor) as above. */
ATHMHD_API int athmhd_restrict_box(athmhd_t h, const double* fine_cons, const double* fine_bface, double* coarse_cons,
                                   double* coarse_bface, const int* fine_lo, const int* coarse_lo, const int* extent,
                                   void* stream);
ATHMHD_API int athmhd_prolong_box(athmhd_t h, const double* coarse_cons, const double* coarse_bface, double* fine_cons,
                                  double* fine_bface, const int* fine_lo, const int* coarse_lo, const int* extent,
                                  int primitive, int keep, void* stream);

/* Text of the last error recorded on `h` (or of the last failed create when
 * h is NULL).  Valid until the next call on the same handle. */
ATHMHD_API const char* athmhd_last_error(athmhd_t h);

/* Release the handle and its device memory (synchronises the device). */
ATHMHD_API void athmhd_destroy(athmhd_t h);

#ifdef __cplusplus
}
#endif

#endif /* ATHMHD_H */
