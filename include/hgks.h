/*
 * hgks.h -- C ABI of the MI355X (gfx950) HGKS library: the explicit
 * high-order gas-kinetic step on tetrahedral and hexahedral meshes of arXiv
 * 2407.00656 (Wang, Cao, Pan), run in hand-written HIP kernels on one GPU.
 *
 * One step (Sec. 2.2, two-stage fourth-order "S2O4" update) is
 *   Q*      = Q^n + dt/2 L(Q^n) + dt^2/8 dL/dt(Q^n)
 *   Q^{n+1} = Q^n + dt L(Q^n) + dt^2/6 (dL/dt(Q^n) + 2 dL/dt(Q*)),
 * with L = -(1/|Omega_i|) sum_faces F S (Sec. 2.1, Eq. finite), where each face
 * flux F and its time derivative come from the gas-kinetic interface
 * distribution (Sec. 2.1, Eq. flux) evaluated at the face Gauss points on the
 * third-order WENO reconstruction of both neighbours (Sec. 2.3, Eqs. polys and
 * weno), and fitted linearly in time (Sec. 2.2, Eq. expansion-1).
 *
 * Conventions for every call:
 *  - Every function returns hgks_status (0 = HGKS_OK); no C++ exception crosses
 *    the ABI.  On failure hgks_last_error() returns a message.
 *  - Host pointers are read (or written) during the call only; the library never
 *    keeps a caller pointer.  Device memory is obtained through the allocator
 *    given at creation (hipMalloc when none is given) and freed by destroy.
 *  - Indices are 0-based.  Cell states are conservative cell averages
 *    (rho, rho U, rho V, rho W, rho E) (Sec. 2.1), row-major [n_cells][5], in the
 *    caller's cell order; the library renumbers internally and restores order.
 *  - A context is not thread-safe; use one per host thread.  All GPU work of a
 *    context is queued on its stream; step may return before the GPU finishes.
 *    Device-side failures (non-physical state) surface at the next call that
 *    synchronises (get_state, sync).
 *  - Call order: create -> mesh_upload -> init_state -> step* -> get_state.
 *    A call out of order returns HGKS_E_STATE.
 */
#ifndef HGKS_H
#define HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HGKS_ABI_VERSION 2

typedef enum {
    HGKS_OK = 0,
    HGKS_E_INVALID_ARG = 1,   /* null pointer, size out of range, unsupported option */
    HGKS_E_BAD_MESH = 2,      /* degenerate cell, non-conforming face, rank-deficient stencil */
    HGKS_E_STATE = 3,         /* call out of order */
    HGKS_E_OOM = 4,           /* device allocation failed or pool budget exceeded */
    HGKS_E_DEVICE = 5,        /* HIP runtime error */
    HGKS_E_NONPHYSICAL = 6    /* rho <= 0, p <= 0 or a non-finite value appeared */
} hgks_status;

typedef enum {
    HGKS_FP64 = 0,            /* every step in double precision */
    HGKS_FP32_MIXED = 1       /* FP64 geometry, pseudo-inverse contraction, state and
                                 accumulation; FP32 smoothness indicators, weights,
                                 Gauss-point reconstruction and gas-kinetic flux
                                 (with tau > 0, a face with a Gauss point that has a
                                 cold side, whose energy is more than 90% kinetic, or a
                                 non-finite FP32 flux is evaluated again in FP64 by a
                                 separate pass: there FP32 loses the pressure and the
                                 micro-slopes) */,
    HGKS_FP32 = 2             /* the single-precision build (Sec. 5.1, the memory and time
                                 comparison of FP32 against FP64): the state (Q^n, Q*, and
                                 the stage-2 base), the cell and face geometry, the face
                                 fluxes and the accumulators are stored in FP32, and so is
                                 the big-stencil pseudo-inverse (each value rounded once);
                                 both WENO contractions, the sub-stencil fits, the weights
                                 and the gas-kinetic flux run in FP32 (tau > 0 faces with
                                 a cold side in FP64, as in the FP32-mixed form).  The
                                 few operations of the stage update run in FP64 registers
                                 on FP32 operands and are rounded once on store; dt and the
                                 time stay FP64, and so do the centroids the sub-stencil
                                 fits are formed from.  About half the device memory of
                                 FP64 */
} hgks_precision;

typedef enum {
    HGKS_ACC_GATHER = 0,      /* per-face flux buffer, then a per-cell gather in fixed
                                 local-face order (one flux launch per stage) */
    HGKS_ACC_COLOURED = 1     /* faces split into colour classes with no shared cell;
                                 one flux launch per class adds into the cells
                                 (non-atomic read-modify-write, class order fixed) */
} hgks_accumulation;

/* Kinds of listed boundary faces (Sec. 5.2), hexahedral meshes. */
typedef enum {
    HGKS_BC_WALL = 1,         /* no-slip adiabatic wall: the ghost holds (rho, -rho U, rho E) */
    HGKS_BC_FAR = 2           /* far field: the ghost holds the Riemann-invariant state of the
                                 cell and the free stream (hgks_params.farfield) */
} hgks_bc_kind;

typedef struct {
    double gamma;             /* specific-heat ratio; internal DOF K = (5 - 3 gamma)/(gamma - 1) (Sec. 2.1) */
    double cfl;               /* dt = cfl * min_i h_i / (|U_i| + c_i), h_i = 6|Omega_i| / sum_p S_ip */
    int tau_mode;             /* 0: tau = 0 (smooth flow, f = g(1 + A t), Sec. 5.1);
                                 1: tau = tau_eps*dt + tau_C*|p_l - p_r|/(p_l + p_r)*dt;
                                 2: viscous (Sec. 5.2, hexahedral meshes): tau = mu(T0)/p0 +
                                    tau_C*|p_l - p_r|/(p_l + p_r)*dt with mu = mu_ref (T0/T_ref)^mu_exp,
                                    T = p/rho of the collided interface state */
    double tau_eps;
    double tau_C;
    double weno_eps;          /* epsilon of the WENO-Z weights (Sec. 2.3) */
    double gamma_lin;         /* linear weight of each sub-stencil; gamma_0 = 1 - M gamma_lin with M = 4
                                 sub-stencils (tetrahedra) or 8 (hexahedra) (Sec. 2.3: 0.025) */
    int precision;            /* hgks_precision */
    int accumulation;         /* hgks_accumulation */
    int reorder;              /* 1: renumber cells along a Morton curve of the centroids (default); 0: keep order */
    double mu_ref;            /* tau_mode 2: viscosity at T_ref */
    double T_ref;             /* tau_mode 2: reference temperature (T = p/rho) */
    double mu_exp;            /* tau_mode 2: exponent of the power law (Sec. 5.2: 0.7) */
    double prandtl;           /* tau_mode 2: Prandtl number; the energy flux takes (1/Pr - 1) times the
                                 heat flux of the interface distribution in the frame of the collided
                                 state's velocity (BGK alone has Pr = 1) */
    double farfield[5];       /* free stream (rho, U, V, W, p) of HGKS_BC_FAR faces */
} hgks_params;

/* Fills the defaults: gamma 1.4, cfl 0.3, tau_mode 0, tau_eps 0.05, tau_C 1,
 * weno_eps 1e-8, gamma_lin 0.025, FP64, gather accumulation, reorder 1,
 * mu_ref 0, T_ref 1, mu_exp 0.7, prandtl 1, farfield (1, 0, 0, 0, 1). */
void hgks_default_params(hgks_params *p);

typedef struct {
    /* Returns device memory of `bytes` bytes usable on `stream`, or NULL. */
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} hgks_allocator;

typedef struct hgks_ctx hgks_ctx;

/* Passed as the stream of hgks_create or hgks_pool_create: the context (pool)
 * creates a non-blocking stream of default priority for its work and destroys it
 * with itself, so that work of different contexts and pools can overlap. */
#define HGKS_OWN_STREAM ((void *)1)

/* Creates a context on HIP device `device`, queueing work on `hip_stream`
 * (a hipStream_t; NULL selects the device's null stream; HGKS_OWN_STREAM a stream
 * of its own).  `alloc` may be NULL.
 * Errors: INVALID_ARG (bad params or device), DEVICE. */
hgks_status hgks_create(const hgks_params *params, int device, void *hip_stream,
                        const hgks_allocator *alloc, hgks_ctx **out);

/*
 * Uploads a mesh (Sec. 3.1: CellNode connectivity plus node coordinates) and
 * builds, on the host, everything the step needs: faces, neighbours, the two-layer
 * WENO stencil of Algorithm 1 and the sub-stencils of Sec. 2.3, cell and face
 * geometry, the least-squares pseudo-inverses, and the renumbering; then copies
 * the packed arrays to the device.
 *   xyz         [n_nodes][3] node coordinates
 *   cell_nodes  [n_cells][nodes_per_cell] node ids.
 *               nodes_per_cell 4: tetrahedra, face p opposite node p, four
 *               sub-stencils, three Gauss points a face.
 *               nodes_per_cell 8: hexahedra (trilinear), nodes 0-3 around one face
 *               and node k+4 above node k; faces (0,1,2,3), (0,1,5,4), (1,2,6,5),
 *               (2,3,7,6), (3,0,4,7), (4,5,6,7) are the paper's faces 1..6 (1 and 6
 *               opposite), eight sub-stencils, and on each bilinear face the 2x2
 *               Gauss points with their own normals.  Hexahedral meshes take the
 *               FP64 and FP32-mixed precisions and the gather accumulation; a
 *               two-layer stencil of more than 24 cells (an edge shared by five or
 *               more cells) is refused (BAD_MESH).
 *   period      [3]: period[a] > 0 identifies x_a with x_a + period[a] (NULL = none)
 *               Tetrahedra: an axis with period 0 ends in two transmissive walls,
 *               the planes through its lowest and highest node coordinate: every
 *               face that belongs to one cell only must lie in one of them (all
 *               three nodes there).  Algorithm 1 gives such a face a ghost neighbour
 *               "according to the boundary condition"; here the ghost is the mirror
 *               image of the wall cell in the wall, holding the wall cell's state,
 *               and a ghost's neighbours are the mirror images of the wall cell's.
 *   n_bfaces, bface_nodes [n_bfaces][4], bface_kind [n_bfaces] (hgks_bc_kind):
 *               listed boundary faces of a hexahedral mesh without periodic axes
 *               (0 / NULL otherwise); every face of one cell must be listed.  The
 *               ghost across a listed face is the cell's mirror image in the face's
 *               plane, holds the ghost state of the cell (no-slip wall or far field)
 *               and has no neighbours of its own; at the face's Gauss points the
 *               right side is the ghost map of the left reconstruction (wall: the
 *               momentum negated and the gradient reflected; far field: the
 *               Riemann-invariant state of the left value, no gradient).
 * Replaces any previous mesh and state.
 * Errors: INVALID_ARG, BAD_MESH (degenerate or folded cell, a face shared by more
 * than two cells, an unshared face off the walls or not listed, a stencil reaching
 * both walls of an axis, a rank-deficient least-squares stencil), OOM, DEVICE.
 */
hgks_status hgks_mesh_upload(hgks_ctx *ctx, int64_t n_nodes, const double *xyz,
                             int64_t n_cells, int nodes_per_cell, const int64_t *cell_nodes,
                             const double *period, int64_t n_bfaces, const int64_t *bface_nodes,
                             const int32_t *bface_kind);

/* Sets the state: q [n_cells][5] conservative cell averages, caller order; t0 the time.
 * Errors: STATE (no mesh), INVALID_ARG, NONPHYSICAL (rho <= 0 or p <= 0 in q). */
hgks_status hgks_init_state(hgks_ctx *ctx, const double *q, double t0);

/* Advances nsteps S2O4 steps.  dt_fixed > 0 uses that step; otherwise each step
 * takes the CFL rule from its starting state (computed and kept on the device).
 * dt_last (nullable) receives the last step's dt, which synchronises the stream.
 * Errors: STATE, INVALID_ARG (nsteps < 0), DEVICE; NONPHYSICAL when dt_last is
 * requested and a step produced a non-physical state. */
hgks_status hgks_step_s2o4(hgks_ctx *ctx, int32_t nsteps, double dt_fixed, double *dt_last);

/* Copies the state to q_out [n_cells][5] (caller order) and the time to t_out.
 * Both are nullable; with q_out NULL only the time and the non-physical flag are
 * read back (a few bytes).  Synchronises.  Errors: STATE, NONPHYSICAL (a step went
 * non-physical; the state returned is the last one computed), DEVICE. */
hgks_status hgks_get_state(hgks_ctx *ctx, double *q_out, double *t_out);

/* Waits for the context's queued work.  Errors: DEVICE, NONPHYSICAL. */
hgks_status hgks_sync(hgks_ctx *ctx);

/* Mesh sizes after upload: cells, faces, two-layer stencil slots (16 for tetrahedra,
 * 24 for hexahedra), colour classes
 * (with HGKS_ACC_COLOURED: 4 when the cell graph is bipartite, else at most 5;
 * 1 with the gather accumulation). */
hgks_status hgks_mesh_info(const hgks_ctx *ctx, int64_t *n_cells, int64_t *n_faces,
                           int32_t *stencil_slots, int32_t *n_colours);

/* Device bytes the context holds for its mesh and state. */
hgks_status hgks_footprint(const hgks_ctx *ctx, size_t *bytes);

/* Per-kernel timing with HIP events on the context's stream (off by default).
 * kernel ids: 0 dt, 1 weno, 2 flux, 3 update.  read() synchronises and returns
 * the summed milliseconds and launch count since the last reset. */
hgks_status hgks_profile_enable(hgks_ctx *ctx, int on);
hgks_status hgks_profile_read(hgks_ctx *ctx, int kernel_id, double *ms_total, int64_t *launches);
hgks_status hgks_profile_reset(hgks_ctx *ctx);

const char *hgks_last_error(const hgks_ctx *ctx);
/* Frees the context; a context still in a pool is first removed from it (after the
 * pool's queued steps finish). */
void hgks_destroy(hgks_ctx *ctx);

/*
 * Host-only inspection of the mesh precompute (no GPU needed): builds exactly
 * what mesh_upload would build (without listed boundary faces) and reports it in
 * the library's internal order.
 *   stats [8]: n_faces, stencil slots (16 for tetrahedra, 24 for hexahedra),
 *              max distinct big-stencil members, min distinct
 *              big-stencil members, n_colours, max |pinv A - I| over all cells,
 *              max |sum_p n_p S_p| over all cells (closure), number of duplicate
 *              slots (tetrahedra)
 *   perm  [n_cells] (nullable): internal cell c holds caller cell perm[c]
 *   sten  [slots][n_cells] (nullable): slot cell ids (internal numbering); for
 *         hexahedra size it from a first call's stats[1]
 * Errors as mesh_upload.
 */
hgks_status hgks_inspect_mesh(const hgks_params *params, int64_t n_nodes, const double *xyz,
                              int64_t n_cells, int nodes_per_cell, const int64_t *cell_nodes,
                              const double *period, double *stats, int64_t *perm, int32_t *sten);

/*
 * Continuous batching (serving many solves on one GPU).  A pool owns no meshes:
 * it borrows contexts that are uploaded and initialised on the same device and
 * steps any subset of them together, one launch per phase covering every
 * slot's tiles, with each slot's own dt.  Per-cell arithmetic never depends on
 * the batch, so a slot's results are bitwise the same alone or in a mix.
 * Contexts of every precision may share a pool (their phases launch separately).
 */
typedef struct hgks_pool hgks_pool;

/* hbm_budget: admission limit on the summed footprints of the slots (0 = none).
 * hip_stream as in hgks_create (HGKS_OWN_STREAM: the pool's own stream). */
hgks_status hgks_pool_create(int device, void *hip_stream, size_t hbm_budget, hgks_pool **out);
/* Bytes a context with this mesh size will hold (used for admission; exact for a
 * periodic mesh, wall faces add 8 + 128 + 80 bytes each, 8 + 64 + 40 in the FP32 form).  HGKS_E_INVALID_ARG for
 * parameters hgks_create would reject, n_cells <= 0 or nodes_per_cell != 4. */
hgks_status hgks_pool_footprint(const hgks_params *params, int64_t n_cells, int nodes_per_cell, size_t *bytes);
/* Adds a context (mesh uploaded, state initialised); returns its slot id.  A context
 * belongs to at most one pool at a time; pools take tetrahedral contexts (a
 * hexahedral context steps on its own: INVALID_ARG).
 * Errors: STATE, INVALID_ARG (other device, already in a pool), OOM (budget exceeded). */
hgks_status hgks_pool_add(hgks_pool *pool, hgks_ctx *ctx, int *slot);
/* Advances the listed slots by nsteps S2O4 steps each (CFL dt per slot). */
hgks_status hgks_pool_step(hgks_pool *pool, const int *slots, int n, int32_t nsteps);
/*
 * hgks_pool_step with no device allocation, for callers that cannot allocate
 * device memory while stepping (tight serving loops, harnesses that forbid
 * hipMalloc).  hgks_pool_step keeps its launch tables (problem descriptors and
 * tile tables) in memory it allocates and grows; this call puts them in a static
 * array of the library, HGKS_STATIC_TABLE_BYTES (8 MiB) per GPU, held until the
 * process ends.  The tables take about 0.75 bytes a cell (one 16-byte tile per 64
 * cells and per 64 faces), so a batch may hold about 11 M cells: sixteen problems
 * of 6*48^3 cells, or five of 6*64^3.  Same kernels and results as
 * hgks_pool_step, bitwise.
 * Every call on a GPU shares that GPU's array, which holds the last call's
 * tables; a call whose tables are not the ones the array holds rewrites them,
 * waiting first for its pool's stream (and for the whole device when another
 * pool wrote the array last).  Calls from several host threads take turns on a
 * lock; steps still queued when another process-local pool rewrites the array
 * are waited for as above, so only work launched outside the library on these
 * tables could race.
 * Errors: INVALID_ARG (bad slot list, or tables larger than the static array; the
 * message is set on each listed slot's context, see hgks_last_error), DEVICE.
 */
#define HGKS_STATIC_TABLE_BYTES ((size_t)8 << 20)
hgks_status hgks_pool_step_static(hgks_pool *pool, const int *slots, int n, int32_t nsteps);
/* Releases a slot (the context stays valid and owned by the caller). */
hgks_status hgks_pool_remove(hgks_pool *pool, int slot);
hgks_status hgks_pool_used(const hgks_pool *pool, size_t *bytes, int *n_slots);
void hgks_pool_destroy(hgks_pool *pool);

#ifdef __cplusplus
}
#endif
#endif /* HGKS_H */
