// Kernel-side descriptors and launch wrappers (host interface of kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "../../include/hgks.h"

namespace hgks {

// One problem's device arrays and constants; kernels read it from a table so
// that one launch can cover the tiles of many problems (continuous batching).
struct ProbDesc {
    int32_t nc, nf;
    int32_t n_cell_tiles, pad0;
    const int32_t *sten;
    const double *pinv0;          // big-stencil pseudo-inverse, FP64 pair rows [72][nc]
    const float *pinv32;          // the same rounded to FP32 as quad rows [36][nc] (FP32 form)
    const double *cen;            // centroids [3][nc]
    const uint32_t *sshift;       // periodic image codes of the stencil slots [4][nc]
    const double *cgeo;
    const int32_t *cface;
    const int32_t *fcell;
    const double *fgeo;
    double *Q;          // state Q^n [5][nc]
    double *Qs;         // stage state Q* [5][nc]
    double *R;          // Q^n + dt L^n + dt^2/6 dL^n [5][nc]
    double *C;          // FP64 reconstruction [50][nc]
    float *C32;         // FP32 reconstruction deviation [50][nc]
    double *FF;         // face fluxes [10][nf]
    double *acc;        // coloured accumulation [10][nc]
    double *dtpart;     // per cell tile minimum of h/(|U|+c)
    double *dt;         // [0] dt of the current step
    double *time;       // [0] simulated time
    int32_t *flag;      // [0] non-physical state seen, [1] the tau = 0 flux fix-up pass has work
    double per[3];                // period per axis (0: not periodic, walls at both ends)
    double mir[3][2];             // twice the low / high wall coordinate of a non-periodic axis
                                  // (a member mirrored in a wall sits at mir - x)
    double gamma, K, weno_eps, gamma_lin, cfl, tau_eps, tau_C;
    int32_t tau_mode, mixed;
    // viscous collision time (tau_mode 2) and the free stream of far-field faces
    double mu_ref, T_ref, mu_exp, prandtl;
    double farfield[5];
    // hexahedral meshes (ns stencil slots, ng ghosts of listed boundary faces)
    int32_t ns, ng;
    const double *hpinv;          // big-stencil pseudo-inverse [9 ns][nc]
    const double *hbinv;          // sub-stencil inverses [72][nc]
    const int32_t *gcell;         // ghost -> its cell [ng]
    const int32_t *gkind;         // ghost kind (HGKS_BC_WALL / HGKS_BC_FAR) [ng]
    const double *gnrm;           // ghost face's outward mean normal [3][ng]
    double *G;                    // ghost states of the current stage [5][ng]
};

struct Tile {
    int32_t prob;   // index into the problem table
    int32_t begin;  // first cell / face of the tile
    int32_t local;  // tile index within its problem (cell tiles: dtpart slot)
    int32_t end;    // one past the last cell / face of the tile
};

constexpr int GP_FACES = 21;     // tau > 0 flux without colouring: faces per single-wave workgroup;
                                 // its face tiles hold 3 * GP_FACES = 63 faces
constexpr int WENO_TILE = 64;    // cells per WENO workgroup (5 waves: one per variable)
constexpr int UPD_TILE = 64;     // cells per update / dt workgroup

// prec: 0 FP64, 1 FP32-mixed, 2 FP32 (the hgks_precision values)
void launch_weno(const ProbDesc *probs, const Tile *tiles, int ntiles, int stage, int prec, bool walls,
                 hipStream_t s);
// prec as for launch_weno: 2 means FP32 state, geometry and face-flux storage
void launch_flux(const ProbDesc *probs, int nprobs, const Tile *tiles, int ntiles, int stage, int prec, bool tau0,
                 bool coloured, bool walls, hipStream_t s);
// s32: the FP32 form's storage (state, cell geometry, face fluxes in FP32)
void launch_update(const ProbDesc *probs, const Tile *tiles, int ntiles, int stage, bool coloured, bool s32,
                   hipStream_t s, int faces_per_cell = 4);

// Hexahedral meshes: ghost states, WENO (one wave per variable of 64 cells), the
// Gauss-point flux (tau = 0, tau > 0 shock mode, or viscous) into the per-face buffer.
constexpr int HEX_WENO_CELLS = 64;
constexpr int HEX_NS = HEX_SLOTS;    // stencil slots the WENO kernel holds (shorter stencils padded)
constexpr int HEX_FLUX_FACES = 64;   // faces per flux workgroup (four lanes a face)
void launch_hex_ghost(const ProbDesc *d, int ng, int stage, hipStream_t s);
void launch_hex_weno(const ProbDesc *d, const Tile *tiles, int ntiles, int stage, bool mixed, hipStream_t s);
void launch_hex_flux(const ProbDesc *d, const Tile *tiles, int ntiles, int stage, bool mixed, int tau_mode,
                     hipStream_t s);
void launch_dt_local(const ProbDesc *probs, const Tile *tiles, int ntiles, bool s32, hipStream_t s);
void launch_dt_final(const ProbDesc *probs, int nprobs, double dt_fixed, hipStream_t s);
void launch_fill(double *p, double v, int64_t n, hipStream_t s);

// Size of the per-GPU static launch-table array of the allocation-free pool step:
// the descriptors and tiles of a batch of about 11 M cells (0.75 bytes a cell).
constexpr size_t STATIC_TABLE_BYTES = HGKS_STATIC_TABLE_BYTES;
// Device address of that array on `device`, which must be the current device.
// Looked up once per device (the runtime call) and cached.
hipError_t static_table_ptr(int device, void **ptr);

}  // namespace hgks
