// Internal layouts shared by the host precompute, the HIP kernels and the C ABI.
//
// Device layout (everything structure-of-arrays over the internal cell / face
// numbering, so that consecutive lanes touch consecutive addresses):
//
//   sten   int32  [16][nc]       two-layer stencil slots: 0..3 the face neighbours
//                                i_1..i_4 (face p opposite node p), 4+3m..6+3m the
//                                three other neighbours of i_{m+1} (Sec. 2.3); a cell
//                                reached twice keeps both slots (the later one gets
//                                zero weight), so sub-stencil membership is static
//   pinv0  double [72][nc][2]    big-stencil pseudo-inverse, 9 rows x 16 slots;
//                                element (r, s) in pair r*8 + s/2, lane s%2
//   cen    double [3][nc]        cell centroids (the sub-stencil fits are formed on
//                                the device from them)
//   sshift uint32 [4][nc]        placement of each stencil slot: byte s%4 of word s/4
//                                holds (sx+2) + 5 (sy+2) + 25 (sz+2); on a periodic axis
//                                the member sits at its centroid + s * period, on a
//                                non-periodic axis s = -1 / +1 is its mirror image in the
//                                low / high wall (2 wall - x) and s = 0 the cell itself
//   cgeo   double [9][nc]        1/h, scaled second moments (xx,yy,zz,xy,xz,yz),
//                                1/|Omega|, h_dt = 6|Omega|/sum S
//   cface  int32  [4][nc]        (face << 1) | (cell is the face's right cell)
//   fcell  int32  [2][nf]        left, right cell of each face (normal points left->right);
//                                right = -1 at a wall face (the ghost: the left cell's
//                                mirror image, evaluated from the left cell's record)
//   fgeo   double [8][nf][2]     16 values per face as pair rows (value v in pair v/2,
//                                lane v%2): n(3), S, Gauss-point offsets from the left
//                                centroid [3][3], left minus right centroid (3; the
//                                right offsets are the left ones plus it, zero at a wall)
//   C      double [25][nc][2]    reconstruction: per variable (c0, g(3), H(6)) of
//                                P(y) = c0 + g.y + H_xx y_x^2 + ... + H_yz y_y y_z,
//                                y = x - centroid, stored as five coefficient pairs
//                                (k, k+1) per variable (FP32 pairs in the mixed form,
//                                where c0 holds the deviation from the cell mean)
//   FF     double [10][nf]       per face S * sum_G w_G (F, dF/dt); with tau = 0 the
//                                second stage stores only the dF/dt rows
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hgks.h"

namespace hgks {

constexpr int SLOTS = 16;
constexpr int NCOEF = 10;          // per variable: c0, g(3), H(6)
constexpr int CGEO = 9;
constexpr int FGEO = 16;
constexpr int CELL_TILE = 256;     // cells per workgroup (weno, update, dt)
constexpr int FACE_TILE = 64;      // faces per workgroup (flux: 3 waves, one per Gauss point)

// Sub-stencil m takes first-layer slots SUBFIRST[m][0..2] and slots 4+3m..6+3m.
// S_1 = {i1,i2,i3} + N(i1), S_2 = {i1,i2,i4} + N(i2), S_3 = {i2,i3,i4} + N(i3),
// S_4 = {i3,i1,i4} + N(i4)   (Sec. 2.3, tetrahedral sub-stencils)
constexpr int SUBFIRST[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {2, 0, 3}};

// Allocator whose value-less construct leaves trivially constructible elements
// uninitialised: resize() of the packed arrays then skips a serial zero fill of
// memory the precompute writes in full, in parallel, right after.
template <class T>
struct UninitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <class U>
    UninitAlloc(const UninitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <class T>
using hvec = std::vector<T, UninitAlloc<T>>;

struct HostMesh {
    int64_t nc = 0, nf = 0;
    std::vector<int64_t> perm;      // internal cell c holds caller cell perm[c]
    hvec<int32_t> sten;             // [16][nc]
    hvec<double> pinv0;             // [72][nc][2]
    hvec<double> cen;               // [3][nc]
    hvec<uint32_t> sshift;          // [4][nc]
    hvec<double> cgeo;              // [9][nc]
    hvec<int32_t> cface;            // [4][nc]
    hvec<int32_t> fcell;            // [2][nf]
    hvec<double> fgeo;              // [8][nf][2]
    // faces grouped by colour (coloured accumulation); colour_offsets[c]..[c+1]
    std::vector<int32_t> colour_offsets;
    // diagnostics
    int max_members = 0, min_members = 0, dup_slots = 0;
    double pinv_residual = 0.0, closure = 0.0;
    // walls of the non-periodic axes: twice the lowest / highest node coordinate
    double mir[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int64_t n_wall_faces = 0;
};

// Builds the device-ready arrays on the host.  Returns HGKS_OK or an error with `err` set.
// diagnostics: also measure max |P A - I| of the big-stencil pseudo-inverses (inspection).
hgks_status build_mesh(const hgks_params &prm, int64_t n_nodes, const double *xyz, int64_t n_cells,
                       int nodes_per_cell, const int64_t *cell_nodes, const double *period,
                       HostMesh &out, std::string &err, bool diagnostics = false);

int host_threads();

// (A^T A)^{-1} A^T of a full-column-rank m x n matrix (row-major, n = 9 or 3) through a
// Cholesky factor of A^T A; false on a negligible pivot (rank deficiency).
bool pinv_normal(int m, int n, const double *A, double *P);

// Runs f(begin, end) over [0, n) on the host threads.
void parallel_range(int64_t n, const std::function<void(int64_t, int64_t)> &f);

// Hexahedral meshes (nodes 0-3 around one face, node k+4 above node k; faces in
// the order 0 = (0,1,2,3), 1 = (0,1,5,4), 2 = (1,2,6,5), 3 = (2,3,7,6), 4 = (3,0,4,7),
// 5 = (4,5,6,7), so that faces 0 and 5 are opposite, as faces 1 and 6 of Sec. 2.3).
constexpr int HEX_FGEO = 34;       // per face: 4 x (n(3), w, y_l(3)), dlr(3), mean normal(3)
constexpr int HEX_BINV = 72;       // per cell: 8 sub-stencils x 3 x 3
// Stencil slots of a hexahedral cell: the two layers of a hexahedral lattice (6 face
// neighbours, 12 across the edges, 6 two faces away).  Shorter stencils (cells at a
// listed boundary or at an edge shared by three cells) are padded; a mesh with a
// longer one (an edge shared by five or more cells) is refused.
constexpr int HEX_SLOTS = 24;
// sub-stencils of Sec. 2.3 as face indices: S_1 = {i1,i2,i3}, ..., S_8 = {i6,i5,i2}
constexpr int HEXSUB[8][3] = {{0, 1, 2}, {0, 2, 3}, {0, 3, 4}, {0, 4, 1}, {5, 1, 2}, {5, 2, 3}, {5, 3, 4}, {5, 4, 1}};

struct HexMesh {
    int64_t nc = 0, nf = 0, ng = 0;
    int ns = 0;                     // stencil slots, HEX_SLOTS (0..5 the face neighbours in face order)
    std::vector<int64_t> perm;      // internal cell c holds caller cell perm[c]
    hvec<int32_t> sten;             // [ns][nc] member ids; id >= nc is ghost id - nc
    hvec<double> pinv;              // pair rows [9 ns / 2][nc][2]: row r, slot s at ((r ns / 2 + s / 2) nc + c) 2 + s % 2
    hvec<double> binv;              // [72][nc]: sub-stencil m, row k, member t at (m 3 + k) 3 + t
    hvec<double> cgeo;              // [9][nc] as the tetrahedral layout
    hvec<int32_t> cface;            // [6][nc] (face << 1) | (cell is the face's right cell)
    hvec<int32_t> fcell;            // [2][nf]; right = -kind at a listed boundary face
    hvec<double> fgeo;              // [34][nf]
    hvec<int32_t> gcell, gkind;     // [ng]
    hvec<double> gnrm;              // [3][ng] outward (mean) normal of the ghost's face
    // diagnostics
    int max_members = 0, min_members = 0;
    double pinv_residual = 0.0, closure = 0.0;
};

// Builds the device-ready arrays of a hexahedral mesh.  Boundary faces: listed faces
// (kinds HGKS_BC_WALL, HGKS_BC_FAR; no periodic axis then), every other face shared
// by two cells (periodic images allowed).
hgks_status build_hex_mesh(const hgks_params &prm, int64_t n_nodes, const double *xyz, int64_t n_cells,
                           const int64_t *cell_nodes, const double *period, int64_t n_bfaces,
                           const int64_t *bface_nodes, const int32_t *bface_kind, HexMesh &out, std::string &err,
                           bool diagnostics = false);

// The big-stencil pseudo-inverse rounded to FP32 in quad rows: quad row k of cell i
// holds pair rows 2k and 2k+1, out[(k * nc + i) * 4 + e] (FP32 form; multithreaded).
void pinv0_quads_f32(const HostMesh &hm, float *out);

}  // namespace hgks
