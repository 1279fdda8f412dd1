// HIP kernels of the HGKS S2O4 step for gfx950 (CDNA4, 64-lane wavefronts).
//
//   k_weno     third-order least-squares WENO per cell (Sec. 2.3).  A workgroup
//              takes WC cells: its threads first copy the cells' pseudo-inverse
//              rows into LDS (streamed from HBM once, the dominant traffic of the
//              step), then lane (v, c) forms variable v of cell c.  The non-linear
//              weights are per variable, so lanes never talk to each other.
//   k_flux_t0  gas-kinetic flux at tau = 0 (Sec. 2.1 Eq. flux, Sec. 2.2 time
//              fit, Sec. 5.1): one lane per face loads both reconstruction
//              records once, evaluates them at the three Gauss points and writes
//              S * sum_G w_G (F, dF) (dF only in the second stage, whose L(Q*)
//              the S2O4 update does not use).
//   k_flux_gp  the same for tau > 0: one lane per Gauss point, a face's three
//              lanes summed by neighbour shuffles (k_flux: the coloured mode, one
//              wave per Gauss point summed through LDS).
//   k_flux_fix, k_flux_fix_full, k_flux_hex_fix
//              rare passes over faces the main flux left non-finite (positivity
//              fallback at tau = 0; FP32 points refused to FP64 at tau > 0).
//   k_*_hex    the same steps on hexahedral meshes (eight sub-stencils, 2x2 Gauss
//              points on bilinear faces, listed wall and far-field boundaries,
//              viscous collision time).
//   k_update   S2O4 stage update (Sec. 2.2).  Each cell gathers its four (six)
//              face fluxes in a fixed order: deterministic, no atomics.  The second
//              stage also forms the next step's CFL bound per tile.
//   k_dt_*     CFL time step kept on the device.
//
// Every kernel reads its problem from a descriptor table and its range from a
// tile table, so one launch can cover many problems (continuous batching);
// the arithmetic of a cell never depends on what else is in the launch.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "hgks_internal.h"
#include "kernels.h"
#include "erfcx_table.h"

#ifndef HGKS_WENO_CELLS
#define HGKS_WENO_CELLS 16
#endif

namespace hgks {

// ----------------------------------------------------------------------------
// memory helpers: global loads / stores with a wave-uniform 64-bit base (scalar
// registers) and a 32-bit per-lane byte offset, so the compiler emits the
// "vector offset + scalar base" form of global_load / global_store instead of
// generic (flat) accesses with 64-bit per-lane address arithmetic.
// ----------------------------------------------------------------------------
struct alignas(16) d2 {
    double x, y;
};
struct alignas(8) f2 {
    float x, y;
};
struct alignas(16) f4 {
    float x, y, z, w;
};

#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ T ldg(const void *base, uint32_t off) {
    return *(gptr<const T>)((gptr<const char>)base + off);
}
template <class T>
__device__ __forceinline__ void stg(void *base, uint32_t off, const T &v) {
    *(gptr<T>)((gptr<char>)base + off) = v;
}
// Streaming load: the data is used once, so it should not displace reusable lines.
__device__ __forceinline__ d2 ldg_stream(const void *base, uint32_t off) {
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = __builtin_nontemporal_load((gptr<const v2d>)((gptr<const char>)base + off));
    return {v.x, v.y};
}
__device__ __forceinline__ f4 ldg_stream_f4(const void *base, uint32_t off) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = __builtin_nontemporal_load((gptr<const v4f>)((gptr<const char>)base + off));
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ f2 ldg_stream_f2(const void *base, uint32_t off) {
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = __builtin_nontemporal_load((gptr<const v2f>)((gptr<const char>)base + off));
    return {v.x, v.y};
}
// Streaming scalar load / store (read once, or written for a later kernel that
// gathers it): kept out of the way of the reusable lines.
template <class T>
__device__ __forceinline__ T ldg_nt(const void *base, uint32_t off) {
    return __builtin_nontemporal_load((gptr<const T>)((gptr<const char>)base + off));
}
template <class T>
__device__ __forceinline__ void stg_nt(void *base, uint32_t off, T v) {
    __builtin_nontemporal_store(v, (gptr<T>)((gptr<char>)base + off));
}
// A global load through a full per-lane address (for a select between two arrays)
template <class T>
__device__ __forceinline__ T ldg_at(const T *p) {
    return *(gptr<const T>)p;
}
#else
__device__ __forceinline__ d2 ldg_stream(const void *base, uint32_t off) {
    return *(const d2 *)((const char *)base + off);
}
__device__ __forceinline__ f4 ldg_stream_f4(const void *base, uint32_t off) {
    return *(const f4 *)((const char *)base + off);
}
__device__ __forceinline__ f2 ldg_stream_f2(const void *base, uint32_t off) {
    return *(const f2 *)((const char *)base + off);
}
template <class T>
__device__ __forceinline__ T ldg_nt(const void *base, uint32_t off) {
    return *(const T *)((const char *)base + off);
}
template <class T>
__device__ __forceinline__ void stg_nt(void *base, uint32_t off, T v) {
    *(T *)((char *)base + off) = v;
}
template <class T>
__device__ __forceinline__ T ldg_at(const T *p) {
    return *p;
}
template <class T>
__device__ __forceinline__ T ldg(const void *base, uint32_t off) {
    return *(const T *)((const char *)base + off);
}
template <class T>
__device__ __forceinline__ void stg(void *base, uint32_t off, const T &v) {
    *(T *)((char *)base + off) = v;
}
#endif

// ----------------------------------------------------------------------------
// precision helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ double hg_exp(double x) { return exp(x); }
__device__ __forceinline__ float hg_exp(float x) { return expf(x); }
__device__ __forceinline__ double hg_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float hg_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double hg_abs(double x) { return fabs(x); }
__device__ __forceinline__ float hg_abs(float x) { return fabsf(x); }
// Reciprocal and reciprocal square root.  FP64: the hardware estimate refined by
// two Newton steps, e <- 1 - x r, r <- r + r e (and the analogous step for x^-1/2),
// which leaves a few ulp of error instead of the correctly rounded result that
// costs twice the instructions.  FP32: the hardware estimate (1 ulp).
__device__ __forceinline__ double hg_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float hg_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double hg_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);     // 1 - x y^2
        y = fma(0.5 * y, e, y);                   // y (1 + e/2)
    }
    return y;
}
__device__ __forceinline__ float hg_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
// the bare hardware estimate (NaN for x < 0, infinity at 0)
__device__ __forceinline__ double hg_rsq_raw(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float hg_rsq_raw(float x) { return __builtin_amdgcn_rsqf(x); }

// Storage of the state (Q, Q*, R), the cell geometry, the face fluxes and the
// coloured accumulators: FP64, or FP32 in the FP32 form (S32).  Arrays keep their
// row layout [rows][n]; only the element size changes.  Values are handled as
// double in registers and rounded once when stored.
template <bool S32>
struct Sto {
    using E = std::conditional_t<S32, float, double>;
    static constexpr uint32_t SZ = (uint32_t)sizeof(E);
    __device__ static __forceinline__ double ld(const double *base, size_t row, uint32_t n, uint32_t i) {
        return (double)ldg<E>(reinterpret_cast<const E *>(base) + row * n, i * SZ);
    }
    __device__ static __forceinline__ void st(double *base, size_t row, uint32_t n, uint32_t i, double v) {
        stg<E>(reinterpret_cast<E *>(base) + row * n, i * SZ, (E)v);
    }
    __device__ static __forceinline__ void st_nt(double *base, size_t row, uint32_t n, uint32_t i, double v) {
        stg_nt<E>(reinterpret_cast<E *>(base) + row * n, i * SZ, (E)v);
    }
};

// erfcx(a) = exp(a^2) erfc(a) for a >= 0: Chebyshev series in t = (a - k)/(a + k),
// summed by Clenshaw's recurrence (the coefficients come from gen_erfcx_table.py).
template <class T>
__device__ __forceinline__ T erfcx_pos(T a) {
    constexpr int NT = sizeof(T) == 8 ? ERFCX_TERMS_F64 : ERFCX_TERMS_F32;
    const T t = (a - T(ERFCX_K)) * hg_rcp(a + T(ERFCX_K));
    const T t2 = t + t;
    T b1 = T(0), b2 = T(0);
#pragma unroll
    for (int j = NT - 1; j >= 1; --j) {
        const T b = fma(t2, b1, T(ERFCX_CHEB[j]) - b2);
        b2 = b1;
        b1 = b;
    }
    return fma(t, b1, T(ERFCX_CHEB[0]) - b2);
}

// ----------------------------------------------------------------------------
// WENO reconstruction
// ----------------------------------------------------------------------------
// Slot of member t (0..5) of sub-stencil m: three first-layer cells, then N(i_m).
__device__ constexpr int sub_slot(int m, int t) { return t < 3 ? SUBFIRST[m][t] : 4 + 3 * m + (t - 3); }

template <class T>
__device__ __forceinline__ T quad_form(const T M[6], T g0, T g1, T g2) {
    // g^T M g with M stored (xx, yy, zz, xy, xz, yz)
    return M[0] * g0 * g0 + M[1] * g1 * g1 + M[2] * g2 * g2 + T(2) * (M[3] * g0 * g1 + M[4] * g0 * g2 + M[5] * g1 * g2);
}

// Smoothness indicators, WENO-Z weights and the combined polynomial of one
// variable of one cell, written as five coefficient pairs.
template <class T, class PAIR, class A>
__device__ __forceinline__ void weno_combine(const ProbDesc &P, uint32_t i, uint32_t nc, double qi, const A a64[9],
                                             const A b64[4][3], const double geo[7], PAIR *C, bool store) {
    // basis order: x, y, z, xx, yy, zz, xy, xz, yz (scaled coordinates xi = (x-c)/h)
    // geo: 1/h and the six scaled second moments of the cell (cgeo rows 0..6)
    T a[9], b[4][3], M[6];
#pragma unroll
    for (int r = 0; r < 9; ++r) a[r] = (T)a64[r];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k) b[m][k] = (T)b64[m][k];
#pragma unroll
    for (int q = 0; q < 6; ++q) M[q] = (T)geo[1 + q];
    // smoothness indicators in scaled coordinates:
    //   beta_0 = sum_j mean((d_j P0)^2) + sum_{|l|=2} (d^l P0)^2,  beta_m = |grad P_m|^2
    // mean((a_j + g_j.xi)^2) = a_j^2 + g_j^T M g_j since the mean of xi is zero
    T beta[5];
    beta[0] = a[0] * a[0] + quad_form(M, T(2) * a[3], a[6], a[7]) + a[1] * a[1] + quad_form(M, a[6], T(2) * a[4], a[8]) +
              a[2] * a[2] + quad_form(M, a[7], a[8], T(2) * a[5]) +
              T(4) * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) beta[1 + m] = b[m][0] * b[m][0] + b[m][1] * b[m][1] + b[m][2] * b[m][2];
    // WENO-Z weights
    const T gl = (T)P.gamma_lin, g0 = T(1) - T(4) * gl, eps = (T)P.weno_eps;
    T tauZ = T(0.25) * (hg_abs(beta[0] - beta[1]) + hg_abs(beta[0] - beta[2]) + hg_abs(beta[0] - beta[3]) +
                        hg_abs(beta[0] - beta[4]));
    T w[5], ws = T(0);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        w[m] = (m == 0 ? g0 : gl) * (T(1) + tauZ * hg_rcp(beta[m] + eps));
        ws += w[m];
    }
    const T inv = hg_rcp(ws);
    const T s0 = w[0] * inv * hg_rcp(g0);
    T al[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) al[m] = w[1 + m] * inv - s0 * gl;
    // combined polynomial in y = x - centroid
    const T ih = (T)geo[0], ih2 = ih * ih;
    T c[10];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = (s0 * a[k] + al[0] * b[0][k] + al[1] * b[1][k] + al[2] * b[2][k] + al[3] * b[3][k]) * ih;
    T dev = T(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        T cq = s0 * a[3 + q];
        dev -= cq * M[q];
        c[4 + q] = cq * ih2;
    }
    if constexpr (sizeof(T) == 8)
        c[0] = (T)(qi + (double)dev);
    else
        c[0] = dev;  // FP32 form: deviation from the FP64 cell mean
    if (!store) return;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        PAIR pr;
        pr.x = c[2 * k];
        pr.y = c[2 * k + 1];
        stg<PAIR>(C + (size_t)k * nc, i * (uint32_t)sizeof(PAIR), pr);
    }
}

// The linear least-squares fit of sub-stencil m of cell i (Sec. 2.3), formed on the
// device: member t (slot s(m, t)) has the row a_t = (c_k + image shift - c_i)/h_i,
// the mean of the scaled linear basis over the member (the basis has zero mean over
// the cell itself), and the pseudo-inverse is (A^T A)^-1 A^T over the distinct
// members; a member met twice gets a zero column.  The 3x3 normal matrix is
// inverted through its adjugate.  out[k][t]: row k (d/dxi_k), member t.  The rows
// are formed in FP64 (differences of centroids); T is the precision of the normal
// matrix, its inverse and the result (float in the FP32 form).
// With LDSID the stencil ids, and with LDSGEO 1/h, come from the workgroup's LDS
// copy (sid, sgeo, column cs) rather than from global memory.
template <bool WALLS, int WC, bool LDSID, class T, bool LDSGEO = LDSID>
__device__ __forceinline__ void sub_stencil_pinv(const ProbDesc &P, uint32_t i, uint32_t m, const int32_t (*sid)[WC],
                                                 const double (*sgeo)[WC], uint32_t cs, T out[3][6]) {
    const size_t nc = (size_t)P.nc;
    // first-layer slots of sub-stencil m, four bits each: SUBFIRST[m][t]
    constexpr uint64_t FIRST = (uint64_t)SUBFIRST[0][0] | (uint64_t)SUBFIRST[0][1] << 4 |
                               (uint64_t)SUBFIRST[0][2] << 8 | (uint64_t)SUBFIRST[1][0] << 12 |
                               (uint64_t)SUBFIRST[1][1] << 16 | (uint64_t)SUBFIRST[1][2] << 20 |
                               (uint64_t)SUBFIRST[2][0] << 24 | (uint64_t)SUBFIRST[2][1] << 28 |
                               (uint64_t)SUBFIRST[2][2] << 32 | (uint64_t)SUBFIRST[3][0] << 36 |
                               (uint64_t)SUBFIRST[3][1] << 40 | (uint64_t)SUBFIRST[3][2] << 44;
    const double ih = LDSGEO ? sgeo[0][cs] : ldg<double>(P.cgeo, i * 8u);
    const double ci[3] = {ldg<double>(P.cen, i * 8u), ldg<double>(P.cen + nc, i * 8u), ldg<double>(P.cen + 2 * nc, i * 8u)};
    const uint32_t w0 = ldg<uint32_t>(P.sshift, i * 4u), w1 = ldg<uint32_t>(P.sshift + nc, i * 4u),
                   w2 = ldg<uint32_t>(P.sshift + 2 * nc, i * 4u), w3 = ldg<uint32_t>(P.sshift + 3 * nc, i * 4u);
    T A[6][3];
    int32_t id[6];
    uint32_t code[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const uint32_t sl = t < 3 ? (uint32_t)(FIRST >> (12 * m + 4 * t)) & 15u : 4u + 3u * m + (uint32_t)(t - 3);
        const uint32_t wsel = sl >> 2;
        const uint32_t word = wsel == 0 ? w0 : (wsel == 1 ? w1 : (wsel == 2 ? w2 : w3));
        code[t] = (word >> (8 * (sl & 3u))) & 0xFFu;
        id[t] = LDSID ? sid[sl][cs] : ldg<int32_t>(P.sten + sl * nc, i * 4u);
        const int sh[3] = {(int)(code[t] % 5u) - 2, (int)((code[t] / 5u) % 5u) - 2, (int)(code[t] / 25u) - 2};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // periodic image, or on a non-periodic axis the cell (s = 0) or its mirror in a wall
            const double c = ldg<double>(P.cen + a * nc, (uint32_t)id[t] * 8u);
            double x = c + (double)sh[a] * P.per[a];
            if constexpr (WALLS) {      // meshes without walls keep the plain periodic form
                const double mlo = P.mir[a][0], mhi = P.mir[a][1];
                if (!(P.per[a] > 0.0)) x = sh[a] == 0 ? c : (sh[a] > 0 ? mhi : mlo) - c;
            }
            A[t][a] = (T)((x - ci[a]) * ih);
        }
    }
    bool dup[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        dup[t] = false;
#pragma unroll
        for (int u = 0; u < t; ++u) dup[t] = dup[t] || (id[u] == id[t] && code[u] == code[t]);
    }
    T n00 = 0, n01 = 0, n02 = 0, n11 = 0, n12 = 0, n22 = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const T x = dup[t] ? T(0) : A[t][0], y = dup[t] ? T(0) : A[t][1], z = dup[t] ? T(0) : A[t][2];
        n00 = fma(x, x, n00); n01 = fma(x, y, n01); n02 = fma(x, z, n02);
        n11 = fma(y, y, n11); n12 = fma(y, z, n12); n22 = fma(z, z, n22);
    }
    const T c00 = n11 * n22 - n12 * n12, c01 = n02 * n12 - n01 * n22, c02 = n01 * n12 - n02 * n11;
    const T c11 = n00 * n22 - n02 * n02, c12 = n01 * n02 - n00 * n12, c22 = n00 * n11 - n01 * n01;
    const T idet = T(1) / (n00 * c00 + n01 * c01 + n02 * c02);
    const T inv[3][3] = {{c00 * idet, c01 * idet, c02 * idet},
                         {c01 * idet, c11 * idet, c12 * idet},
                         {c02 * idet, c12 * idet, c22 * idet}};
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            out[k][t] = dup[t] ? T(0) : inv[k][0] * A[t][0] + inv[k][1] * A[t][1] + inv[k][2] * A[t][2];
}

// Pseudo-inverse pair rows in LDS (FP64 forms): 72 of the big stencil (row r,
// slots 2s, 2s+1 at pair r*8+s); once the big contraction has read them, the first
// 36 take the sub-stencil fits (row k of sub-stencil m, members 2u, 2u+1 at pair
// (m*3+k)*3+u).  A workgroup handles WC cells: its threads copy the WC cells'
// big-stencil rows from HBM (streamed, each value read once) while 4 WC of them
// form the sub-stencil fits from the centroids into registers; one barrier, the big
// contraction, two barriers around the fits' LDS write, then lane (v, c) finishes
// variable v of cell c.  Five variables x WC cells are spread over whole waves;
// spare lanes only help with the copy.
constexpr int WPAIRS0 = 72;

// The (tile, part) unit of this workgroup when each 64-cell tile is split over SPLIT
// workgroups.  Workgroups go to the eight XCDs round-robin by id, and the tile table
// is laid out so that XCD x owns a contiguous run of tiles at one workgroup a tile;
// with SPLIT a tile, XCD x takes a contiguous run of (tile, part) units in cell order,
// and the tile's slot in the table is found by inverting that layout.
template <int SPLIT>
__device__ __forceinline__ void split_tile(uint32_t &kt, uint32_t &part) {
    const uint32_t nb = gridDim.x, xcd = blockIdx.x & 7u;
    const uint32_t bx = xcd * (nb >> 3) + min(xcd, nb & 7u) + (blockIdx.x >> 3);
    const uint32_t jt = bx / SPLIT, nt = nb / SPLIT;
    kt = jt;
    if (nt >= 16u) {
        const uint32_t q8 = nt >> 3, r8 = nt & 7u, big = r8 * (q8 + 1u);
        const uint32_t xx = jt < big ? jt / (q8 + 1u) : r8 + (jt - big) / q8;
        const uint32_t qq = jt < big ? jt % (q8 + 1u) : (jt - big) % q8;
        kt = 8u * qq + xx;
    }
    part = bx % SPLIT;
}

template <int WC>
constexpr int weno_threads() { return (5 * WC + 63) / 64 * 64; }

template <int PREC, int WC, bool WALLS>
__global__ __launch_bounds__(weno_threads<WC>()) void k_weno(const ProbDesc *__restrict__ probs,
                                                              const Tile *__restrict__ tiles, int stage) {
    // PREC 0: FP64; 1: FP32-mixed (FP32 from the weights on); 2: FP32 form (the
    // big-stencil pseudo-inverse arrives as FP32 quad rows, both contractions in FP32)
    constexpr bool F32 = PREC == 2;
    constexpr int NT = weno_threads<WC>();
    constexpr int SPLIT = WENO_TILE / WC;              // workgroups per cell tile
    static_assert(4 * WC <= NT, "one sub-stencil fit per thread");
    // LDS: 72 big-stencil FP64 pair rows, reused for the sub-stencil fits, then the
    // cells' stencil ids (19.5 KB at 16 cells: eight workgroups per CU); or in the
    // FP32 form 36 big-stencil FP32 quad rows + 36 sub-stencil FP32 pair rows, then
    // the cells' geometry and stencil ids.  Ids (and the FP32 form's geometry) are
    // read once per cell rather than once per variable lane, at the cost of one
    // barrier; the FP64 forms keep per-lane geometry loads, which start before the
    // barrier and need no LDS.
    constexpr int ROWS = F32 ? 36 : WPAIRS0;           // streamed rows per cell
    constexpr size_t LDS_BYTES =
        F32 ? (size_t)(36 * 16 + 36 * 8 + SLOTS * 4 + 7 * 8) * WC : (size_t)(WPAIRS0 * 16 + SLOTS * 4) * WC;
    __shared__ __attribute__((aligned(16))) char smem[LDS_BYTES];
    d2(*stage_buf)[WC] = reinterpret_cast<d2(*)[WC]>(smem);
    f4(*big32)[WC] = reinterpret_cast<f4(*)[WC]>(smem);
    f2(*sub32)[WC] = reinterpret_cast<f2(*)[WC]>(smem + 36 * 16 * WC);
    double(*sgeo)[WC] = reinterpret_cast<double(*)[WC]>(smem + (36 * 16 + 36 * 8) * WC);   // FP32 form only
    int32_t(*sid)[WC] = reinterpret_cast<int32_t(*)[WC]>(smem + (F32 ? 36 * 16 + 36 * 8 + 7 * 8 : WPAIRS0 * 16) * WC);
    uint32_t kt, part;
    split_tile<SPLIT>(kt, part);
    const Tile tl = tiles[kt];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t nc = (uint32_t)P.nc;
    const uint32_t c0 = tl.begin + part * WC;   // first cell of this workgroup
    const uint32_t last = (uint32_t)tl.end - 1;
    const d2 *p0 = reinterpret_cast<const d2 *>(P.pinv0);
    const f4 *p32 = reinterpret_cast<const f4 *>(P.pinv32);
    // 1. the cells' stencil ids (and in the FP32 form geometry), once per cell, then the
    // stream of the big-stencil pseudo-inverses of cells c0 .. c0+WC-1 (clamped to the
    // tile).  The ids are loaded first: their LDS copy then waits for them alone, not
    // for the stream behind them (the wait counter is in order).
    constexpr int IDS = (SLOTS * WC + NT - 1) / NT;
    int32_t idv[IDS];
#pragma unroll
    for (int k = 0; k < IDS; ++k) {     // (clamped rather than guarded: no branch per load)
        const uint32_t e = min(threadIdx.x + k * NT, (uint32_t)(SLOTS * WC - 1));
        idv[k] = ldg<int32_t>(P.sten + (size_t)(e / WC) * nc, min(c0 + e % WC, last) * 4u);
    }
    double gv = 0.0;
    if (F32 && threadIdx.x < 7u * WC) gv = Sto<F32>::ld(P.cgeo, threadIdx.x / WC, nc, min(c0 + threadIdx.x % WC, last));
    using SV = std::conditional_t<F32, f4, d2>;
    using DT = std::conditional_t<F32, float, double>;   // contraction precision
    constexpr int PER = (ROWS * WC + NT - 1) / NT;
    SV reg[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t e = min(threadIdx.x + k * NT, (uint32_t)(ROWS * WC - 1));
        const uint32_t row = e / WC, c = min(c0 + e % WC, last);
        if constexpr (F32)
            reg[k] = ldg_stream_f4(p32 + (size_t)row * nc, c * 16u);
        else
            reg[k] = ldg_stream(p0 + (size_t)row * nc, c * 16u);
    }
    {
#pragma unroll
        for (int k = 0; k < IDS; ++k) {
            const uint32_t e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= SLOTS * WC || e < (uint32_t)(SLOTS * WC)) sid[e / WC][e % WC] = idv[k];
        }
        if (F32 && threadIdx.x < 7u * WC) sgeo[threadIdx.x / WC][threadIdx.x % WC] = gv;
        __syncthreads();
    }
    // 2. the sub-stencil fits: thread (m, c) for m < 4.  The FP32 form stages them
    // now; the FP64 forms hold them in registers and write them over the first 36
    // big-stencil rows once the big contraction has read those (LDS for 8 rather
    // than 5 workgroups per CU)
    const bool fitter = threadIdx.x < 4u * WC;
    DT ps[3][6];
    if (fitter) {
        const uint32_t m = threadIdx.x / WC, cs = threadIdx.x % WC;
        sub_stencil_pinv<WALLS, WC, true, DT, F32>(P, min(c0 + cs, last), m, sid, sgeo, cs, ps);
        if constexpr (F32) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int u = 0; u < 3; ++u) sub32[(m * 3 + k) * 3 + u][cs] = f2{ps[k][2 * u], ps[k][2 * u + 1]};
        }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t e = threadIdx.x + k * NT;
        if ((k + 1) * NT <= ROWS * WC || e < (uint32_t)(ROWS * WC)) {
            if constexpr (F32)
                big32[e / WC][e % WC] = reg[k];
            else
                stage_buf[e / WC][e % WC] = reg[k];
        }
    }
    // 2. this lane's variable and cell; gather the stencil differences meanwhile
    const uint32_t v = threadIdx.x / WC, cl = threadIdx.x % WC;
    const bool active = v < 5u;
    const uint32_t i0 = c0 + cl;
    const bool ok = active && i0 <= last;
    const uint32_t i = min(i0, last);
    // the state: FP64, or FP32 in the FP32 form
    const double *Qb = stage == 1 ? P.Q : P.Qs;
    const uint32_t vrow = active ? v : 0u;
    double qi = 0.0, geo[7];
    DT d[SLOTS];
    if (active) {
        qi = Sto<F32>::ld(Qb, vrow, nc, i);
#pragma unroll
        for (int q = 0; q < 7; ++q) geo[q] = F32 ? sgeo[q][cl] : ldg<double>(P.cgeo + (size_t)q * nc, i * 8u);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const uint32_t j = (uint32_t)sid[s][cl];
            d[s] = (DT)(Sto<F32>::ld(Qb, vrow, nc, j) - qi);   // the difference in FP64, then rounded once
        }
    }
    __syncthreads();
    // 3. a = Pinv0 (Q_k - Q_i) on the big stencil; b^m = Pinv_m (Q_k - Q_i) on sub-stencil m
    DT a[9], b[4][3];
    if constexpr (F32) {
        if (!active) return;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f4 pp = big32[r * 4 + q][cl];
                acc = fmaf(pp.x, d[4 * q], acc);
                acc = fmaf(pp.y, d[4 * q + 1], acc);
                acc = fmaf(pp.z, d[4 * q + 2], acc);
                acc = fmaf(pp.w, d[4 * q + 3], acc);
            }
            a[r] = acc;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float acc = 0.0f;
#pragma unroll
                for (int t2 = 0; t2 < 3; ++t2) {
                    const f2 pp = sub32[(m * 3 + k) * 3 + t2][cl];
                    acc = fmaf(pp.x, d[sub_slot(m, 2 * t2)], acc);
                    acc = fmaf(pp.y, d[sub_slot(m, 2 * t2 + 1)], acc);
                }
                b[m][k] = acc;
            }
    } else {
        if (active) {
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < SLOTS / 2; ++s2) {
                    const d2 pp = stage_buf[r * 8 + s2][cl];
                    acc = fma(pp.x, d[2 * s2], acc);
                    acc = fma(pp.y, d[2 * s2 + 1], acc);
                }
                a[r] = acc;
            }
        }
        __syncthreads();   // every lane has read the big rows
        if (fitter) {
            const uint32_t m = threadIdx.x / WC, cs = threadIdx.x % WC;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int u = 0; u < 3; ++u) stage_buf[(m * 3 + k) * 3 + u][cs] = d2{ps[k][2 * u], ps[k][2 * u + 1]};
        }
        __syncthreads();
        if (!active) return;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int t2 = 0; t2 < 3; ++t2) {
                    const d2 pp = stage_buf[(m * 3 + k) * 3 + t2][cl];
                    acc = fma(pp.x, d[sub_slot(m, 2 * t2)], acc);
                    acc = fma(pp.y, d[sub_slot(m, 2 * t2 + 1)], acc);
                }
                b[m][k] = acc;
            }
    }
    if constexpr (PREC != 0)
        weno_combine<float>(P, i, nc, qi, a, b, geo, reinterpret_cast<f2 *>(P.C32) + (size_t)v * 5 * nc, ok);
    else
        weno_combine<double>(P, i, nc, qi, a, b, geo, reinterpret_cast<d2 *>(P.C) + (size_t)v * 5 * nc, ok);
}

// ----------------------------------------------------------------------------
// Maxwellian moments and the gas-kinetic flux
// ----------------------------------------------------------------------------
template <class T>
struct Mom {                 // normalised moments <u^n>, <v^n>, <w^n>, <xi^2>, <xi^4>
    T u[7], v[7], w[7], xi2, xi4;
};

// A Maxwellian state in the local frame, with the constants its micro-slope
// solve needs (no divisions there): i2l = 1/(2 lam) = p/rho.
template <class T>
struct State {
    T rho, ir, U, V, W, p, i2l, lam;
    T tl, c4, e2;            // 2 lam, 4 lam^2/(K+3), |U|^2 + (K+3)/(2 lam)
};

template <class T>
__device__ __forceinline__ State<T> make_state(const T q[5], T gam, T Kp3, T c4k) {
    State<T> s;
    s.rho = q[0];
    const T ir = hg_rcp(q[0]);
    s.ir = ir;
    s.U = q[1] * ir;
    s.V = q[2] * ir;
    s.W = q[3] * ir;
    const T q2 = s.U * s.U + s.V * s.V + s.W * s.W;
    s.p = (gam - T(1)) * (q[4] - T(0.5) * s.rho * q2);
    s.i2l = s.p * ir;
    s.lam = T(0.5) * s.rho * hg_rcp(s.p);
    s.tl = T(2) * s.lam;
    s.c4 = c4k * s.lam * s.lam;
    s.e2 = q2 + Kp3 * s.i2l;
    return s;
}

template <class T>
__device__ __forceinline__ void mom_full(T U, T i2l, T *m) {
    m[0] = T(1);
    m[1] = U;
#pragma unroll
    for (int n = 2; n < 7; ++n) m[n] = U * m[n - 1] + T(n - 1) * i2l * m[n - 2];
}

// <u^n>, n < NM, over u > 0 (sgn = +1) or u < 0 (sgn = -1) of the normalised
// Maxwellian with mean U and lam = rho / (2p), i2l = 1/(2 lam):
//   <u^0> = erfc(-sgn sqrt(lam) U)/2,  <u^1> = U <u^0> + sgn exp(-lam U^2)/(2 sqrt(pi lam)),
//   <u^n> = U <u^(n-1)> + (n-1)/(2 lam) <u^(n-2)>.
// erfc(z) = exp(-z^2) erfcx(|z|) for z >= 0 and 2 - exp(-z^2) erfcx(|z|) for z < 0,
// so one exponential serves both of the first two moments.
template <class T, int NM>
__device__ __forceinline__ void mom_half(T U, T lam, T i2l, T sgn, T *m) {
    const T rs = hg_rsqrt(lam);                       // 1/sqrt(lam)
    const T x = lam * rs * U;                         // sqrt(lam) U
    const T e = hg_exp(-lam * U * U);
    const T ee = e * erfcx_pos(hg_abs(x));
    m[0] = T(0.5) * (sgn * x <= T(0) ? ee : T(2) - ee);
    m[1] = U * m[0] + sgn * e * (T(0.28209479177387814347) * rs);   // 1/(2 sqrt(pi))
#pragma unroll
    for (int n = 2; n < NM; ++n) m[n] = U * m[n - 1] + T(n - 1) * i2l * m[n - 2];
}

// <u^P v^Q w^R (a.psi) psi>, psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2)
template <class T, int P, int Q, int R>
__device__ __forceinline__ void apsi(const Mom<T> &M, const T a[5], T out[5]) {
    auto B = [&](int p, int q, int r) { return M.u[p] * M.v[q] * M.w[r]; };
    auto G = [&](int p, int q, int r) {
        return a[0] * B(p, q, r) + a[1] * B(p + 1, q, r) + a[2] * B(p, q + 1, r) + a[3] * B(p, q, r + 1) +
               T(0.5) * a[4] * (B(p + 2, q, r) + B(p, q + 2, r) + B(p, q, r + 2) + B(p, q, r) * M.xi2);
    };
    auto Gx = [&](int p, int q, int r) {  // the same with an extra factor xi^2
        return M.xi2 * (a[0] * B(p, q, r) + a[1] * B(p + 1, q, r) + a[2] * B(p, q + 1, r) + a[3] * B(p, q, r + 1)) +
               T(0.5) * a[4] * (M.xi2 * (B(p + 2, q, r) + B(p, q + 2, r) + B(p, q, r + 2)) + M.xi4 * B(p, q, r));
    };
    out[0] = G(P, Q, R);
    out[1] = G(P + 1, Q, R);
    out[2] = G(P, Q + 1, R);
    out[3] = G(P, Q, R + 1);
    out[4] = T(0.5) * (G(P + 2, Q, R) + G(P, Q + 2, R) + G(P, Q, R + 2) + Gx(P, Q, R));
}

// <u psi>
template <class T>
__device__ __forceinline__ void u_psi(const Mom<T> &M, T out[5]) {
    out[0] = M.u[1];
    out[1] = M.u[2];
    out[2] = M.u[1] * M.v[1];
    out[3] = M.u[1] * M.w[1];
    out[4] = T(0.5) * (M.u[3] + M.u[1] * (M.v[2] + M.w[2] + M.xi2));
}

// Solve <(a.psi) psi> = b for a: closed form of the 5x5 moment system.
template <class T>
__device__ __forceinline__ void slope(const T b[5], const State<T> &s, T a[5]) {
    const T R1 = b[1] - s.U * b[0], R2 = b[2] - s.V * b[0], R3 = b[3] - s.W * b[0];
    const T R4 = T(2) * b[4] - s.e2 * b[0];
    a[4] = s.c4 * (R4 - T(2) * (s.U * R1 + s.V * R2 + s.W * R3));
    a[1] = s.tl * R1 - s.U * a[4];
    a[2] = s.tl * R2 - s.V * a[4];
    a[3] = s.tl * R3 - s.W * a[4];
    a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - T(0.5) * a[4] * s.e2;
}

// Time-integral weights q0..q5 of Eq. (flux) over [0, d].
template <class T>
__device__ __forceinline__ void q_coef(T d, T tau, T E, T q[6]) {
    // E = exp(-d / tau), passed in: the weights over [0, dt] and [0, dt/2] share one
    // exponential (exp(-dt/tau) = exp(-dt/(2 tau))^2)
    if (tau == T(0)) {
        q[0] = d; q[1] = T(0); q[2] = T(0.5) * d * d; q[3] = T(0); q[4] = T(0); q[5] = T(0);
        return;
    }
    q[0] = d - tau * (T(1) - E);
    q[1] = T(2) * tau * tau - tau * d - tau * (d + T(2) * tau) * E;
    q[2] = T(0.5) * d * d - tau * d + tau * tau * (T(1) - E);
    q[3] = tau * (T(1) - E);
    q[4] = -T(2) * tau * tau + tau * (d + T(2) * tau) * E;
    q[5] = -tau * tau * (T(1) - E);
}

// Local frame (n, t1, t2): t1 = n x e* / |n x e*| with e* the axis least aligned with n.
template <class T>
__device__ __forceinline__ void frame(const T n[3], T t1[3], T t2[3]) {
    const T ax = hg_abs(n[0]), ay = hg_abs(n[1]), az = hg_abs(n[2]);
    if (ax <= ay && ax <= az) {
        const T s = hg_rsqrt(n[1] * n[1] + n[2] * n[2]);
        t1[0] = T(0); t1[1] = n[2] * s; t1[2] = -n[1] * s;
    } else if (ay <= az) {
        const T s = hg_rsqrt(n[0] * n[0] + n[2] * n[2]);
        t1[0] = -n[2] * s; t1[1] = T(0); t1[2] = n[0] * s;
    } else {
        const T s = hg_rsqrt(n[0] * n[0] + n[1] * n[1]);
        t1[0] = n[1] * s; t1[1] = -n[0] * s; t1[2] = T(0);
    }
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

template <class T>
__device__ __forceinline__ void rot_in(const T q[5], const T n[3], const T t1[3], const T t2[3], T o[5]) {
    o[0] = q[0];
    o[1] = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    o[2] = q[1] * t1[0] + q[2] * t1[1] + q[3] * t1[2];
    o[3] = q[1] * t2[0] + q[2] * t2[1] + q[3] * t2[2];
    o[4] = q[4];
}

template <class T>
__device__ __forceinline__ void rot_out(const T f[5], const T n[3], const T t1[3], const T t2[3], T o[5]) {
    o[0] = f[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) o[1 + a] = f[1] * n[a] + f[2] * t1[a] + f[3] * t2[a];
    o[4] = f[4];
}

// Directional derivative of the five (global-frame) variables along e, rotated into the frame.
template <class T>
__device__ __forceinline__ void dir_deriv(const T g[5][3], const T e[3], const T n[3], const T t1[3], const T t2[3],
                                          T scale, T o[5]) {
    T d[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) d[q] = (g[q][0] * e[0] + g[q][1] * e[1] + g[q][2] * e[2]) * scale;
    rot_in(d, n, t1, t2, o);
}

// tau = 0 (smooth flow, Sec. 5.1): f = g0 (1 + A t) with g0 the Maxwellian of the
// collided state Q0.  Its moments are exactly those of the Euler equations at Q0:
//   F^n  = rho0 <u_n psi>_0           = F_Euler,n(Q0)
//   dF^n = rho0 <u_n (A.psi) psi>_0   = dF_Euler,n/dQ (Q0) . Q_t,
//   Q_t  = rho0 <(A.psi) psi>_0       = -sum_j dF_Euler,j/dQ (Q0) . dQ0/dx_j,
// because A g0 is the time derivative of g0 once <a.u + A> = 0 fixes A, and the
// micro-slopes of g0 represent dQ0/dx_j = (dQ_l + dQ_r)/2.  Only the collision
// itself needs the half-space moments, and those only along the face normal, so
// the whole evaluation stays in the global frame: the tangential velocity of each
// side is carried by its Maxwellian unchanged.

// A side's state in the global frame with the velocity component along n.
template <class T>
struct SideG {
    T rho, u[3], q2, i2l, lam, un;
};

template <class T>
__device__ __forceinline__ SideG<T> side_state(const T q[5], const T n[3], T gm1) {
    SideG<T> s;
    s.rho = q[0];
    const T ir = hg_rcp(q[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) s.u[a] = q[1 + a] * ir;
    s.q2 = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    const T p = gm1 * (q[4] - T(0.5) * s.rho * s.q2);
    s.i2l = p * ir;
    // lam <= 0 (p <= 0 with rho > 0) makes the half-space moments NaN; rho <= 0 is
    // sent the same way (0 * rho^-1/2 is NaN for rho <= 0), so every non-physical
    // side yields a non-finite flux
    s.lam = T(0.5) * s.rho * hg_rcp(p) + T(0) * hg_rsq_raw(s.rho);
    s.un = s.u[0] * n[0] + s.u[1] * n[1] + s.u[2] * n[2];
    return s;
}

// d F_Euler,d / dQ (Q0) . v for the direction d (|d| = 1), with u, |u|^2, H of Q0.
template <class T>
__device__ __forceinline__ void euler_jvp_dir(const T d[3], T gm1, const T u[3], T u2, T H, const T v[5], T out[5]) {
    const T uv = u[0] * v[1] + u[1] * v[2] + u[2] * v[3];
    const T dp = gm1 * (v[4] - uv + T(0.5) * u2 * v[0]);
    const T vmd = v[1] * d[0] + v[2] * d[1] + v[3] * d[2];
    const T ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    out[0] = vmd;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[1 + a] = u[a] * vmd + ud * (v[1 + a] - u[a] * v[0]) + d[a] * dp;
    out[4] = (v[4] + dp) * ud + H * (vmd - ud * v[0]);
}

// The same along coordinate axis j.
template <class T>
__device__ __forceinline__ void euler_jvp_axis(int j, T gm1, const T u[3], T u2, T H, const T v[5], T out[5]) {
    const T uv = u[0] * v[1] + u[1] * v[2] + u[2] * v[3];
    const T dp = gm1 * (v[4] - uv + T(0.5) * u2 * v[0]);
    const T vmj = v[1 + j], uj = u[j];
    out[0] = vmj;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[1 + a] = u[a] * vmj + uj * (v[1 + a] - u[a] * v[0]) + (a == j ? dp : T(0));
    out[4] = (v[4] + dp) * uj + H * (vmj - uj * v[0]);
}

template <class T>
__device__ __forceinline__ void gks_flux_tau0(const T ql[5], const T qr[5], const T gsum[5][3], const T n[3],
                                              const ProbDesc &P, T F[5], T dF[5]) {
    const T K = (T)P.K, gam = (T)P.gamma, gm1 = gam - T(1);
    const SideG<T> sl = side_state(ql, n, gm1), sr = side_state(qr, n, gm1);
    T ml[3], mr[3];
    mom_half<T, 3>(sl.un, sl.lam, sl.i2l, T(1), ml);
    mom_half<T, 3>(sr.un, sr.lam, sr.i2l, T(-1), mr);
    // Q0 = int_{u_n>0} psi g_l + int_{u_n<0} psi g_r
    const T wl = sl.rho * ml[0], wr = sr.rho * mr[0];
    const T rho0 = wl + wr;
    const T sn = sl.rho * (ml[1] - sl.un * ml[0]) + sr.rho * (mr[1] - sr.un * mr[0]);
    T mom0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) mom0[a] = wl * sl.u[a] + wr * sr.u[a] + sn * n[a];
    const T E0 = T(0.5) * (sl.rho * ml[2] + wl * (sl.q2 - sl.un * sl.un + (K + T(2)) * sl.i2l) +
                           sr.rho * mr[2] + wr * (sr.q2 - sr.un * sr.un + (K + T(2)) * sr.i2l));
    const T ir0 = hg_rcp(rho0);
    const T u0[3] = {mom0[0] * ir0, mom0[1] * ir0, mom0[2] * ir0};
    const T u20 = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
    const T p0 = gm1 * (E0 - T(0.5) * rho0 * u20);
    const T H0 = (E0 + p0) * ir0;
    // Q_t = -sum_j A_j dQ0/dx_j
    T Qt[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T d0[5], jv[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) d0[q] = T(0.5) * gsum[q][j];
        euler_jvp_axis(j, gm1, u0, u20, H0, d0, jv);
#pragma unroll
        for (int q = 0; q < 5; ++q) Qt[q] -= jv[q];
    }
    const T un0 = u0[0] * n[0] + u0[1] * n[1] + u0[2] * n[2];
    F[0] = rho0 * un0;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[1 + a] = F[0] * u0[a] + p0 * n[a];
    F[4] = (E0 + p0) * un0;
    euler_jvp_dir(n, gm1, u0, u20, H0, Qt, dF);
}

// Derivative of the second-moment flux rho <u_n u_a psi> of a Maxwellian along
// the conservative perturbation D_a = dQ0/dx_a, summed over the three axes a:
//   S = sum_a rho <u_n u_a (abar_a.psi) psi>_0
// because abar_a.psi g0 is the derivative of g0 along x_a.  With theta = p/rho the
// Gaussian moments are
//   rho <u_n u_a>       = rho (U_n U_a + theta n_a)
//   rho <u_n u_a u_c>   = rho (U_n U_a U_c + theta (U_n d_ac + U_a n_c + U_c n_a))
//   rho <u_n u_a psi_4> = rho/2 (U_n U_a (|U|^2 + (K+7) theta) + n_a (theta |U|^2 + (K+5) theta^2)),
// and the product rule with rho dU = D_m - U D_0, rho dtheta = dp - theta D_0 gives the
// derivative without a division.  gsum holds dQ_l/dx_a + dQ_r/dx_a (D_a is half of it).
template <class T>
__device__ __forceinline__ void second_moment_jvp(const T n[3], const T U[3], T U2, T th, T K, T gm1,
                                                  const T gsum[5][3], T S[5]) {
    const T Un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
    const T W = U2 + (K + T(7)) * th, Z = th * U2 + (K + T(5)) * th * th;
#pragma unroll
    for (int q = 0; q < 5; ++q) S[q] = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T D0 = T(0.5) * gsum[0][a], D4 = T(0.5) * gsum[4][a];
        T m[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) m[c] = T(0.5) * gsum[1 + c][a] - U[c] * D0;        // rho dU
        const T Um = U[0] * m[0] + U[1] * m[1] + U[2] * m[2];
        // rho dtheta = dp - theta D0, dp = (gamma-1)(D4 - U.D_m + |U|^2 D0 / 2) = (gamma-1)(D4 - U.m - |U|^2 D0 / 2)
        const T tp = gm1 * (D4 - Um - T(0.5) * U2 * D0) - th * D0;
        const T mn = m[0] * n[0] + m[1] * n[1] + m[2] * n[2];
        const T Ua = U[a], ma = m[a], na = n[a];
        S[0] += D0 * (Un * Ua + th * na) + (mn * Ua + Un * ma + tp * na);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T lin = (c == a ? Un : T(0)) + Ua * n[c] + U[c] * na;
            const T dlin = (c == a ? mn : T(0)) + ma * n[c] + m[c] * na;
            S[1 + c] += D0 * (Un * Ua * U[c] + th * lin) +
                        ((mn * Ua + Un * ma) * U[c] + Un * Ua * m[c] + tp * lin + th * dlin);
        }
        const T dW = T(2) * Um + (K + T(7)) * tp;
        const T dZ = tp * U2 + T(2) * th * Um + T(2) * (K + T(5)) * th * tp;
        S[4] += T(0.5) * (D0 * (Un * Ua * W + na * Z) + (mn * Ua + Un * ma) * W + Un * Ua * dW + na * dZ);
    }
}

// One initial (left or right) part of Eq. (flux) in the local frame: the half-space
// integrals of u psi g_k (1 + spatial and temporal micro-slopes), returned as
//   e0 = <u psi>,  e1 = sum_j <u u_j (a_j.psi) psi>,  e2 = <u (A.psi) psi>
// over u > 0 (sgn = +1, the left state) or u < 0 (sgn = -1).  The time slope A
// follows from <a_1 u + a_2 v + a_3 w + A> = 0, i.e. rho <(A.psi) psi> = -sum_j
// dF_j/dQ dQ/dx_j (Euler Jacobians along the frame axes).
template <class T, bool WMOM = false>
__device__ __forceinline__ void initial_part(const T Qf[5], const T g[5][3], const T n[3], const T t1[3],
                                             const T t2[3], T h0, T h1, T K, T gam, T Kp3, T c4k, T e0[5], T e1[5],
                                             T e2[5], const T *u0l = nullptr, T h2 = T(0), T *sw = nullptr) {
    const State<T> s = make_state(Qf, gam, Kp3, c4k);
    const T *e[3] = {n, t1, t2};
    const T u[3] = {s.U, s.V, s.W};
    const T u2 = s.U * s.U + s.V * s.V + s.W * s.W;
    const T H = (Qf[4] + s.p) * s.ir;
    T a[3][5], bt[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T d[5], b[5], jv[5];
        dir_deriv(g, e[j], n, t1, t2, T(1), d);
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = d[q] * s.ir;
        slope(b, s, a[j]);
        euler_jvp_axis(j, gam - T(1), u, u2, H, b, jv);
#pragma unroll
        for (int q = 0; q < 5; ++q) bt[q] -= jv[q];
    }
    T A[5];
    slope(bt, s, A);
    // half-space moments of u: the first two come from the collision (same side, same
    // normal velocity), the rest from the recursion
    Mom<T> M;
    M.u[0] = h0;
    M.u[1] = h1;
#pragma unroll
    for (int k = 2; k < 7; ++k) M.u[k] = s.U * M.u[k - 1] + T(k - 1) * s.i2l * M.u[k - 2];
    mom_full(s.V, s.i2l, M.v);
    mom_full(s.W, s.i2l, M.w);
    M.xi2 = K * s.i2l;
    M.xi4 = K * (K + T(2)) * s.i2l * s.i2l;
    T t[5];
    u_psi(M, e0);
    apsi<T, 2, 0, 0>(M, a[0], e1);
    apsi<T, 1, 1, 0>(M, a[1], t);
#pragma unroll
    for (int k = 0; k < 5; ++k) e1[k] += t[k];
    apsi<T, 1, 0, 1>(M, a[2], t);
#pragma unroll
    for (int k = 0; k < 5; ++k) e1[k] += t[k];
    apsi<T, 1, 0, 0>(M, A, e2);
    if constexpr (WMOM) {
        // the same three pieces without the factor u, the conserved moments
        //   w0 = <psi>,  w1 = sum_j <u_j (a_j.psi) psi>,  w2 = <(A.psi) psi>,
        // each contracted at once to w_E - U0.w_m + |U0|^2/2 w_rho (U0 in this frame:
        // u0l), the only combination the heat flux takes
        auto con = [&](const T w[5]) { return w[4] - (u0l[0] * w[1] + u0l[1] * w[2] + u0l[2] * w[3]) + h2 * w[0]; };
        T w[5];
        w[0] = M.u[0];
        w[1] = M.u[1];
        w[2] = M.u[0] * M.v[1];
        w[3] = M.u[0] * M.w[1];
        w[4] = T(0.5) * (M.u[2] + M.u[0] * (M.v[2] + M.w[2] + M.xi2));
        sw[0] = con(w);
        apsi<T, 1, 0, 0>(M, a[0], w);
        sw[1] = con(w);
        apsi<T, 0, 1, 0>(M, a[1], w);
        sw[1] += con(w);
        apsi<T, 0, 0, 1>(M, a[2], w);
        sw[1] += con(w);
        apsi<T, 0, 0, 0>(M, A, w);
        sw[2] = con(w);
    }
}

// General collision time (Eq. flux with tau > 0): the equilibrium part and both
// initial (left / right) parts, fitted linearly in time over [0, dt].
//   * Equilibrium part, in the global frame: rho0 <u psi>_0 is the Euler flux of Q0,
//     rho0 <u (Abar.psi) psi>_0 its time derivative through the Euler Jacobians
//     (as at tau = 0), and rho0 sum_j <u u_j (abar_j.psi) psi>_0 the derivative of
//     the second-moment flux (second_moment_jvp); the micro-slopes of g0 are never
//     formed.  The sum over the frame directions j equals the sum over the axes.
//   * Initial parts, in the local frame (n, t1, t2), where the half-space moments
//     factorise (initial_part).
//   * VISC (tau_mode 2): tau = mu(T0)/p0 + the pressure-jump term with the power-law
//     viscosity of the collided state, and for Pr != 1 the energy flux takes
//     (1/Pr - 1) times the heat flux of the interface distribution in the frame of
//     U0: q = F_E - U0.F_m + |U0|^2/2 F_rho - U0.n (W_E - U0.W_m + |U0|^2/2 W_rho), with
//     W the distribution's conserved moments (time-fitted like F): the equilibrium
//     part's are Q0 and its time derivative (the u_j-weighted slope term is -Q_t),
//     the initial parts' come from their half-space moments.
template <class T, bool VISC = false>
__device__ __forceinline__ void gks_flux_full(const T ql[5], const T gl[5][3], const T qr[5], const T gr[5][3],
                                              const T n[3], T dt, const ProbDesc &P, T F[5], T dF[5]) {
    const T K = (T)P.K, Kp3 = K + T(3), gam = (T)P.gamma, gm1 = gam - T(1), c4k = T(4) / Kp3;
    const SideG<T> sl = side_state(ql, n, gm1), sr = side_state(qr, n, gm1);
    const T pl = sl.rho * sl.i2l, pr = sr.rho * sr.i2l;
    // collision: Q0 = int_{u_n>0} psi g_l + int_{u_n<0} psi g_r (normal moments only)
    T ml[3], mr[3];
    mom_half<T, 3>(sl.un, sl.lam, sl.i2l, T(1), ml);
    mom_half<T, 3>(sr.un, sr.lam, sr.i2l, T(-1), mr);
    const T wl = sl.rho * ml[0], wr = sr.rho * mr[0];
    const T rho0 = wl + wr;
    const T sn = sl.rho * (ml[1] - sl.un * ml[0]) + sr.rho * (mr[1] - sr.un * mr[0]);
    T mom0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) mom0[a] = wl * sl.u[a] + wr * sr.u[a] + sn * n[a];
    const T E0 = T(0.5) * (sl.rho * ml[2] + wl * (sl.q2 - sl.un * sl.un + (K + T(2)) * sl.i2l) +
                           sr.rho * mr[2] + wr * (sr.q2 - sr.un * sr.un + (K + T(2)) * sr.i2l));
    const T ir0 = hg_rcp(rho0);
    const T u0[3] = {mom0[0] * ir0, mom0[1] * ir0, mom0[2] * ir0};
    const T u20 = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
    const T p0 = gm1 * (E0 - T(0.5) * rho0 * u20);
    const T H0 = (E0 + p0) * ir0;
    // time-integral weights: F = (4 I(dt/2) - I(dt)) / dt, dF = 4 (I(dt) - 2 I(dt/2)) / dt^2
    T tau = T(0);
    if (P.tau_mode == 1) tau = (T)P.tau_eps * dt + (T)P.tau_C * hg_abs(pl - pr) / (pl + pr) * dt;
    if constexpr (VISC)   // mu_ref (T0/T_ref)^mu_exp as exp(mu_exp log(T0/T_ref)): no library call
        tau = (T)P.mu_ref * hg_exp((T)P.mu_exp * log(p0 * ir0 / (T)P.T_ref)) / p0 +
              (T)P.tau_C * hg_abs(pl - pr) / (pl + pr) * dt;
    T q1[6], qh[6], cF[6], cD[6];
    const T Eh = tau > T(0) ? hg_exp(T(-0.5) * dt / tau) : T(0);
    q_coef(dt, tau, Eh * Eh, q1);
    q_coef(T(0.5) * dt, tau, Eh, qh);
    const T idt = T(1) / dt;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        cF[k] = (T(4) * qh[k] - q1[k]) * idt;
        cD[k] = T(4) * (q1[k] - T(2) * qh[k]) * idt * idt;
    }
    T gsum[5][3];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) gsum[q][a] = gl[q][a] + gr[q][a];
    // equilibrium part
    T Qt[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T d0[5], jv[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) d0[q] = T(0.5) * gsum[q][j];
        euler_jvp_axis(j, gm1, u0, u20, H0, d0, jv);
#pragma unroll
        for (int q = 0; q < 5; ++q) Qt[q] -= jv[q];
    }
    T Fe[5], Ft[5], Se[5];
    const T un0 = u0[0] * n[0] + u0[1] * n[1] + u0[2] * n[2];
    Fe[0] = rho0 * un0;
#pragma unroll
    for (int a = 0; a < 3; ++a) Fe[1 + a] = Fe[0] * u0[a] + p0 * n[a];
    Fe[4] = (E0 + p0) * un0;
    euler_jvp_dir(n, gm1, u0, u20, H0, Qt, Ft);
    second_moment_jvp(n, u0, u20, p0 * ir0, K, gm1, gsum, Se);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        F[k] = cF[0] * Fe[k] + cF[1] * Se[k] + cF[2] * Ft[k];
        dF[k] = cD[0] * Fe[k] + cD[1] * Se[k] + cD[2] * Ft[k];
    }
    const T h2 = T(0.5) * u20;
    T SW = T(0), dSW = T(0);
    if constexpr (VISC) {
        // the equilibrium part's conserved moments for the heat flux: Q0, and Q_t through
        // the slope and time terms (the u_j-weighted slope term integrates to -Q_t),
        // contracted here so that Q0 and Q_t need not stay live
        auto con = [&](T r, T m0, T m1, T m2, T e) { return e - (u0[0] * m0 + u0[1] * m1 + u0[2] * m2) + h2 * r; };
        const T cq0 = con(rho0, mom0[0], mom0[1], mom0[2], E0), cqt = con(Qt[0], Qt[1], Qt[2], Qt[3], Qt[4]);
        SW = cF[0] * cq0 + (cF[2] - cF[1]) * cqt;
        dSW = cD[0] * cq0 + (cD[2] - cD[1]) * cqt;
    }
    // initial parts, local frame
    T t1[3], t2[3];
    frame(n, t1, t2);
    const T u0l[3] = {un0, u0[0] * t1[0] + u0[1] * t1[1] + u0[2] * t1[2], u0[0] * t2[0] + u0[1] * t2[1] + u0[2] * t2[2]};
    T Fl[5], dFl[5];
    {
        T Qf[5], e0[5], e1[5], e2[5], sw[3];
        rot_in(ql, n, t1, t2, Qf);
        initial_part<T, VISC>(Qf, gl, n, t1, t2, ml[0], ml[1], K, gam, Kp3, c4k, e0, e1, e2, u0l, h2, sw);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            Fl[k] = sl.rho * (cF[3] * e0[k] + cF[4] * e1[k] + cF[5] * e2[k]);
            dFl[k] = sl.rho * (cD[3] * e0[k] + cD[4] * e1[k] + cD[5] * e2[k]);
        }
        if constexpr (VISC) {
            SW += sl.rho * (cF[3] * sw[0] + cF[4] * sw[1] + cF[5] * sw[2]);
            dSW += sl.rho * (cD[3] * sw[0] + cD[4] * sw[1] + cD[5] * sw[2]);
        }
    }
    {
        T Qf[5], e0[5], e1[5], e2[5], sw[3];
        rot_in(qr, n, t1, t2, Qf);
        initial_part<T, VISC>(Qf, gr, n, t1, t2, mr[0], mr[1], K, gam, Kp3, c4k, e0, e1, e2, u0l, h2, sw);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            Fl[k] += sr.rho * (cF[3] * e0[k] + cF[4] * e1[k] + cF[5] * e2[k]);
            dFl[k] += sr.rho * (cD[3] * e0[k] + cD[4] * e1[k] + cD[5] * e2[k]);
        }
        if constexpr (VISC) {
            SW += sr.rho * (cF[3] * sw[0] + cF[4] * sw[1] + cF[5] * sw[2]);
            dSW += sr.rho * (cD[3] * sw[0] + cD[4] * sw[1] + cD[5] * sw[2]);
        }
    }
    T Fg[5], dFg[5];
    rot_out(Fl, n, t1, t2, Fg);
    rot_out(dFl, n, t1, t2, dFg);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        F[k] += Fg[k];
        dF[k] += dFg[k];
    }
    if constexpr (VISC) {
        if (P.prandtl != 1.0) {
            const T qh = F[4] - (u0[0] * F[1] + u0[1] * F[2] + u0[2] * F[3]) + h2 * F[0] - un0 * SW;
            const T dqh = dF[4] - (u0[0] * dF[1] + u0[1] * dF[2] + u0[2] * dF[3]) + h2 * dF[0] - un0 * dSW;
            const T cpr = T(1) / (T)P.prandtl - T(1);
            F[4] += cpr * qh;
            dF[4] += cpr * dqh;
        }
    }
}

// At a wall face the ghost side is the wall cell's reconstruction mirrored in the
// wall: at the (in-wall) Gauss point the same value and the gradient reflected,
// g - 2 (g.n) n.  Where only the sum of both sides' gradients is kept (2 g after
// adding the wall cell's gradient twice), the reflection removes its normal part.
template <class T>
__device__ __forceinline__ void reflect_grad(T g[5][3], const T n[3], T times) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const T gn = times * (g[v][0] * n[0] + g[v][1] * n[1] + g[v][2] * n[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) g[v][a] -= gn * n[a];
    }
}

// Positivity fallback (not in the paper, which has no limiter): at a Gauss point
// where the reconstructed state of either side has rho <= 0 or p <= 0, the point
// is first order: both gradients are zero and each non-physical side takes its
// cell average.  It acts only at strong discontinuities.
template <class T>
__device__ __forceinline__ bool physical_point(const T q[5]) {
    // p > 0  <=>  2 rho E > |rho u|^2 (for rho > 0); no division needed
    return q[0] > T(0) && T(2) * q[0] * q[4] > q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
}

template <class T>
__device__ __forceinline__ bool finite_flux(const T F[5], const T dF[5]) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) s += F[k] * T(0) + dF[k] * T(0);   // NaN for any non-finite entry
    return s == T(0);
}

template <class T, bool S32 = false>
__device__ __forceinline__ void cell_mean(const ProbDesc &P, int stage, uint32_t c, T q[5]) {
    const double *Qa = stage == 1 ? P.Q : P.Qs;
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = (T)Sto<S32>::ld(Qa, v, (uint32_t)P.nc, c);
}

// Value and gradient of a cell's reconstruction at offset y from its centroid;
// ADD accumulates the gradient into g (tau = 0 needs only the sum of both sides).
// REC32: the records are the FP32-mixed ones (FP32 coefficients, c0 the deviation from
// the FP64 cell mean); they may be evaluated in FP64 (T = double).
template <class T, bool ADD, bool REC32 = (sizeof(T) == 4), bool S32 = false>
__device__ __forceinline__ void recon_point(const ProbDesc &P, int stage, uint32_t c, const T y[3], T q[5], T g[5][3]) {
    const uint32_t nc = (uint32_t)P.nc;
    const T yy[6] = {y[0] * y[0], y[1] * y[1], y[2] * y[2], y[0] * y[1], y[0] * y[2], y[1] * y[2]};
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        T cf[10];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if constexpr (!REC32) {
                const d2 pr = ldg<d2>(reinterpret_cast<const d2 *>(P.C) + (size_t)(v * 5 + k) * nc, c * 16u);
                cf[2 * k] = pr.x;
                cf[2 * k + 1] = pr.y;
            } else {
                const f2 pr = ldg<f2>(reinterpret_cast<const f2 *>(P.C32) + (size_t)(v * 5 + k) * nc, c * 8u);
                cf[2 * k] = pr.x;
                cf[2 * k + 1] = pr.y;
            }
        }
        T val = cf[0] + cf[1] * y[0] + cf[2] * y[1] + cf[3] * y[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) val += cf[4 + k] * yy[k];
        if constexpr (!REC32) {
            q[v] = val;
        } else {
            // FP32 records: the cell mean plus the deviation, rounded once to T
            const double mean = Sto<S32>::ld(stage == 1 ? P.Q : P.Qs, v, nc, c);
            q[v] = (T)(mean + (double)val);
        }
        const T gx = cf[1] + T(2) * cf[4] * y[0] + cf[7] * y[1] + cf[8] * y[2];
        const T gy = cf[2] + T(2) * cf[5] * y[1] + cf[7] * y[0] + cf[9] * y[2];
        const T gz = cf[3] + T(2) * cf[6] * y[2] + cf[8] * y[0] + cf[9] * y[1];
        if constexpr (ADD) {
            g[v][0] += gx; g[v][1] += gy; g[v][2] += gz;
        } else {
            g[v][0] = gx; g[v][1] = gy; g[v][2] = gz;
        }
    }
}

// Values at the three Gauss points y[p] and gradients of the five variables of one
// cell's reconstruction, evaluated while its coefficients stream in, so that each
// coefficient is loaded once per face.  ADD accumulates the gradients.
// REFL: the gradient is reflected before it is added, g - refl (g.n) n (refl = 2 at a
// wall face, 0 elsewhere; the ghost side of a wall face)
template <class T, bool ADD, bool REFL = false, bool S32 = false>
__device__ __forceinline__ void recon_gp3(const ProbDesc &P, int stage, uint32_t c, const T y[3][3], T q[3][5],
                                          T g[3][5][3], const T *nrm = nullptr, T refl = T(0)) {
    const uint32_t nc = (uint32_t)P.nc;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        T cf[10];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if constexpr (sizeof(T) == 8) {
                const d2 pr = ldg<d2>(reinterpret_cast<const d2 *>(P.C) + (size_t)(v * 5 + k) * nc, c * 16u);
                cf[2 * k] = pr.x;
                cf[2 * k + 1] = pr.y;
            } else {
                const f2 pr = ldg<f2>(reinterpret_cast<const f2 *>(P.C32) + (size_t)(v * 5 + k) * nc, c * 8u);
                cf[2 * k] = pr.x;
                cf[2 * k + 1] = pr.y;
            }
        }
        double mean = 0.0;
        if constexpr (sizeof(T) == 4) mean = Sto<S32>::ld(stage == 1 ? P.Q : P.Qs, v, nc, c);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const T *yp = y[p];
            T val = cf[0] + cf[1] * yp[0] + cf[2] * yp[1] + cf[3] * yp[2];
            val += cf[4] * (yp[0] * yp[0]);
            val += cf[5] * (yp[1] * yp[1]);
            val += cf[6] * (yp[2] * yp[2]);
            val += cf[7] * (yp[0] * yp[1]);
            val += cf[8] * (yp[0] * yp[2]);
            val += cf[9] * (yp[1] * yp[2]);
            if constexpr (sizeof(T) == 8)
                q[p][v] = val;
            else  // FP32 form: FP64 cell mean plus FP32 deviation, rounded once
                q[p][v] = (float)(mean + (double)val);
            T gx = cf[1] + T(2) * cf[4] * yp[0] + cf[7] * yp[1] + cf[8] * yp[2];
            T gy = cf[2] + T(2) * cf[5] * yp[1] + cf[7] * yp[0] + cf[9] * yp[2];
            T gz = cf[3] + T(2) * cf[6] * yp[2] + cf[8] * yp[0] + cf[9] * yp[1];
            if constexpr (REFL) {
                const T gn = refl * (gx * nrm[0] + gy * nrm[1] + gz * nrm[2]);
                gx -= gn * nrm[0];
                gy -= gn * nrm[1];
                gz -= gn * nrm[2];
            }
            if constexpr (ADD) {
                g[p][v][0] += gx; g[p][v][1] += gy; g[p][v][2] += gz;
            } else {
                g[p][v][0] = gx; g[p][v][1] = gy; g[p][v][2] = gz;
            }
        }
    }
}

// Face geometry: 16 values per face in pair rows [8][nf] (value v in pair v/2, lane
// v%2): the unit normal (3), the area, the offsets of the three Gauss points from the
// left centroid (3 x 3), and the left centroid minus the right one (periodic image
// applied).  A point's offset from the right centroid is its left offset plus that
// difference; it is zero at a wall face, whose ghost side is evaluated at the wall
// cell's own offsets.
// (FP32 pairs in the FP32 form.)
template <bool S32 = false>
__device__ __forceinline__ void load_fgeo(const ProbDesc &P, uint32_t f, double v[16]) {
    const size_t nf = (size_t)P.nf;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if constexpr (S32) {
            const f2 pr = ldg_stream_f2(reinterpret_cast<const f2 *>(P.fgeo) + k * nf, f * 8u);
            v[2 * k] = pr.x;
            v[2 * k + 1] = pr.y;
        } else {
            const d2 pr = ldg_stream(reinterpret_cast<const d2 *>(P.fgeo) + k * nf, f * 16u);
            v[2 * k] = pr.x;
            v[2 * k + 1] = pr.y;
        }
    }
}
template <bool S32 = false>
__device__ __forceinline__ double fgeo_area(const ProbDesc &P, uint32_t f) {
    // value 3: pair 1, lane 1
    if constexpr (S32) return (double)ldg<float>(reinterpret_cast<const float *>(P.fgeo) + (size_t)2 * P.nf, f * 8u + 4u);
    else return ldg<double>(P.fgeo + (size_t)2 * P.nf, f * 16u + 8u);
}
// One value of a face's geometry record (v as above)
template <bool S32 = false>
__device__ __forceinline__ double fgeo_value(const ProbDesc &P, uint32_t f, uint32_t v) {
    const size_t row = (size_t)(v >> 1) * 2 * (size_t)P.nf;       // pair row v/2, in elements
    if constexpr (S32) return (double)ldg<float>(reinterpret_cast<const float *>(P.fgeo) + row, (f * 2u + (v & 1u)) * 4u);
    else return ldg<double>(P.fgeo + row, (f * 2u + (v & 1u)) * 8u);
}
// The normal and the offsets of Gauss point g from both centroids, loading only
// those nine values (for kernels that evaluate one point of a face per lane)
template <class T, bool S32 = false>
__device__ __forceinline__ void fgeo_gauss(const ProbDesc &P, uint32_t f, uint32_t g, T n[3], T yl[3], T yr[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        n[a] = (T)fgeo_value<S32>(P, f, (uint32_t)a);
        const double y = fgeo_value<S32>(P, f, 4u + 3u * g + (uint32_t)a);
        yl[a] = (T)y;
        yr[a] = (T)(y + fgeo_value<S32>(P, f, 13u + (uint32_t)a));
    }
}
// Gauss point p: offsets from the left and the right centroid (p may differ across
// lanes: the point is selected, never indexed, so v stays in registers)
template <class T>
__device__ __forceinline__ void fgeo_point(const double v[16], int p, T yl[3], T yr[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double y = p == 0 ? v[4 + a] : (p == 1 ? v[7 + a] : v[10 + a]);
        yl[a] = (T)y;
        yr[a] = (T)(y + v[13 + a]);
    }
}

// The tau = 0 flux of face f with the positivity fallback, one Gauss point at a
// time from reloaded inputs (only faces that need it come here).
template <class T, bool S32 = false>
__device__ __forceinline__ void flux_face_fallback(const ProbDesc &P, int stage, uint32_t f, uint32_t l,
                                                             uint32_t r, bool wall, double out[10]) {
    double fv[16];
    load_fgeo<S32>(P, f, fv);
    const T n[3] = {(T)fv[0], (T)fv[1], (T)fv[2]};
    const double w = fv[3] * (1.0 / 3.0);
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        T yl[3], yr[3];
        fgeo_point(fv, p, yl, yr);
        T qL[5], qR[5], gs[5][3];
        recon_point<T, false, (sizeof(T) == 4), S32>(P, stage, l, yl, qL, gs);
        recon_point<T, true, (sizeof(T) == 4), S32>(P, stage, r, yr, qR, gs);
        if (wall) reflect_grad(gs, n, T(1));
        const bool okL = physical_point(qL), okR = physical_point(qR);
        if (!(okL && okR)) {
            if (!okL) cell_mean<T, S32>(P, stage, l, qL);
            if (!okR) cell_mean<T, S32>(P, stage, r, qR);
#pragma unroll
            for (int v = 0; v < 5; ++v) gs[v][0] = gs[v][1] = gs[v][2] = T(0);
        }
        T F[5], dF[5];
        gks_flux_tau0<T>(qL, qR, gs, n, P, F, dF);
        if (!finite_flux(F, dF)) {          // (FP32 form) a non-finite point flux: first order
            cell_mean<T, S32>(P, stage, l, qL);
            cell_mean<T, S32>(P, stage, r, qR);
#pragma unroll
            for (int v = 0; v < 5; ++v) gs[v][0] = gs[v][1] = gs[v][2] = T(0);
            gks_flux_tau0<T>(qL, qR, gs, n, P, F, dF);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            out[k] = p == 0 ? w * (double)F[k] : out[k] + w * (double)F[k];
            out[5 + k] = p == 0 ? w * (double)dF[k] : out[5 + k] + w * (double)dF[k];
        }
    }
}

// tau = 0: one lane per face, the three Gauss points in turn.  Each lane reads
// both cells' reconstruction records once and evaluates them at all three points
// (the per-face loads are scattered on the right-hand side, so the address units,
// not the arithmetic, bound this kernel: loading every record byte once per face
// rather than once per Gauss point is what counts), then evaluates the three
// Gauss-point fluxes and writes S * sum_G w_G (F, dF).  No LDS and no barriers.
// DF_ONLY (second stage, per-face buffer): only dF is stored, since the S2O4 update
// of that stage does not use L(Q*).  The wall variants are held to two waves per
// SIMD: left alone the FP64 one takes a few accumulation registers beyond 256 and
// runs one wave (a few bytes of scratch per lane cost less than that).
template <bool MIXED, bool COLOURED, bool WALLS, bool DF_ONLY = false, bool S32 = false>
__global__ __launch_bounds__(FACE_TILE) __attribute__((amdgpu_waves_per_eu(COLOURED ? 1 : (MIXED ? 3 : 2)))) void
k_flux_t0(const ProbDesc *__restrict__ probs,
                                                       const Tile *__restrict__ tiles, int stage) {
    static_assert(!(DF_ONLY && COLOURED), "the coloured mode accumulates both");
    static_assert(MIXED || !S32, "FP32 storage comes with the FP32 flux");
    using ST = Sto<S32>;
    using T = typename std::conditional<MIXED, float, double>::type;
    // tiles in reverse order: the reconstruction records written last by the WENO
    // pass are the likeliest still to sit in the last-level cache
    const Tile tl = tiles[gridDim.x - 1 - blockIdx.x];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t f = tl.begin + threadIdx.x;
    if (f >= (uint32_t)tl.end) return;
    const uint32_t nf = (uint32_t)P.nf;
    const uint32_t l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
    const int32_t rr = ldg<int32_t>(P.fcell + nf, f * 4u);
    const bool wall = WALLS && rr < 0;           // the ghost side is l's record mirrored
    const uint32_t r = rr < 0 ? l : (uint32_t)rr;
    double fv[16];
    load_fgeo<S32>(P, f, fv);
    const T n[3] = {(T)fv[0], (T)fv[1], (T)fv[2]};
    const double S = fv[3];
    T yl[3][3], yr[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p) fgeo_point(fv, p, yl[p], yr[p]);
    T qL[3][5], qR[3][5], gs[3][5][3];
    recon_gp3<T, false, false, S32>(P, stage, l, yl, qL, gs);
    // at a wall face the ghost side adds l's gradient reflected in the wall (branch-free:
    // a branch on the wall flag here costs the kernel half its occupancy)
    recon_gp3<T, true, WALLS, S32>(P, stage, r, yr, qR, gs, n, wall ? T(2) : T(0));
    const double w = S * (1.0 / 3.0);          // three Gauss points of equal weight
    double out[10];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        T F[5], dF[5];
        gks_flux_tau0<T>(qL[p], qR[p], gs[p], n, P, F, dF);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            out[k] = p == 0 ? w * (double)F[k] : out[k] + w * (double)F[k];
            out[5 + k] = p == 0 ? w * (double)dF[k] : out[5 + k] + w * (double)dF[k];
        }
    }
    if constexpr (COLOURED) {      // this mode accumulates at once: take the fallback inline
        if (!(out[0] == out[0])) flux_face_fallback<T, S32>(P, stage, f, l, r, wall, out);
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        if constexpr (COLOURED) {
            const uint32_t ncu = (uint32_t)P.nc;      // no other face of this colour touches l or r
            ST::st(P.acc, k, ncu, l, ST::ld(P.acc, k, ncu, l) - out[k]);
            if (!wall) ST::st(P.acc, k, ncu, r, ST::ld(P.acc, k, ncu, r) + out[k]);
        } else if (!DF_ONLY || k >= 5) {
            // streaming stores (the update gathers them later).  In the FP64-storage
            // forms the generic-address form of the store is used: with it the compiler
            // keeps up to 21 record loads in flight rather than 9 (356 against 371 us a
            // launch at 6 64^3, FP64)
            if constexpr (!S32) __builtin_nontemporal_store(out[k], P.FF + (size_t)k * nf + f);
            else ST::st_nt(P.FF, k, nf, f, out[k]);
        }
    }
    if constexpr (!COLOURED) {
        // the fix-up pass has work: a non-finite face (flag cleared by the stage update)
        const double chk = DF_ONLY ? out[5] : out[0];
        const uint64_t bad = __ballot(!(chk - chk == 0.0));
        if (bad != 0 && threadIdx.x == 0) P.flag[1] = 1;
    }
}

// Faces whose tau = 0 flux came out non-finite had a non-physical reconstructed
// side at some Gauss point (rho <= 0 or p <= 0 make lam <= 0, and the half-space
// moments then return NaN); they are recomputed here with the positivity
// fallback.  The flux kernel raises flag[1] of the problem when it wrote such a
// face (the stage update clears it); with the flag clear, as in smooth flow, the
// pass reads one word per tile.
// Each workgroup (one wave) walks tiles with a grid stride, so the scan is a
// few waves per SIMD reading one double per face; the recomputation is rare and
// may use scratch memory.
template <bool MIXED, bool S32 = false>
__global__ __launch_bounds__(FACE_TILE) __attribute__((amdgpu_waves_per_eu(4))) void k_flux_fix(
    const ProbDesc *__restrict__ probs, int nprobs, const Tile *__restrict__ tiles, int ntiles, int stage) {
    using T = typename std::conditional<MIXED, float, double>::type;
    using ST = Sto<S32>;
    // one look at every problem's flag: nothing to do in any of them is the common case
    bool any = false;
    for (int k = threadIdx.x; k < nprobs; k += FACE_TILE) any = any || ldg<int32_t>(probs[k].flag, 4u) != 0;
    if (__ballot(any) == 0) return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const ProbDesc &P = probs[tl.prob];
        if (ldg<int32_t>(P.flag, 4u) == 0) continue;   // no non-finite face in this problem
        const uint32_t f = tl.begin + threadIdx.x;
        if (f >= (uint32_t)tl.end) continue;
        const uint32_t nf = (uint32_t)P.nf;
        // the first row of F, or in the second stage (F not stored) of dF
        const double f0 = ST::ld(P.FF, stage == 1 ? 0 : 5, nf, f);
        if (f0 - f0 == 0.0) continue;            // finite
        const uint32_t l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
        const int32_t rr = ldg<int32_t>(P.fcell + nf, f * 4u);
        double out[10];
        flux_face_fallback<T, S32>(P, stage, f, l, rr < 0 ? l : (uint32_t)rr, rr < 0, out);
#pragma unroll
        for (int k = 0; k < 10; ++k) ST::st(P.FF, k, nf, f, out[k]);
    }
}

// The tau > 0 flux at Gauss point g of face f (between cells l and r; wall: r = l and
// the ghost side mirrored), in FP64.  MIXED: from the FP32-mixed records (the points
// the FP32 pass leaves, and the coloured mode of the FP32-mixed form).
template <bool MIXED, bool WALLS, bool S32 = false>
__device__ __forceinline__ void point_flux_full(const ProbDesc &P, int stage, uint32_t f, uint32_t g, uint32_t l,
                                                uint32_t r, bool wall, double Fo[5], double dFo[5]) {
    double nd[3], yld[3], yrd[3];
    fgeo_gauss<double, S32>(P, f, g, nd, yld, yrd);
    double qL[5], gL[5][3], qR[5], gR[5][3];
    recon_point<double, false, MIXED, S32>(P, stage, l, yld, qL, gL);
    recon_point<double, false, MIXED, S32>(P, stage, r, yrd, qR, gR);
    if constexpr (WALLS) reflect_grad(gR, nd, wall ? 2.0 : 0.0);
    const bool okL = physical_point(qL), okR = physical_point(qR);
    if (!(okL && okR)) {
        if (!okL) cell_mean<double, S32>(P, stage, l, qL);
        if (!okR) cell_mean<double, S32>(P, stage, r, qR);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            gL[v][0] = gL[v][1] = gL[v][2] = 0.0;
            gR[v][0] = gR[v][1] = gR[v][2] = 0.0;
        }
    }
    gks_flux_full<double>(qL, gL, qR, gR, nd, ldg<double>(P.dt, 0u), P, Fo, dFo);
}

// Whether a point state is well conditioned for the FP32 tau > 0 flux: its energy
// is not mostly kinetic, kappa = E / (rho e) <= 10 (ke <= 0.9 E; a local Mach
// number up to 5.7 in the frame of the stored state).  The pressure
// (gamma-1)(E - |m|^2 / 2 rho) of a state loses about eps kappa of relative
// precision; the closed-form micro-slope solve (energy component c4 (R4 - 2 U.R),
// c4 ~ lam^2, terms of size |U|^2 b cancelling) and the initial parts' half-space
// slope moments (terms growing like U^k that cancel) amplify it further.  In FP32
// the slope solve alone stays within 1e-5 for kappa <= 10 and exceeds 1e-4 from
// kappa = 1e3.  Every FP32 point flux that departed from FP64 by more than 1e-3 on
// the 12.6 M-cell doubled shock tube (753 points, all in the first steps after the
// diaphragm) had a side with kappa >= 37: a reconstructed state almost without
// internal energy, whose slope moments came out wrong by up to four orders of
// magnitude; none with kappa < 37 departed.
template <class T>
__device__ __forceinline__ bool warm_point(const T q[5]) {
    return T(18) * q[0] * q[4] >= T(10) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

// The FP32-mixed (and FP32) form evaluates the tau > 0 flux in FP32 where both
// reconstructed sides are warm (warm_point).  A point with a cold side, where the
// positivity fallback acts, or whose flux is not finite, is left to the FP64
// evaluation of the fix-up pass (returns false).
template <bool WALLS, bool S32 = false>
__device__ __forceinline__ bool point_flux_full32(const ProbDesc &P, int stage, uint32_t f, uint32_t g, uint32_t l,
                                                  uint32_t r, bool wall, double Fo[5], double dFo[5]) {
    float n[3], yl[3], yr[3];
    fgeo_gauss<float, S32>(P, f, g, n, yl, yr);
    float qL[5], gL[5][3], qR[5], gR[5][3];
    recon_point<float, false, true, S32>(P, stage, l, yl, qL, gL);
    recon_point<float, false, true, S32>(P, stage, r, yr, qR, gR);
    if constexpr (WALLS) reflect_grad(gR, n, wall ? 2.0f : 0.0f);
    if (!(physical_point(qL) && physical_point(qR))) return false;
    if (!(warm_point(qL) && warm_point(qR))) return false;
    float F[5], dF[5];
    gks_flux_full<float>(qL, gL, qR, gR, n, (float)ldg<double>(P.dt, 0u), P, F, dF);
    if (!finite_flux(F, dF)) return false;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        Fo[k] = (double)F[k];
        dFo[k] = (double)dF[k];
    }
    return true;
}

template <bool MIXED, bool TAU0, bool COLOURED, bool WALLS, bool S32 = false>
__global__ __launch_bounds__(3 * FACE_TILE) void k_flux(const ProbDesc *__restrict__ probs,
                                                         const Tile *__restrict__ tiles, int stage) {
    using T = typename std::conditional<MIXED, float, double>::type;
    using ST = Sto<S32>;
    __shared__ double red[3][10][FACE_TILE];
    const Tile tl = tiles[blockIdx.x];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t lane = threadIdx.x % FACE_TILE;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / FACE_TILE);   // Gauss point of this wave
    const uint32_t f = tl.begin + lane;
    const bool ok = f < (uint32_t)tl.end;
    const uint32_t nf = (uint32_t)P.nf;
    double out[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k] = 0.0;
    uint32_t l = 0, r = 0;
    bool wall = false;
    if (ok) {
        l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
        const int32_t rr = ldg<int32_t>(P.fcell + nf, f * 4u);
        wall = WALLS && rr < 0;                  // the ghost side is l's record mirrored
        r = rr < 0 ? l : (uint32_t)rr;
        T n[3], yl[3], yr[3];
        fgeo_gauss<T, S32>(P, f, (uint32_t)g, n, yl, yr);
        const double S = fgeo_area<S32>(P, f);
        double Fo[5], dFo[5];
        if constexpr (TAU0) {
            T qL[5], qR[5], gs[5][3], F[5], dF[5];
            recon_point<T, false, (sizeof(T) == 4), S32>(P, stage, l, yl, qL, gs);
            recon_point<T, true, (sizeof(T) == 4), S32>(P, stage, r, yr, qR, gs);
            if constexpr (WALLS) reflect_grad(gs, n, wall ? T(1) : T(0));
            gks_flux_tau0<T>(qL, qR, gs, n, P, F, dF);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                Fo[k] = (double)F[k];
                dFo[k] = (double)dF[k];
            }
        } else {
            point_flux_full<MIXED, WALLS, S32>(P, stage, f, (uint32_t)g, l, r, wall, Fo, dFo);
        }
        const double w = S * (1.0 / 3.0);      // three Gauss points of equal weight
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            out[k] = w * Fo[k];
            out[5 + k] = w * dFo[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) red[g][k][lane] = out[k];
    __syncthreads();
    if (g == 0 && ok) {
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const double s = red[0][k][lane] + red[1][k][lane] + red[2][k][lane];
            if constexpr (COLOURED) {
                const uint32_t ncu = (uint32_t)P.nc;     // no other face of this colour touches l or r
                ST::st(P.acc, k, ncu, l, ST::ld(P.acc, k, ncu, l) - s);
                if (!wall) ST::st(P.acc, k, ncu, r, ST::ld(P.acc, k, ncu, r) + s);
            } else {
                ST::st(P.FF, k, nf, f, s);
            }
        }
    }
}

// tau > 0 with the per-face buffer: single-wave workgroups, lane 3j + g evaluating
// Gauss point g of face j of the workgroup's 21 faces (tiles of 63 faces, three
// workgroups each).  The three points of a face are summed across neighbouring lanes
// in the order (g0 + g1) + g2, as the three-wave kernel sums them.  At two waves per
// SIMD a three-wave workgroup leaves a quarter of a CU's wave slots idle; single-wave
// workgroups fill them all.
template <bool MIXED, bool WALLS, bool S32 = false>
__global__ __launch_bounds__(64) void k_flux_gp(const ProbDesc *__restrict__ probs, const Tile *__restrict__ tiles,
                                                int stage) {
    using ST = Sto<S32>;
    constexpr uint32_t SPLIT = 3;                        // workgroups per tile
    // XCD x takes a contiguous run of (tile, part) units (the tile table is laid out
    // for one workgroup per tile: invert that layout, as the WENO kernel does)
    const uint32_t nb = gridDim.x, xcd = blockIdx.x & 7u;
    const uint32_t bx = xcd * (nb >> 3) + min(xcd, nb & 7u) + (blockIdx.x >> 3);
    const uint32_t jt = bx / SPLIT, nt = nb / SPLIT;
    uint32_t kt = jt;
    if (nt >= 16u) {
        const uint32_t q8 = nt >> 3, r8 = nt & 7u, big = r8 * (q8 + 1u);
        const uint32_t xx = jt < big ? jt / (q8 + 1u) : r8 + (jt - big) / q8;
        const uint32_t qq = jt < big ? jt % (q8 + 1u) : (jt - big) % q8;
        kt = 8u * qq + xx;
    }
    const Tile tl = tiles[kt];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t j = threadIdx.x / 3u, g = threadIdx.x % 3u;
    const uint32_t f = tl.begin + (bx % SPLIT) * (uint32_t)GP_FACES + j;
    const bool ok = threadIdx.x < 3u * GP_FACES && f < (uint32_t)tl.end;
    const uint32_t nf = (uint32_t)P.nf;
    double out[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k] = 0.0;
    if (ok) {
        const uint32_t l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
        const int32_t rr = ldg<int32_t>(P.fcell + nf, f * 4u);
        const bool wall = WALLS && rr < 0;               // the ghost side is l's record mirrored
        const uint32_t r = rr < 0 ? l : (uint32_t)rr;
        double Fo[5], dFo[5];
        bool done = true;
        if constexpr (MIXED)
            done = point_flux_full32<WALLS, S32>(P, stage, f, g, l, r, wall, Fo, dFo);
        else
            point_flux_full<false, WALLS>(P, stage, f, g, l, r, wall, Fo, dFo);
        const double w = fgeo_area<S32>(P, f) * (1.0 / 3.0);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            out[k] = done ? w * Fo[k] : __builtin_nan("");   // NaN: the face goes to the fix-up pass
            out[5 + k] = done ? w * dFo[k] : __builtin_nan("");
        }
    }
    double s0 = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const double o1 = __shfl_down(out[k], 1u), o2 = __shfl_down(out[k], 2u);
        const double sum = (out[k] + o1) + o2;
        if (k == 0) s0 = sum;
        if (ok && g == 0u) ST::st_nt(P.FF, k, nf, f, sum);
    }
    if constexpr (MIXED) {
        // the fix-up pass has work: a face left to FP64 (flag cleared by the stage update)
        const uint64_t bad = __ballot(ok && g == 0u && !(s0 - s0 == 0.0));
        if (bad != 0 && threadIdx.x == 0) P.flag[1] = 1;
    }
}

// Faces the FP32 tau > 0 pass left (their flux is NaN): the three Gauss points again,
// in FP64 from the FP32 records, summed in the same order.  Grid-stride over the face
// tiles, after one look at every problem's flag (nothing to do is the common case).
template <bool WALLS, bool S32 = false>
__global__ __launch_bounds__(64) void k_flux_fix_full(const ProbDesc *__restrict__ probs, int nprobs,
                                                      const Tile *__restrict__ tiles, int ntiles, int stage) {
    using ST = Sto<S32>;
    bool any = false;
    for (int k = threadIdx.x; k < nprobs; k += 64) any = any || ldg<int32_t>(probs[k].flag, 4u) != 0;
    if (__ballot(any) == 0) return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const ProbDesc &P = probs[tl.prob];
        if (ldg<int32_t>(P.flag, 4u) == 0) continue;
        const uint32_t f = tl.begin + threadIdx.x;
        if (f >= (uint32_t)tl.end) continue;
        const uint32_t nf = (uint32_t)P.nf;
        const double f0 = ST::ld(P.FF, 0, nf, f);
        if (f0 - f0 == 0.0) continue;                     // finite: done in FP32
        const uint32_t l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
        const int32_t rr = ldg<int32_t>(P.fcell + nf, f * 4u);
        const bool wall = WALLS && rr < 0;
        const uint32_t r = rr < 0 ? l : (uint32_t)rr;
        const double w = fgeo_area<S32>(P, f) * (1.0 / 3.0);
        double out[10];
#pragma unroll 1
        for (uint32_t g = 0; g < 3u; ++g) {
            double Fo[5], dFo[5];
            point_flux_full<true, WALLS, S32>(P, stage, f, g, l, r, wall, Fo, dFo);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                out[k] = g == 0u ? w * Fo[k] : out[k] + w * Fo[k];
                out[5 + k] = g == 0u ? w * dFo[k] : out[5 + k] + w * dFo[k];
            }
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) ST::st(P.FF, k, nf, f, out[k]);
    }
}

// ----------------------------------------------------------------------------
// S2O4 update and the CFL time step
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
    return x;
}

// h / (|U| + c) of a cell, and whether its state is physical (rho > 0, p > 0, finite)
template <bool S32 = false>
__device__ __forceinline__ double cfl_bound(const ProbDesc &P, uint32_t i, const double q[5], bool &ok) {
    const double rho = q[0], ir = 1.0 / rho;
    const double u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
    const double p = (P.gamma - 1.0) * (q[4] - 0.5 * rho * (u * u + v * v + w * w));
    ok = rho > 0.0 && p > 0.0 && isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) &&
         isfinite(q[4]);
    const double c = sqrt(P.gamma * p * ir);
    return Sto<S32>::ld(P.cgeo, 8, (uint32_t)P.nc, i) / (sqrt(u * u + v * v + w * w) + c);
}

template <int STAGE, bool COLOURED, bool S32 = false, int NFC = 4>
__global__ __launch_bounds__(UPD_TILE) void k_update(const ProbDesc *__restrict__ probs,
                                                      const Tile *__restrict__ tiles) {
    using ST = Sto<S32>;
    const Tile tl = tiles[blockIdx.x];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t nc = (uint32_t)P.nc;
    const uint32_t i = tl.begin + threadIdx.x;
    double bound = DBL_MAX;
    if (i < (uint32_t)tl.end) {
        double s[10];
        if constexpr (COLOURED) {
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                s[k] = ST::ld(P.acc, k, nc, i);
                ST::st(P.acc, k, nc, i, 0.0);
            }
        } else {
            const uint32_t nf = (uint32_t)P.nf;
#pragma unroll
            for (int k = 0; k < 10; ++k) s[k] = 0.0;
#pragma unroll
            for (int p = 0; p < NFC; ++p) {     // the cell's faces, fixed order
                const uint32_t code = (uint32_t)ldg<int32_t>(P.cface + (size_t)p * nc, i * 4u);
                const uint32_t f = code >> 1;
                const double sg = (code & 1u) ? 1.0 : -1.0;   // the normal points out of the left cell
#pragma unroll
                for (int k = 0; k < 10; ++k) s[k] = fma(sg, ST::ld(P.FF, k, nf, f), s[k]);
            }
        }
        const double iv = ST::ld(P.cgeo, 7, nc, i);
        const double dt = ldg<double>(P.dt, 0u);
        double qn[5];
        bool ok;
        if constexpr (STAGE == 1) {
            // Q* = Q + dt/2 L + dt^2/8 dL,   R = Q + dt L + dt^2/6 dL
            const double h2 = 0.5 * dt, h8 = 0.125 * dt * dt, h6 = dt * dt * (1.0 / 6.0);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double q = ST::ld(P.Q, v, nc, i);
                const double L = s[v] * iv, dL = s[5 + v] * iv;
                qn[v] = q + h2 * L + h8 * dL;
                ST::st(P.Qs, v, nc, i, qn[v]);
                ST::st(P.R, v, nc, i, q + dt * L + h6 * dL);
            }
            cfl_bound<S32>(P, i, qn, ok);
        } else {
            // Q^{n+1} = R + dt^2/3 dL(Q*)
            const double h3 = dt * dt * (1.0 / 3.0);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qn[v] = ST::ld(P.R, v, nc, i) + h3 * (s[5 + v] * iv);
                ST::st(P.Q, v, nc, i, qn[v]);
                qn[v] = (double)(typename ST::E)qn[v];        // the CFL bound of the stored state
            }
            bound = cfl_bound<S32>(P, i, qn, ok);
        }
        if (!ok) P.flag[0] = 1;
    }
    if (tl.local == 0 && threadIdx.x == 0) P.flag[1] = 0;   // the flux fix-up flag of this stage is spent
    if constexpr (STAGE == 2) {
        bound = wave_min(bound);
        if (threadIdx.x == 0) P.dtpart[tl.local] = bound;
    }
}

template <bool S32 = false>
__global__ __launch_bounds__(UPD_TILE) void k_dt_local(const ProbDesc *__restrict__ probs,
                                                        const Tile *__restrict__ tiles) {
    const Tile tl = tiles[blockIdx.x];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t i = tl.begin + threadIdx.x;
    double bound = DBL_MAX;
    if (i < (uint32_t)tl.end) {
        double q[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = Sto<S32>::ld(P.Q, v, (uint32_t)P.nc, i);
        bool ok;
        bound = cfl_bound<S32>(P, i, q, ok);
        if (!ok) P.flag[0] = 1;
    }
    bound = wave_min(bound);
    if (threadIdx.x == 0) P.dtpart[tl.local] = bound;
}

__global__ __launch_bounds__(1024) void k_dt_final(const ProbDesc *__restrict__ probs, double dt_fixed) {
    __shared__ double part[16];
    const ProbDesc &P = probs[blockIdx.x];
    double m0 = DBL_MAX, m1 = DBL_MAX, m2 = DBL_MAX, m3 = DBL_MAX;   // four independent chains
    const uint32_t n = (uint32_t)P.n_cell_tiles;
    uint32_t k = threadIdx.x;
    for (; k + 3 * 1024 < n; k += 4 * 1024) {
        m0 = fmin(m0, ldg<double>(P.dtpart, k * 8u));
        m1 = fmin(m1, ldg<double>(P.dtpart, (k + 1024) * 8u));
        m2 = fmin(m2, ldg<double>(P.dtpart, (k + 2048) * 8u));
        m3 = fmin(m3, ldg<double>(P.dtpart, (k + 3072) * 8u));
    }
    for (; k < n; k += 1024) m0 = fmin(m0, ldg<double>(P.dtpart, k * 8u));
    double m = wave_min(fmin(fmin(m0, m1), fmin(m2, m3)));
    if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < 16; ++w) m = fmin(m, part[w]);
        m = fmin(m, part[0]);
        const double dt = dt_fixed > 0.0 ? dt_fixed : P.cfl * m;
        P.dt[0] = dt;
        P.time[0] += dt;
    }
}

__global__ void k_fill(double *p, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ----------------------------------------------------------------------------
// hexahedral meshes
// ----------------------------------------------------------------------------

// Far-field state by Riemann invariants (characteristic boundary, Sec. 5.2) for the
// outward normal n: the outgoing invariant U.n + 2c/(g-1) comes from q, the incoming
// U.n - 2c/(g-1) from the free stream; entropy p/rho^g and tangential velocity from
// q at an outflow, from the free stream at an inflow.  A supersonic outflow keeps
// q, a supersonic inflow takes the free stream.
template <class T>
__device__ __forceinline__ void farfield_state(const ProbDesc &P, const T q[5], const T n[3], T out[5]) {
    const T g = (T)P.gamma, gm1 = g - T(1);
    const T ir = T(1) / q[0];
    const T u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const T pi = gm1 * (q[4] - T(0.5) * q[0] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
    const T rf = (T)P.farfield[0], pf = (T)P.farfield[4];
    const T uf[3] = {(T)P.farfield[1], (T)P.farfield[2], (T)P.farfield[3]};
    const T ci = sqrt(g * pi * ir), cf = sqrt(g * pf / rf);
    const T vi = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    const T vf = uf[0] * n[0] + uf[1] * n[1] + uf[2] * n[2];
    T rb, pb, ub[3];
    if (vi >= ci) {
#pragma unroll
        for (int k = 0; k < 5; ++k) out[k] = q[k];
        return;
    }
    if (vi <= -ci) {
        rb = rf;
        pb = pf;
#pragma unroll
        for (int a = 0; a < 3; ++a) ub[a] = uf[a];
    } else {
        const T Rp = vi + T(2) * ci / gm1, Rm = vf - T(2) * cf / gm1;
        const T vb = T(0.5) * (Rp + Rm), cb = T(0.25) * gm1 * (Rp - Rm);
        const bool outflow = vb > T(0);
        const T ent = outflow ? pi / hg_pow(q[0], g) : pf / hg_pow(rf, g);
        const T vt = outflow ? vi : vf;
        rb = hg_pow(cb * cb / (g * ent), T(1) / gm1);
        pb = rb * cb * cb / g;
#pragma unroll
        for (int a = 0; a < 3; ++a) ub[a] = (outflow ? u[a] : uf[a]) - vt * n[a] + vb * n[a];
    }
    out[0] = rb;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[1 + a] = rb * ub[a];
    out[4] = pb / gm1 + T(0.5) * rb * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
}

// Ghost states of the listed boundary faces for the stage's state: a wall ghost holds
// (rho, -rho U, rho E) of its cell, a far-field ghost the Riemann-invariant state of
// its cell for the face's mean normal.  The WENO pass reads them as stencil members.
__global__ __launch_bounds__(256) void k_ghost_hex(const ProbDesc *__restrict__ d, int stage) {
    const ProbDesc &P = *d;
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    const uint32_t ng = (uint32_t)P.ng, nc = (uint32_t)P.nc;
    if (g >= ng) return;
    const uint32_t c = (uint32_t)P.gcell[g];
    const double *Qa = stage == 1 ? P.Q : P.Qs;
    double q[5], o[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Qa[(size_t)v * nc + c];
    if (P.gkind[g] == HGKS_BC_WALL) {
        o[0] = q[0]; o[1] = -q[1]; o[2] = -q[2]; o[3] = -q[3]; o[4] = q[4];
    } else {
        const double n[3] = {P.gnrm[g], P.gnrm[ng + g], P.gnrm[2 * ng + g]};
        farfield_state<double>(P, q, n, o);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) P.G[(size_t)v * ng + g] = o[v];
}

// WENO on hexahedra (Sec. 2.3, M = 8).  A workgroup of 128 threads takes 16 cells
// (four workgroups per 64-cell tile, XCD-contiguous as for tetrahedra):
//  - the threads load the cells' HEX_NS stencil ids into LDS and stream the 16
//    cells' big-stencil pseudo-inverses (9 rows x HEX_NS slots as 108 pair rows,
//    non-temporal, each value read from HBM once) through registers into LDS in
//    NCH chunks of slots, the next chunk fetched as the previous one is consumed
//    (two chunks: 15.4 KB of LDS, six to eight workgroups a CU);
//  - lane (v, c), v < 5, gathers all HEX_NS member differences of variable v of
//    cell c at once (ghost members from the stage's ghost states), then forms the
//    big-stencil fit a = P (Q_k - Q_i) chunk by chunk from LDS;
//  - thread (m, c) loads the 3x3 inverse of sub-stencil m of cell c, the exactly
//    determined fit on {i, i_a, i_b, i_c} with i_a.. among the face neighbours (slots
//    0-5 in face order), and writes it over the consumed rows; the lanes form the
//    eight linear fits from there;
//  - the smoothness indicators, WENO-Z weights (gamma_0 = 1 - 8 gamma) and the
//    combined polynomial follow the tetrahedral kernel, in the same record layout.
constexpr int HEX_WC = 16;

template <bool MIXED, int NCH>
__global__ __launch_bounds__(weno_threads<HEX_WC>()) __attribute__((amdgpu_waves_per_eu(MIXED ? 4 : 1))) void k_weno_hex(const ProbDesc *__restrict__ probs,
                                                                      const Tile *__restrict__ tiles, int stage) {
    using T = typename std::conditional<MIXED, float, double>::type;
    constexpr int WC = HEX_WC, NT = weno_threads<WC>(), NS = HEX_NS;
    constexpr int SPLIT = HEX_WENO_CELLS / WC;
    constexpr int CH = NS / 2 / NCH, CROWS = 9 * CH;    // pair columns and pair rows of a chunk
    static_assert(8 * WC <= NT, "one sub-stencil inverse per thread");
    static_assert(CROWS * 16 >= 72 * 8, "the inverses fit over a chunk");
    __shared__ __attribute__((aligned(16))) char smem[(CROWS * 16 + NS * 4) * WC];
    d2(*sp)[WC] = reinterpret_cast<d2(*)[WC]>(smem);
    double(*sb)[WC] = reinterpret_cast<double(*)[WC]>(smem);          // the inverses, after the big fit
    int32_t(*sid)[WC] = reinterpret_cast<int32_t(*)[WC]>(smem + CROWS * 16 * WC);
    uint32_t kt, part;
    split_tile<SPLIT>(kt, part);
    const Tile tl = tiles[kt];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t nc = (uint32_t)P.nc, ng = (uint32_t)P.ng;
    const uint32_t c0 = (uint32_t)tl.begin + part * WC, last = (uint32_t)tl.end - 1;
    // 1. stencil ids, then the pseudo-inverse stream into registers (the ids' LDS copy
    // then waits for the ids alone: the wait counter is in order)
    constexpr int IDS = (NS * WC + NT - 1) / NT;
    int32_t idv[IDS];
#pragma unroll
    for (int k = 0; k < IDS; ++k) {     // (clamped rather than guarded: no branch per load)
        const uint32_t e = min(threadIdx.x + k * NT, (uint32_t)(NS * WC - 1));
        idv[k] = ldg<int32_t>(P.sten + (size_t)(e / WC) * nc, min(c0 + e % WC, last) * 4u);
    }
    constexpr int PER = (CROWS * WC + NT - 1) / NT;
    const d2 *p0 = reinterpret_cast<const d2 *>(P.hpinv);
    d2 reg[NCH][PER];                    // (one chunk live at a time)
    auto stream = [&](int h) {           // chunk h: pair columns h CH .. h CH + CH - 1 of the nine rows
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t e = min(threadIdx.x + k * NT, (uint32_t)(CROWS * WC - 1)), lr = e / WC;
            const uint32_t grow = (lr / CH) * (NS / 2) + h * CH + lr % CH;
            reg[h][k] = ldg_stream(p0 + (size_t)grow * nc, min(c0 + e % WC, last) * 16u);
        }
    };
    auto put = [&](int h) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t e = threadIdx.x + k * NT;
            if ((k + 1) * NT <= CROWS * WC || e < (uint32_t)(CROWS * WC)) sp[e / WC][e % WC] = reg[h][k];
        }
    };
    stream(0);                           // later chunks are fetched as the previous one is consumed
#pragma unroll
    for (int k = 0; k < IDS; ++k) {
        const uint32_t e = threadIdx.x + k * NT;
        if ((k + 1) * NT <= NS * WC || e < (uint32_t)(NS * WC)) sid[e / WC][e % WC] = idv[k];
    }
    const uint32_t v = threadIdx.x / WC, cl = threadIdx.x % WC;
    const bool active = v < 5u;
    const uint32_t i = min(c0 + cl, last);
    const bool ok = active && c0 + cl <= last;
    const uint32_t vrow = active ? v : 0u;
    const double *Qv = (stage == 1 ? P.Q : P.Qs) + (size_t)vrow * nc;
    const double *Gv = P.G + (size_t)vrow * ng;
    const double qi = ldg<double>(Qv, i * 8u);
    double geo[7];
    if (active) {
#pragma unroll
        for (int q = 0; q < 7; ++q) geo[q] = ldg<double>(P.cgeo + (size_t)q * nc, i * 8u);
    }
    __syncthreads();                     // ids in LDS
    // 2. the member differences, all gathers in flight together (no branch per member:
    // the address selects the state or the ghost array; spare lanes gather variable 0)
    uint32_t id[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) id[s] = (uint32_t)sid[s][cl];
    double d[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) d[s] = ldg_at(id[s] < nc ? Qv + id[s] : Gv + (id[s] - nc)) - qi;
    // 3. the big-stencil fit, chunk by chunk (slot order within each row's sum);
    // thread (m, c) fetches its sub-stencil inverse meanwhile
    const uint32_t fm = threadIdx.x / WC;
    double binv[9], a64[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) a64[r] = 0.0;
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        if (h > 0) __syncthreads();      // the previous chunk is consumed
        if (h > 0) stream(h);
        put(h);
        __syncthreads();
        if (h == NCH - 1) {
#pragma unroll
            for (int q = 0; q < 9; ++q) binv[q] = ldg<double>(P.hbinv + (size_t)(fm * 9 + q) * nc, i * 8u);
        }
#pragma unroll 3                         // fully unrolled, the LDS reads of all rows go up front (512 registers)
        for (int r = 0; r < 9; ++r) {
            double acc = a64[r];
#pragma unroll
            for (int s2 = 0; s2 < CH; ++s2) {
                const d2 pp = sp[r * CH + s2][cl];
                acc = fma(pp.x, d[2 * (h * CH + s2)], acc);
                acc = fma(pp.y, d[2 * (h * CH + s2) + 1], acc);
            }
            a64[r] = acc;
        }
    }
    __syncthreads();                     // every lane has read the big rows
#pragma unroll
    for (int q = 0; q < 9; ++q) sb[fm * 9 + q][cl] = binv[q];
    __syncthreads();
    if (!ok) return;
    T a[9], M[6];
#pragma unroll
    for (int r = 0; r < 9; ++r) a[r] = (T)a64[r];
#pragma unroll
    for (int q = 0; q < 6; ++q) M[q] = (T)geo[1 + q];
    T b[8][3];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < 3; ++u) t = fma(sb[(m * 3 + k) * 3 + u][cl], d[HEXSUB[m][u]], t);
            b[m][k] = (T)t;
        }
    // smoothness indicators in scaled coordinates (mean over the cell of the squared
    // first derivatives, plus the squared second derivatives of P0)
    T beta[9];
    beta[0] = a[0] * a[0] + quad_form(M, T(2) * a[3], a[6], a[7]) + a[1] * a[1] + quad_form(M, a[6], T(2) * a[4], a[8]) +
              a[2] * a[2] + quad_form(M, a[7], a[8], T(2) * a[5]) +
              T(4) * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) beta[1 + m] = b[m][0] * b[m][0] + b[m][1] * b[m][1] + b[m][2] * b[m][2];
    const T gl = (T)P.gamma_lin, g0 = T(1) - T(8) * gl, eps = (T)P.weno_eps;
    T tauZ = T(0);
#pragma unroll
    for (int m = 1; m < 9; ++m) tauZ += hg_abs(beta[0] - beta[m]);
    tauZ *= T(0.125);
    T w[9], ws = T(0);
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        w[m] = (m == 0 ? g0 : gl) * (T(1) + tauZ * hg_rcp(beta[m] + eps));
        ws += w[m];
    }
    const T inv = hg_rcp(ws);
    const T s0 = w[0] * inv * hg_rcp(g0);
    const T ih = (T)geo[0], ih2 = ih * ih;
    T c[10];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = s0 * a[k];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const T al = w[1 + m] * inv - s0 * gl;
#pragma unroll
        for (int k = 0; k < 3; ++k) c[1 + k] += al * b[m][k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] *= ih;
    T dev = T(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const T cq = s0 * a[3 + q];
        dev -= cq * M[q];
        c[4 + q] = cq * ih2;
    }
    if constexpr (!MIXED) {
        c[0] = qi + dev;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            stg<d2>(reinterpret_cast<d2 *>(P.C) + (size_t)(v * 5 + k) * nc, i * 16u, d2{c[2 * k], c[2 * k + 1]});
    } else {
        c[0] = dev;                       // deviation from the FP64 cell mean
#pragma unroll
        for (int k = 0; k < 5; ++k)
            stg<f2>(reinterpret_cast<f2 *>(P.C32) + (size_t)(v * 5 + k) * nc, i * 8u, f2{c[2 * k], c[2 * k + 1]});
    }
}

// The two sides of Gauss point g of face f in precision T: the left reconstruction,
// and on the right the right cell's, or at a listed boundary face the ghost's (wall:
// the momentum negated and the gradient reflected in the face's mean plane; far
// field: the Riemann-invariant state of the left value for the point's normal, no
// gradient).  Where a side is non-physical the point is first order (zero
// gradients, cell averages for the non-physical sides; the ghost's average is the
// ghost state of the left cell's).  Returns the point's normal and weight.
template <class T, bool REC32>
__device__ __forceinline__ void hex_point(const ProbDesc &P, int stage, uint32_t f, uint32_t g, T n[3], double &w,
                                          T qL[5], T gL[5][3], T qR[5], T gR[5][3]) {
    const uint32_t nf = (uint32_t)P.nf;
    auto fg = [&](uint32_t k) { return ldg<double>(P.fgeo + (size_t)k * nf, f * 8u); };
    T yl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        n[a] = (T)fg(7 * g + a);
        yl[a] = (T)fg(7 * g + 4 + a);
    }
    w = fg(7 * g + 3);
    const uint32_t l = (uint32_t)ldg<int32_t>(P.fcell, f * 4u);
    const int32_t r = ldg<int32_t>(P.fcell + nf, f * 4u);
    recon_point<T, false, REC32>(P, stage, l, yl, qL, gL);
    T nm[3];
    if (r >= 0) {
        T yr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) yr[a] = yl[a] + (T)fg(28 + a);
        recon_point<T, false, REC32>(P, stage, (uint32_t)r, yr, qR, gR);
    } else if (r == -HGKS_BC_WALL) {
#pragma unroll
        for (int a = 0; a < 3; ++a) nm[a] = (T)fg(31 + a);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T sg = (q >= 1 && q <= 3) ? T(-1) : T(1);
            const T gn = gL[q][0] * nm[0] + gL[q][1] * nm[1] + gL[q][2] * nm[2];
            qR[q] = sg * qL[q];
#pragma unroll
            for (int a = 0; a < 3; ++a) gR[q][a] = sg * (gL[q][a] - T(2) * gn * nm[a]);
        }
    } else {
        farfield_state<T>(P, qL, n, qR);
#pragma unroll
        for (int q = 0; q < 5; ++q) gR[q][0] = gR[q][1] = gR[q][2] = T(0);
    }
    const bool okL = physical_point(qL), okR = physical_point(qR);
    if (!(okL && okR)) {
        T ml[5];
        cell_mean<T>(P, stage, l, ml);
        if (!okL)
#pragma unroll
            for (int q = 0; q < 5; ++q) qL[q] = ml[q];
        if (!okR) {
            if (r >= 0) {
                cell_mean<T>(P, stage, (uint32_t)r, qR);
            } else if (r == -HGKS_BC_WALL) {
#pragma unroll
                for (int q = 0; q < 5; ++q) qR[q] = (q >= 1 && q <= 3) ? -ml[q] : ml[q];
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) nm[a] = (T)fg(31 + a);
                farfield_state<T>(P, ml, nm, qR);
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a) gL[q][a] = gR[q][a] = T(0);
    }
}

// Point flux of Gauss point g of face f in precision T (TM: tau mode), times the
// point's weight.  With T = float a point with a cold side under tau > 0
// (warm_point), or whose flux is not finite, is refused (false): its face is then
// evaluated in FP64 by the fix-up pass, as on tetrahedra.
template <class T, bool REC32, int TM>
__device__ __forceinline__ bool hex_point_flux(const ProbDesc &P, int stage, uint32_t f, uint32_t g, double Fo[5],
                                               double dFo[5]) {
    T n[3], qL[5], gL[5][3], qR[5], gR[5][3], F[5], dF[5];
    double w;
    hex_point<T, REC32>(P, stage, f, g, n, w, qL, gL, qR, gR);
    if constexpr (sizeof(T) == 4 && TM != 0)
        if (!(warm_point(qL) && warm_point(qR))) return false;
    if constexpr (TM == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a) gL[q][a] += gR[q][a];
        gks_flux_tau0<T>(qL, qR, gL, n, P, F, dF);
    } else {
        gks_flux_full<T, TM == 2>(qL, gL, qR, gR, n, (T)ldg<double>(P.dt, 0u), P, F, dF);
    }
    if constexpr (sizeof(T) == 4)
        if (!finite_flux(F, dF)) return false;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        Fo[k] = w * (double)F[k];
        dFo[k] = w * (double)dF[k];
    }
    return true;
}

// Face flux on hexahedra: four consecutive lanes take the four Gauss points of a
// face and sum their weighted fluxes across the lanes ((g0 + g1) + (g2 + g3)); the
// first lane writes S-weighted (F, dF) to the per-face buffer.
// FP32-mixed: a point the FP32 flux refuses makes its face's sum NaN, and the face is
// left to the FP64 pass below (flag[1] raised, cleared by the stage update), as on
// tetrahedra; with no FP64 code inline the FP32 kernels need 113 / 129 / 208 registers
// (tau = 0 / shock mode / viscous) instead of 155 / 256 / 256 plus 264 spilled.
// Two waves per SIMD, except the FP64 viscous variant: held to 256 registers it spills
// some 700 bytes a lane and runs at less than half the speed of one wave with its
// 256 + 174 registers (1.9 against 4.4 ms a launch on the 884,736-cell O-grid).
template <bool MIXED, int TM>
__global__ __launch_bounds__(4 * HEX_FLUX_FACES) __attribute__((amdgpu_waves_per_eu((MIXED || TM != 2) ? 2 : 1))) void k_flux_hex(
    const ProbDesc *__restrict__ probs, const Tile *__restrict__ tiles, int stage) {
    const Tile tl = tiles[blockIdx.x];
    const ProbDesc &P = probs[tl.prob];
    const uint32_t g = threadIdx.x & 3u;
    const uint32_t f = (uint32_t)tl.begin + threadIdx.x / 4u;
    const bool ok = f < (uint32_t)tl.end;
    double Fo[5], dFo[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Fo[k] = dFo[k] = 0.0;
    if (ok) {
        if constexpr (MIXED) {
            if (!hex_point_flux<float, true, TM>(P, stage, f, g, Fo, dFo)) Fo[0] = __builtin_nan("");
        } else {
            hex_point_flux<double, false, TM>(P, stage, f, g, Fo, dFo);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        Fo[k] += __shfl_xor(Fo[k], 1);
        Fo[k] += __shfl_xor(Fo[k], 2);
        dFo[k] += __shfl_xor(dFo[k], 1);
        dFo[k] += __shfl_xor(dFo[k], 2);
    }
    if (ok && g == 0) {
        const uint32_t nf = (uint32_t)P.nf;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            stg_nt<double>(P.FF + (size_t)k * nf, f * 8u, Fo[k]);
            stg_nt<double>(P.FF + (size_t)(5 + k) * nf, f * 8u, dFo[k]);
        }
    }
    if constexpr (MIXED) {
        const uint64_t bad = __ballot(ok && g == 0u && !(Fo[0] - Fo[0] == 0.0));
        if (bad != 0 && (threadIdx.x & 63u) == 0) P.flag[1] = 1;
    }
}

// Faces the FP32-mixed hexahedral flux left (a NaN flux): the four Gauss points again
// in FP64 from the FP32 records, summed in the same order.  One lane a face, a grid
// stride over the face tiles, after one look at the flag (nothing to do is the
// common case); the recomputation is rare and may use scratch memory.
template <int TM>
__global__ __launch_bounds__(HEX_FLUX_FACES) void k_flux_hex_fix(const ProbDesc *__restrict__ d,
                                                                  const Tile *__restrict__ tiles, int ntiles, int stage) {
    const ProbDesc &P = *d;
    if (ldg<int32_t>(P.flag, 4u) == 0) return;
    const uint32_t nf = (uint32_t)P.nf;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const uint32_t f = (uint32_t)tl.begin + threadIdx.x;
        if (f >= (uint32_t)tl.end) continue;
        const double f0 = P.FF[f];
        if (f0 - f0 == 0.0) continue;                     // finite: done in FP32
        double F[4][5], dF[4][5];
#pragma unroll 1
        for (uint32_t g = 0; g < 4u; ++g) hex_point_flux<double, true, TM>(P, stage, f, g, F[g], dF[g]);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            P.FF[(size_t)k * nf + f] = (F[0][k] + F[1][k]) + (F[2][k] + F[3][k]);
            P.FF[(size_t)(5 + k) * nf + f] = (dF[0][k] + dF[1][k]) + (dF[2][k] + dF[3][k]);
        }
    }
}

// ----------------------------------------------------------------------------
// launch wrappers
// ----------------------------------------------------------------------------
constexpr int WENO_CELLS = HGKS_WENO_CELLS;     // cells per WENO workgroup (16, 32 or 64)

void launch_weno(const ProbDesc *probs, const Tile *tiles, int ntiles, int stage, int prec, bool walls,
                 hipStream_t s) {
    if (ntiles <= 0) return;
    dim3 g(ntiles * (WENO_TILE / WENO_CELLS)), b(weno_threads<WENO_CELLS>());
#define HGKS_WENO(M, WA) hipLaunchKernelGGL((k_weno<M, WENO_CELLS, WA>), g, b, 0, s, probs, tiles, stage)
    if (prec == 2) { if (walls) HGKS_WENO(2, true); else HGKS_WENO(2, false); }
    else if (prec == 1) { if (walls) HGKS_WENO(1, true); else HGKS_WENO(1, false); }
    else { if (walls) HGKS_WENO(0, true); else HGKS_WENO(0, false); }
#undef HGKS_WENO
}

// Compute units of the current device (queried once per device).
static int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

void launch_flux(const ProbDesc *probs, int nprobs, const Tile *tiles, int ntiles, int stage, int prec, bool tau0,
                 bool coloured, bool walls, hipStream_t s) {
    if (ntiles <= 0) return;
    // prec 0: FP64; 1: FP32 flux on FP64 storage; 2: FP32 flux on FP32 storage
    const bool mixed = prec != 0;
    if (tau0) {
        dim3 g(ntiles), b(FACE_TILE);
#define HGKS_FLUX0(M, CO, D, S)                                                                             \
    do {                                                                                                    \
        if (walls) hipLaunchKernelGGL((k_flux_t0<M, CO, true, D, S>), g, b, 0, s, probs, tiles, stage);     \
        else hipLaunchKernelGGL((k_flux_t0<M, CO, false, D, S>), g, b, 0, s, probs, tiles, stage);          \
    } while (0)
#define HGKS_FLUX0P(CO, D)                                                                                  \
    do {                                                                                                    \
        if (prec == 2) HGKS_FLUX0(true, CO, D, true);                                                       \
        else if (prec == 1) HGKS_FLUX0(true, CO, D, false);                                                 \
        else HGKS_FLUX0(false, CO, D, false);                                                               \
    } while (0)
        if (coloured) HGKS_FLUX0P(true, false);
        else if (stage == 1) HGKS_FLUX0P(false, false);
        else HGKS_FLUX0P(false, true);
#undef HGKS_FLUX0P
#undef HGKS_FLUX0
        if (!coloured) {
            const dim3 gf(std::min(ntiles, 8 * device_cus()));
            if (prec == 2) hipLaunchKernelGGL((k_flux_fix<true, true>), gf, b, 0, s, probs, nprobs, tiles, ntiles, stage);
            else if (prec == 1) hipLaunchKernelGGL((k_flux_fix<true, false>), gf, b, 0, s, probs, nprobs, tiles, ntiles, stage);
            else hipLaunchKernelGGL((k_flux_fix<false, false>), gf, b, 0, s, probs, nprobs, tiles, ntiles, stage);
        }
        return;
    }
    if (!coloured) {          // tiles of 3 * GP_FACES faces, three single-wave workgroups each
        dim3 g(ntiles * 3), b(64);
#define HGKS_GP(M, W, S) hipLaunchKernelGGL((k_flux_gp<M, W, S>), g, b, 0, s, probs, tiles, stage)
        if (prec == 2) { if (walls) HGKS_GP(true, true, true); else HGKS_GP(true, false, true); }
        else if (prec == 1) { if (walls) HGKS_GP(true, true, false); else HGKS_GP(true, false, false); }
        else { if (walls) HGKS_GP(false, true, false); else HGKS_GP(false, false, false); }
#undef HGKS_GP
        if (mixed) {            // faces left to FP64 by the FP32 pass
            const dim3 gf(std::min(ntiles, 8 * device_cus())), bf(64);
#define HGKS_FIX(W, S) hipLaunchKernelGGL((k_flux_fix_full<W, S>), gf, bf, 0, s, probs, nprobs, tiles, ntiles, stage)
            if (prec == 2) { if (walls) HGKS_FIX(true, true); else HGKS_FIX(false, true); }
            else { if (walls) HGKS_FIX(true, false); else HGKS_FIX(false, false); }
#undef HGKS_FIX
        }
        return;
    }
    // tau > 0 with colour classes: one wave per Gauss point, summed through LDS
    dim3 g(ntiles), b(3 * FACE_TILE);
#define HGKS_FLUX(M, S)                                                                                     \
    do {                                                                                                    \
        if (walls) hipLaunchKernelGGL((k_flux<M, false, true, true, S>), g, b, 0, s, probs, tiles, stage);  \
        else hipLaunchKernelGGL((k_flux<M, false, true, false, S>), g, b, 0, s, probs, tiles, stage);       \
    } while (0)
    if (prec == 2) HGKS_FLUX(true, true);
    else if (prec == 1) HGKS_FLUX(true, false);
    else HGKS_FLUX(false, false);
#undef HGKS_FLUX
}

void launch_hex_ghost(const ProbDesc *d, int ng, int stage, hipStream_t s) {
    if (ng <= 0) return;
    hipLaunchKernelGGL(k_ghost_hex, dim3((ng + 255) / 256), dim3(256), 0, s, d, stage);
}

void launch_hex_weno(const ProbDesc *d, const Tile *tiles, int ntiles, int stage, bool mixed, hipStream_t s) {
    if (ntiles <= 0) return;
    const dim3 g(ntiles * (HEX_WENO_CELLS / HEX_WC)), b(weno_threads<HEX_WC>());
    if (mixed) hipLaunchKernelGGL((k_weno_hex<true, 2>), g, b, 0, s, d, tiles, stage);
    else hipLaunchKernelGGL((k_weno_hex<false, 2>), g, b, 0, s, d, tiles, stage);
}

void launch_hex_flux(const ProbDesc *d, const Tile *tiles, int ntiles, int stage, bool mixed, int tau_mode,
                     hipStream_t s) {
    if (ntiles <= 0) return;
    dim3 g(ntiles), b(4 * HEX_FLUX_FACES);
#define HGKS_HF(M, TM) hipLaunchKernelGGL((k_flux_hex<M, TM>), g, b, 0, s, d, tiles, stage)
    if (mixed) {
        if (tau_mode == 0) HGKS_HF(true, 0); else if (tau_mode == 1) HGKS_HF(true, 1); else HGKS_HF(true, 2);
    } else {
        if (tau_mode == 0) HGKS_HF(false, 0); else if (tau_mode == 1) HGKS_HF(false, 1); else HGKS_HF(false, 2);
    }
#undef HGKS_HF
    if (mixed) {              // faces left to FP64 by the FP32 pass
        const dim3 gf(std::min(ntiles, 8 * device_cus())), bf(HEX_FLUX_FACES);
#define HGKS_HX(TM) hipLaunchKernelGGL((k_flux_hex_fix<TM>), gf, bf, 0, s, d, tiles, ntiles, stage)
        if (tau_mode == 0) HGKS_HX(0); else if (tau_mode == 1) HGKS_HX(1); else HGKS_HX(2);
#undef HGKS_HX
    }
}

void launch_update(const ProbDesc *probs, const Tile *tiles, int ntiles, int stage, bool coloured, bool s32,
                   hipStream_t s, int faces_per_cell) {
    if (ntiles <= 0) return;
    dim3 g(ntiles), b(UPD_TILE);
    if (faces_per_cell == 6) {          // hexahedra: FP64 storage, per-face buffer
        if (stage == 1) hipLaunchKernelGGL((k_update<1, false, false, 6>), g, b, 0, s, probs, tiles);
        else hipLaunchKernelGGL((k_update<2, false, false, 6>), g, b, 0, s, probs, tiles);
        return;
    }
#define HGKS_UPD(ST, CO, S) hipLaunchKernelGGL((k_update<ST, CO, S>), g, b, 0, s, probs, tiles)
    if (stage == 1) {
        if (s32) { if (coloured) HGKS_UPD(1, true, true); else HGKS_UPD(1, false, true); }
        else { if (coloured) HGKS_UPD(1, true, false); else HGKS_UPD(1, false, false); }
    } else {
        if (s32) { if (coloured) HGKS_UPD(2, true, true); else HGKS_UPD(2, false, true); }
        else { if (coloured) HGKS_UPD(2, true, false); else HGKS_UPD(2, false, false); }
    }
#undef HGKS_UPD
}

void launch_dt_local(const ProbDesc *probs, const Tile *tiles, int ntiles, bool s32, hipStream_t s) {
    if (ntiles <= 0) return;
    if (s32) hipLaunchKernelGGL(k_dt_local<true>, dim3(ntiles), dim3(UPD_TILE), 0, s, probs, tiles);
    else hipLaunchKernelGGL(k_dt_local<false>, dim3(ntiles), dim3(UPD_TILE), 0, s, probs, tiles);
}

void launch_dt_final(const ProbDesc *probs, int nprobs, double dt_fixed, hipStream_t s) {
    if (nprobs <= 0) return;
    hipLaunchKernelGGL(k_dt_final, dim3(nprobs), dim3(1024), 0, s, probs, dt_fixed);
}

void launch_fill(double *p, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

// ----------------------------------------------------------------------------
// Static launch tables (the allocation-free pool step): one file-scope device
// array per GPU, holding the problem descriptors and tile tables of the last
// batch stepped through it.  In host code `scratch` names a host-side stand-in,
// not device memory, so only the address fetched from the runtime below is ever
// handed to kernels or copies.
// ----------------------------------------------------------------------------
static __device__ __align__(256) char scratch[STATIC_TABLE_BYTES];

hipError_t static_table_ptr(int device, void **ptr) {
    static std::mutex mu;
    static std::vector<void *> addr;         // per device; null until fetched
    std::lock_guard<std::mutex> g(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
    if (!addr[(size_t)device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[(size_t)device] = p;
    }
    *ptr = addr[(size_t)device];
    return hipSuccess;
}

}  // namespace hgks
