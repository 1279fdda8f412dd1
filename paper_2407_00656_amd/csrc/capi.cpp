// C ABI of the HGKS library: contexts (one problem each), the step driver and
// the pool that batches many contexts into shared launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hgks.h"
#include "hgks_internal.h"
#include "kernels.h"

using namespace hgks;

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Workgroups are handed to the eight XCDs round-robin by workgroup id.  Give
// each XCD a contiguous run of tiles so that the stencil / neighbour data a
// tile shares with the next one sits in the same XCD's L2.
template <class T>
void xcd_order(std::vector<T> &tiles, size_t b, size_t e) {
    const size_t n = e - b;
    if (n < 16) return;
    std::vector<T> src(tiles.begin() + b, tiles.begin() + e);
    size_t start[8];
    size_t s = 0;
    for (int x = 0; x < 8; ++x) {
        start[x] = s;
        s += (n > (size_t)x) ? (n - x + 7) / 8 : 0;
    }
    for (size_t k = 0; k < n; ++k) tiles[b + k] = src[start[k % 8] + k / 8];
}

struct Layout {
    size_t sten, pinv0, cen, sshift, cgeo, cface, fcell, fgeo, Q, Qs, R, C, C32, FF, acc, dtpart, scal, desc, tiles, total;
};

Layout layout_for(int64_t nc, int64_t nf, int n_ctiles, int n_ftiles, int prec, bool coloured) {
    const bool mixed = prec != HGKS_FP64;
    // the FP32 form stores the state, the cell and face geometry and the face fluxes
    // in FP32 (es = 4): the same row layouts with half the element size
    const size_t es = prec == HGKS_FP32 ? 4 : 8;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t p = o; o += up(bytes); return p; };
    L.sten = take((size_t)SLOTS * nc * 4);
    L.pinv0 = take((size_t)144 * nc * (prec == HGKS_FP32 ? 4 : 8));
    L.cen = take((size_t)3 * nc * 8);
    L.sshift = take((size_t)4 * nc * 4);
    L.cgeo = take((size_t)CGEO * nc * es);
    L.cface = take((size_t)4 * nc * 4);
    L.fcell = take((size_t)2 * nf * 4);
    L.fgeo = take((size_t)FGEO * nf * es);
    L.Q = take((size_t)5 * nc * es);
    L.Qs = take((size_t)5 * nc * es);
    L.R = take((size_t)5 * nc * es);
    L.C = take(mixed ? 0 : (size_t)5 * NCOEF * nc * 8);
    L.C32 = take(mixed ? (size_t)5 * NCOEF * nc * 4 : 0);
    L.FF = take(coloured ? 0 : (size_t)10 * nf * es);
    L.acc = take(coloured ? (size_t)10 * nc * es : 0);
    L.dtpart = take((size_t)n_ctiles * 8);
    L.scal = take(64);
    L.desc = take(sizeof(ProbDesc));
    L.tiles = take((size_t)(n_ctiles + n_ftiles) * sizeof(Tile));
    L.total = o;
    return L;
}

int n_cell_tiles(int64_t nc) { return (int)((nc + UPD_TILE - 1) / UPD_TILE); }

}  // namespace

struct hgks_ctx {
    hgks_params prm{};
    int device = 0;
    hipStream_t stream = nullptr;
    hgks_allocator alloc{};
    bool user_alloc = false;
    std::string err;
    bool has_mesh = false, has_state = false;
    bool walls = false;           // the mesh has wall faces (a non-periodic axis)
    bool hex = false;             // hexahedral mesh (its own kernels; steps alone, not in a pool)
    int64_t ng = 0;               // ghosts of listed boundary faces (hexahedra)
    int ns = 0;                   // stencil slots (hexahedra)
    int64_t nc = 0, nf = 0;
    std::vector<int64_t> perm;
    std::vector<int32_t> colour_offsets;   // face offsets of each colour class
    std::vector<int32_t> colour_tiles;     // tile offsets of each colour class
    char *base = nullptr;                  // the one device allocation
    size_t bytes = 0;
    ProbDesc desc{};
    ProbDesc *d_desc = nullptr;
    Tile *d_ctiles = nullptr, *d_ftiles = nullptr;
    int n_ctiles = 0, n_ftiles = 0;
    std::vector<Tile> h_ctiles, h_ftiles;  // host copies (pool builds its tables from them)
    // profiling
    bool prof = false;
    struct Rec { int id; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> spare;
    double prof_ms[4] = {0, 0, 0, 0};
    int64_t prof_n[4] = {0, 0, 0, 0};
    bool own_stream = false;              // the stream was created here (HGKS_OWN_STREAM)
    int pool_refs = 0;
    hgks_pool *pool = nullptr;            // the pool holding this context (at most one)
    hipStream_t pool_stream = nullptr;    // stream of the pool holding this context
};

void pool_detach(hgks_pool *p, hgks_ctx *c);

namespace {

hgks_status fail(hgks_ctx *c, hgks_status s, const std::string &m) {
    if (c) c->err = m;
    return s;
}

hgks_status hip_fail(hgks_ctx *c, hipError_t e, const char *what) {
    return fail(c, HGKS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, x)                                    \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #x); \
    } while (0)

void release(hgks_ctx *c) {
    if (c->base) {
        if (c->user_alloc)
            c->alloc.free(c->base, c->stream, c->alloc.user);
        else
            (void)hipFree(c->base);
    }
    c->base = nullptr;
    c->bytes = 0;
    c->has_mesh = c->has_state = false;
}

hipEvent_t take_event(hgks_ctx *c) {
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` on the context's stream, bracketed by events when profiling.
template <class F>
void timed(hgks_ctx *c, int id, F &&launch) {
    if (!c->prof) {
        launch();
        return;
    }
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) {
        launch();
        return;
    }
    (void)hipEventRecord(a, c->stream);
    launch();
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({id, a, b});
}

void collect_profile(hgks_ctx *c) {
    for (auto &r : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_ms[r.id] += ms;
            c->prof_n[r.id] += 1;
        }
        c->spare.push_back(r.a);
        c->spare.push_back(r.b);
    }
    c->pending.clear();
}

bool tau0_of(const hgks_params &p) { return p.tau_mode == 0; }

hgks_status check_params(const hgks_params *p) {
    if (!p) return HGKS_E_INVALID_ARG;
    if (!(p->gamma > 1.0 && p->gamma < 5.0 / 3.0 + 1e-12)) return HGKS_E_INVALID_ARG;
    if (!(p->cfl > 0.0) || !(p->weno_eps > 0.0) || !(p->gamma_lin > 0.0 && p->gamma_lin < 0.25)) return HGKS_E_INVALID_ARG;
    if (p->tau_mode < 0 || p->tau_mode > 2) return HGKS_E_INVALID_ARG;
    if (p->tau_mode == 2) {
        if (!(p->mu_ref >= 0.0) || !(p->T_ref > 0.0) || !std::isfinite(p->mu_exp) || !(p->prandtl > 0.0) ||
            !(p->tau_C >= 0.0))
            return HGKS_E_INVALID_ARG;
        if (!(p->farfield[0] > 0.0) || !(p->farfield[4] > 0.0)) return HGKS_E_INVALID_ARG;
    }
    if (p->precision != HGKS_FP64 && p->precision != HGKS_FP32_MIXED && p->precision != HGKS_FP32)
        return HGKS_E_INVALID_ARG;
    if (p->accumulation != HGKS_ACC_GATHER && p->accumulation != HGKS_ACC_COLOURED) return HGKS_E_INVALID_ARG;
    return HGKS_OK;
}

// Queue one S2O4 step of a hexahedral context: per stage the ghost states, WENO,
// the Gauss-point flux into the per-face buffer and the six-face update.
void enqueue_step_hex(hgks_ctx *c, double dt_fixed) {
    const bool mixed = c->prm.precision != HGKS_FP64;
    hipStream_t s = c->stream;
    timed(c, 0, [&] { launch_dt_final(c->d_desc, 1, dt_fixed, s); });
    for (int stage = 1; stage <= 2; ++stage) {
        timed(c, 1, [&] {
            launch_hex_ghost(c->d_desc, (int)c->ng, stage, s);
            launch_hex_weno(c->d_desc, c->d_ctiles, c->n_ctiles, stage, mixed, s);
        });
        timed(c, 2, [&] { launch_hex_flux(c->d_desc, c->d_ftiles, c->n_ftiles, stage, mixed, c->prm.tau_mode, s); });
        timed(c, 3, [&] { launch_update(c->d_desc, c->d_ctiles, c->n_ctiles, stage, false, false, s, 6); });
    }
}

// Queue one S2O4 step of a single context.
void enqueue_step(hgks_ctx *c, double dt_fixed) {
    if (c->hex) {
        enqueue_step_hex(c, dt_fixed);
        return;
    }
    const int prec = c->prm.precision;
    const bool mixed = prec != HGKS_FP64;
    const bool tau0 = tau0_of(c->prm);
    const bool col = c->prm.accumulation == HGKS_ACC_COLOURED;
    hipStream_t s = c->stream;
    timed(c, 0, [&] { launch_dt_final(c->d_desc, 1, dt_fixed, s); });
    for (int stage = 1; stage <= 2; ++stage) {
        timed(c, 1, [&] { launch_weno(c->d_desc, c->d_ctiles, c->n_ctiles, stage, prec, c->walls, s); });
        if (col) {
            for (size_t k = 0; k + 1 < c->colour_tiles.size(); ++k) {
                int t0 = c->colour_tiles[k], t1 = c->colour_tiles[k + 1];
                timed(c, 2, [&] { launch_flux(c->d_desc, 1, c->d_ftiles + t0, t1 - t0, stage, prec, tau0, true, c->walls, s); });
            }
        } else {
            timed(c, 2, [&] { launch_flux(c->d_desc, 1, c->d_ftiles, c->n_ftiles, stage, prec, tau0, false, c->walls, s); });
        }
        timed(c, 3, [&] { launch_update(c->d_desc, c->d_ctiles, c->n_ctiles, stage, col, prec == HGKS_FP32, s); });
    }
}

// Device layout of a hexahedral context (FP64 storage; the FP32-mixed form keeps
// FP32 reconstruction records).
struct HexLayout {
    size_t sten, pinv, binv, cgeo, cface, fcell, fgeo, gcell, gkind, gnrm, G, Q, Qs, R, C, FF, dtpart, scal, desc,
        tiles, total;
};

HexLayout hex_layout(int64_t nc, int64_t nf, int64_t ng, int ns, int n_ctiles, int n_ftiles, bool mixed) {
    HexLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t p = o; o += up(bytes); return p; };
    const size_t g1 = (size_t)std::max<int64_t>(ng, 1);
    L.sten = take((size_t)ns * nc * 4);
    L.pinv = take((size_t)9 * ns * nc * 8);
    L.binv = take((size_t)HEX_BINV * nc * 8);
    L.cgeo = take((size_t)CGEO * nc * 8);
    L.cface = take((size_t)6 * nc * 4);
    L.fcell = take((size_t)2 * nf * 4);
    L.fgeo = take((size_t)HEX_FGEO * nf * 8);
    L.gcell = take(g1 * 4);
    L.gkind = take(g1 * 4);
    L.gnrm = take(3 * g1 * 8);
    L.G = take(5 * g1 * 8);
    L.Q = take((size_t)5 * nc * 8);
    L.Qs = take((size_t)5 * nc * 8);
    L.R = take((size_t)5 * nc * 8);
    L.C = take((size_t)5 * NCOEF * nc * (mixed ? 4 : 8));
    L.FF = take((size_t)10 * nf * 8);
    L.dtpart = take((size_t)n_ctiles * 8);
    L.scal = take(64);
    L.desc = take(sizeof(ProbDesc));
    L.tiles = take((size_t)(n_ctiles + n_ftiles) * sizeof(Tile));
    L.total = o;
    return L;
}

void fill_constants(ProbDesc &D, const hgks_params &p) {
    D.gamma = p.gamma;
    D.K = (5.0 - 3.0 * p.gamma) / (p.gamma - 1.0);
    D.weno_eps = p.weno_eps;
    D.gamma_lin = p.gamma_lin;
    D.cfl = p.cfl;
    D.tau_eps = p.tau_eps;
    D.tau_C = p.tau_C;
    D.tau_mode = p.tau_mode;
    D.mixed = p.precision != HGKS_FP64 ? 1 : 0;
    D.mu_ref = p.mu_ref;
    D.T_ref = p.T_ref;
    D.mu_exp = p.mu_exp;
    D.prandtl = p.prandtl;
    for (int k = 0; k < 5; ++k) D.farfield[k] = p.farfield[k];
}

hgks_status upload_hex(hgks_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_cells, const int64_t *cell_nodes,
                       const double *period, int64_t n_bfaces, const int64_t *bface_nodes, const int32_t *bface_kind) {
    if (c->prm.precision == HGKS_FP32)
        return fail(c, HGKS_E_INVALID_ARG, "hexahedral meshes take the FP64 and FP32-mixed precisions");
    if (c->prm.accumulation != HGKS_ACC_GATHER)
        return fail(c, HGKS_E_INVALID_ARG, "hexahedral meshes take the gather accumulation");
    HexMesh hm;
    std::string err;
    hgks_status st = build_hex_mesh(c->prm, n_nodes, xyz, n_cells, cell_nodes, period, n_bfaces, bface_nodes,
                                    bface_kind, hm, err);
    if (st != HGKS_OK) return fail(c, st, err);
    HIPCHK(c, hipSetDevice(c->device));
    release(c);
    const bool mixed = c->prm.precision != HGKS_FP64;
    std::vector<Tile> ct, ft;
    const int nct = n_cell_tiles(hm.nc);
    for (int t = 0; t < nct; ++t) {
        int b = t * UPD_TILE;
        ct.push_back({0, b, t, (int32_t)std::min<int64_t>(hm.nc, b + UPD_TILE)});
    }
    xcd_order(ct, 0, ct.size());
    for (int64_t b = 0; b < hm.nf; b += HEX_FLUX_FACES)
        ft.push_back({0, (int32_t)b, (int)ft.size(), (int32_t)std::min<int64_t>(hm.nf, b + HEX_FLUX_FACES)});
    xcd_order(ft, 0, ft.size());
    HexLayout L = hex_layout(hm.nc, hm.nf, hm.ng, hm.ns, (int)ct.size(), (int)ft.size(), mixed);
    void *mem = nullptr;
    if (c->user_alloc) {
        mem = c->alloc.alloc(L.total, c->stream, c->alloc.user);
        if (!mem) return fail(c, HGKS_E_OOM, "allocator returned NULL");
    } else {
        hipError_t e = hipMalloc(&mem, L.total);
        if (e != hipSuccess) return fail(c, HGKS_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    c->base = (char *)mem;
    c->bytes = L.total;
    char *B = c->base;
    ProbDesc &D = c->desc;
    D = ProbDesc{};
    D.nc = (int32_t)hm.nc;
    D.nf = (int32_t)hm.nf;
    D.n_cell_tiles = (int32_t)ct.size();
    D.ns = hm.ns;
    D.ng = (int32_t)hm.ng;
    D.sten = (const int32_t *)(B + L.sten);
    D.hpinv = (const double *)(B + L.pinv);
    D.hbinv = (const double *)(B + L.binv);
    D.cgeo = (const double *)(B + L.cgeo);
    D.cface = (const int32_t *)(B + L.cface);
    D.fcell = (const int32_t *)(B + L.fcell);
    D.fgeo = (const double *)(B + L.fgeo);
    D.gcell = (const int32_t *)(B + L.gcell);
    D.gkind = (const int32_t *)(B + L.gkind);
    D.gnrm = (const double *)(B + L.gnrm);
    D.G = (double *)(B + L.G);
    D.Q = (double *)(B + L.Q);
    D.Qs = (double *)(B + L.Qs);
    D.R = (double *)(B + L.R);
    D.C = mixed ? nullptr : (double *)(B + L.C);
    D.C32 = mixed ? (float *)(B + L.C) : nullptr;
    D.FF = (double *)(B + L.FF);
    D.dtpart = (double *)(B + L.dtpart);
    D.dt = (double *)(B + L.scal);
    D.time = (double *)(B + L.scal + 8);
    D.flag = (int32_t *)(B + L.scal + 16);
    fill_constants(D, c->prm);
    c->d_desc = (ProbDesc *)(B + L.desc);
    c->d_ctiles = (Tile *)(B + L.tiles);
    c->d_ftiles = c->d_ctiles + ct.size();
    c->n_ctiles = (int)ct.size();
    c->n_ftiles = (int)ft.size();
    c->h_ctiles = ct;
    c->h_ftiles = ft;
    hipStream_t s = c->stream;
    auto h2d = [&](const void *dst, const void *src, size_t n) {
        return hipMemcpyAsync((void *)dst, src, n, hipMemcpyHostToDevice, s);
    };
    HIPCHK(c, h2d(D.sten, hm.sten.data(), hm.sten.size() * 4));
    HIPCHK(c, h2d(D.hpinv, hm.pinv.data(), hm.pinv.size() * 8));
    HIPCHK(c, h2d(D.hbinv, hm.binv.data(), hm.binv.size() * 8));
    HIPCHK(c, h2d(D.cgeo, hm.cgeo.data(), hm.cgeo.size() * 8));
    HIPCHK(c, h2d(D.cface, hm.cface.data(), hm.cface.size() * 4));
    HIPCHK(c, h2d(D.fcell, hm.fcell.data(), hm.fcell.size() * 4));
    HIPCHK(c, h2d(D.fgeo, hm.fgeo.data(), hm.fgeo.size() * 8));
    if (hm.ng > 0) {
        HIPCHK(c, h2d(D.gcell, hm.gcell.data(), hm.gcell.size() * 4));
        HIPCHK(c, h2d(D.gkind, hm.gkind.data(), hm.gkind.size() * 4));
        HIPCHK(c, h2d(D.gnrm, hm.gnrm.data(), (size_t)3 * hm.ng * 8));
    }
    HIPCHK(c, h2d(c->d_desc, &D, sizeof(ProbDesc)));
    HIPCHK(c, h2d(c->d_ctiles, ct.data(), ct.size() * sizeof(Tile)));
    HIPCHK(c, h2d(c->d_ftiles, ft.data(), ft.size() * sizeof(Tile)));
    HIPCHK(c, hipStreamSynchronize(s));
    c->nc = hm.nc;
    c->nf = hm.nf;
    c->ng = hm.ng;
    c->ns = hm.ns;
    c->perm = std::move(hm.perm);
    c->colour_offsets.assign({0, (int32_t)hm.nf});
    c->walls = false;
    c->hex = true;
    c->has_mesh = true;
    c->has_state = false;
    return HGKS_OK;
}

}  // namespace

extern "C" {

void hgks_default_params(hgks_params *p) {
    if (!p) return;
    p->gamma = 1.4;
    p->cfl = 0.3;
    p->tau_mode = 0;
    p->tau_eps = 0.05;
    p->tau_C = 1.0;
    p->weno_eps = 1e-8;
    p->gamma_lin = 0.025;
    p->precision = HGKS_FP64;
    p->accumulation = HGKS_ACC_GATHER;
    p->reorder = 1;
    p->mu_ref = 0.0;
    p->T_ref = 1.0;
    p->mu_exp = 0.7;
    p->prandtl = 1.0;
    p->farfield[0] = 1.0;
    p->farfield[1] = p->farfield[2] = p->farfield[3] = 0.0;
    p->farfield[4] = 1.0;
}

hgks_status hgks_create(const hgks_params *params, int device, void *hip_stream, const hgks_allocator *alloc,
                        hgks_ctx **out) {
    if (!out) return HGKS_E_INVALID_ARG;
    *out = nullptr;
    if (check_params(params) != HGKS_OK) return HGKS_E_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HGKS_E_INVALID_ARG;
    if (alloc && (!alloc->alloc || !alloc->free)) return HGKS_E_INVALID_ARG;
    hgks_ctx *c = new (std::nothrow) hgks_ctx;
    if (!c) return HGKS_E_OOM;
    c->prm = *params;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (alloc) {
        c->alloc = *alloc;
        c->user_alloc = true;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return HGKS_E_DEVICE;
    }
    if (hip_stream == HGKS_OWN_STREAM) {
        c->stream = nullptr;
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return HGKS_E_DEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return HGKS_OK;
}

hgks_status hgks_mesh_upload(hgks_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_cells, int npc,
                             const int64_t *cell_nodes, const double *period, int64_t n_bfaces,
                             const int64_t *bface_nodes, const int32_t *bface_kind) {
    if (!c) return HGKS_E_INVALID_ARG;
    if (c->pool_refs) return fail(c, HGKS_E_STATE, "context is in a pool");
    if (npc == 8) return upload_hex(c, n_nodes, xyz, n_cells, cell_nodes, period, n_bfaces, bface_nodes, bface_kind);
    if (n_bfaces != 0 || bface_nodes || bface_kind)
        return fail(c, HGKS_E_INVALID_ARG, "listed boundary faces are taken on hexahedral meshes only");
    if (c->prm.tau_mode == 2)
        return fail(c, HGKS_E_INVALID_ARG, "the viscous collision time (tau_mode 2) is taken on hexahedral meshes only");
    HostMesh hm;
    std::string err;
    hgks_status st = build_mesh(c->prm, n_nodes, xyz, n_cells, npc, cell_nodes, period, hm, err);
    if (st != HGKS_OK) return fail(c, st, err);
    HIPCHK(c, hipSetDevice(c->device));
    release(c);
    const int prec = c->prm.precision;
    const bool mixed = prec != HGKS_FP64;
    const bool col = c->prm.accumulation == HGKS_ACC_COLOURED;
    // tile tables
    std::vector<Tile> ct, ft;
    const int nct = n_cell_tiles(hm.nc);
    for (int t = 0; t < nct; ++t) {
        int b = t * UPD_TILE;
        ct.push_back({0, b, t, (int32_t)std::min<int64_t>(hm.nc, b + UPD_TILE)});
    }
    xcd_order(ct, 0, ct.size());
    c->colour_tiles.clear();
    if (col) {
        for (size_t k = 0; k + 1 < hm.colour_offsets.size(); ++k) {
            c->colour_tiles.push_back((int)ft.size());
            size_t b0 = ft.size();
            for (int32_t b = hm.colour_offsets[k]; b < hm.colour_offsets[k + 1]; b += FACE_TILE)
                ft.push_back({0, b, (int)ft.size(), std::min<int32_t>(hm.colour_offsets[k + 1], b + FACE_TILE)});
            xcd_order(ft, b0, ft.size());
        }
        c->colour_tiles.push_back((int)ft.size());
    } else {
        const int fw = tau0_of(c->prm) ? FACE_TILE : 3 * GP_FACES;   // faces per tile of the flux kernel
        for (int64_t b = 0; b < hm.nf; b += fw)
            ft.push_back({0, (int32_t)b, (int)ft.size(), (int32_t)std::min<int64_t>(hm.nf, b + fw)});
        xcd_order(ft, 0, ft.size());
    }
    Layout L = layout_for(hm.nc, hm.nf, (int)ct.size(), (int)ft.size(), prec, col);
    void *mem = nullptr;
    if (c->user_alloc) {
        mem = c->alloc.alloc(L.total, c->stream, c->alloc.user);
        if (!mem) return fail(c, HGKS_E_OOM, "allocator returned NULL");
    } else {
        hipError_t e = hipMalloc(&mem, L.total);
        if (e != hipSuccess) return fail(c, HGKS_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    c->base = (char *)mem;
    c->bytes = L.total;
    char *B = c->base;
    ProbDesc &D = c->desc;
    D = ProbDesc{};
    D.nc = (int32_t)hm.nc;
    D.nf = (int32_t)hm.nf;
    D.n_cell_tiles = (int32_t)ct.size();
    D.sten = (const int32_t *)(B + L.sten);
    D.pinv0 = prec == HGKS_FP32 ? nullptr : (const double *)(B + L.pinv0);
    D.pinv32 = prec == HGKS_FP32 ? (const float *)(B + L.pinv0) : nullptr;
    D.cen = (const double *)(B + L.cen);
    D.sshift = (const uint32_t *)(B + L.sshift);
    for (int a = 0; a < 3; ++a) {
        D.per[a] = (period && period[a] > 0.0) ? period[a] : 0.0;
        D.mir[a][0] = hm.mir[a][0];
        D.mir[a][1] = hm.mir[a][1];
    }
    D.cgeo = (const double *)(B + L.cgeo);
    D.cface = (const int32_t *)(B + L.cface);
    D.fcell = (const int32_t *)(B + L.fcell);
    D.fgeo = (const double *)(B + L.fgeo);
    D.Q = (double *)(B + L.Q);
    D.Qs = (double *)(B + L.Qs);
    D.R = (double *)(B + L.R);
    D.C = mixed ? nullptr : (double *)(B + L.C);
    D.C32 = mixed ? (float *)(B + L.C32) : nullptr;
    D.FF = col ? nullptr : (double *)(B + L.FF);
    D.acc = col ? (double *)(B + L.acc) : nullptr;
    D.dtpart = (double *)(B + L.dtpart);
    D.dt = (double *)(B + L.scal);
    D.time = (double *)(B + L.scal + 8);
    D.flag = (int32_t *)(B + L.scal + 16);
    D.gamma = c->prm.gamma;
    D.K = (5.0 - 3.0 * c->prm.gamma) / (c->prm.gamma - 1.0);
    D.weno_eps = c->prm.weno_eps;
    D.gamma_lin = c->prm.gamma_lin;
    D.cfl = c->prm.cfl;
    D.tau_eps = c->prm.tau_eps;
    D.tau_C = c->prm.tau_C;
    D.tau_mode = c->prm.tau_mode;
    D.mixed = mixed ? 1 : 0;
    c->d_desc = (ProbDesc *)(B + L.desc);
    c->d_ctiles = (Tile *)(B + L.tiles);
    c->d_ftiles = c->d_ctiles + ct.size();
    c->n_ctiles = (int)ct.size();
    c->n_ftiles = (int)ft.size();
    c->h_ctiles = ct;
    c->h_ftiles = ft;
    hipStream_t s = c->stream;
    auto h2d = [&](const void *dst, const void *src, size_t n) {
        return hipMemcpyAsync((void *)dst, src, n, hipMemcpyHostToDevice, s);
    };
    HIPCHK(c, h2d(D.sten, hm.sten.data(), hm.sten.size() * 4));
    if (prec == HGKS_FP32) {
        // pair rows 2k and 2k+1 of a cell become its quad row k, each value rounded once
        hvec<float> p32(hm.pinv0.size());
        pinv0_quads_f32(hm, p32.data());
        HIPCHK(c, h2d(D.pinv32, p32.data(), p32.size() * 4));
        HIPCHK(c, hipStreamSynchronize(s));   // p32 is released on return
    } else {
        HIPCHK(c, h2d(D.pinv0, hm.pinv0.data(), hm.pinv0.size() * 8));
    }
    HIPCHK(c, h2d(D.cen, hm.cen.data(), hm.cen.size() * 8));
    HIPCHK(c, h2d(D.sshift, hm.sshift.data(), hm.sshift.size() * 4));
    const bool s32 = prec == HGKS_FP32;
    std::vector<float> cg32, fg32;            // the FP32 form's geometry, each value rounded once
    if (s32) {
        cg32.assign(hm.cgeo.begin(), hm.cgeo.end());
        fg32.assign(hm.fgeo.begin(), hm.fgeo.end());
        HIPCHK(c, h2d(D.cgeo, cg32.data(), cg32.size() * 4));
    } else {
        HIPCHK(c, h2d(D.cgeo, hm.cgeo.data(), hm.cgeo.size() * 8));
    }
    HIPCHK(c, h2d(D.cface, hm.cface.data(), hm.cface.size() * 4));
    HIPCHK(c, h2d(D.fcell, hm.fcell.data(), hm.fcell.size() * 4));
    if (s32)
        HIPCHK(c, h2d(D.fgeo, fg32.data(), fg32.size() * 4));
    else
        HIPCHK(c, h2d(D.fgeo, hm.fgeo.data(), hm.fgeo.size() * 8));
    HIPCHK(c, h2d(c->d_desc, &D, sizeof(ProbDesc)));
    HIPCHK(c, h2d(c->d_ctiles, ct.data(), ct.size() * sizeof(Tile)));
    HIPCHK(c, h2d(c->d_ftiles, ft.data(), ft.size() * sizeof(Tile)));
    if (col) launch_fill(D.acc, 0.0, (int64_t)(s32 ? 5 : 10) * hm.nc, s);   // zero bits: 0.0 in either size
    HIPCHK(c, hipStreamSynchronize(s));
    c->nc = hm.nc;
    c->nf = hm.nf;
    c->perm = std::move(hm.perm);
    c->colour_offsets = hm.colour_offsets;
    c->walls = hm.n_wall_faces > 0;
    c->hex = false;
    c->ng = 0;
    c->ns = SLOTS;
    c->has_mesh = true;
    c->has_state = false;
    return HGKS_OK;
}

hgks_status hgks_init_state(hgks_ctx *c, const double *q, double t0) {
    if (!c) return HGKS_E_INVALID_ARG;
    if (!c->has_mesh) return fail(c, HGKS_E_STATE, "init_state before mesh_upload");
    if (c->pool_refs) return fail(c, HGKS_E_STATE, "context is in a pool");
    if (!q || !std::isfinite(t0)) return fail(c, HGKS_E_INVALID_ARG, "null state");
    const int64_t nc = c->nc;
    std::vector<double> soa((size_t)5 * nc);
    for (int64_t i = 0; i < nc; ++i) {
        const double *x = q + 5 * c->perm[i];
        double rho = x[0], ke = 0.5 * (x[1] * x[1] + x[2] * x[2] + x[3] * x[3]) / rho;
        double p = (c->prm.gamma - 1.0) * (x[4] - ke);
        bool ok = std::isfinite(x[0]) && std::isfinite(x[1]) && std::isfinite(x[2]) && std::isfinite(x[3]) &&
                  std::isfinite(x[4]) && rho > 0.0 && p > 0.0;
        if (!ok) return fail(c, HGKS_E_NONPHYSICAL, "initial state has rho <= 0, p <= 0 or a non-finite value");
        for (int v = 0; v < 5; ++v) soa[(size_t)v * nc + i] = x[v];
    }
    HIPCHK(c, hipSetDevice(c->device));
    double scal[3] = {0.0, t0, 0.0};
    int32_t zero[2] = {0, 0};     // non-physical flag, flux fix-up flag
    const bool s32 = c->prm.precision == HGKS_FP32;
    std::vector<float> soa32;
    if (s32) {                    // the FP32 form's state: each value rounded once
        soa32.assign(soa.begin(), soa.end());
        HIPCHK(c, hipMemcpyAsync(c->desc.Q, soa32.data(), soa32.size() * 4, hipMemcpyHostToDevice, c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(c->desc.Q, soa.data(), soa.size() * 8, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->desc.dt, scal, 16, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->desc.flag, zero, 8, hipMemcpyHostToDevice, c->stream));
    launch_dt_local(c->d_desc, c->d_ctiles, c->n_ctiles, s32, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_state = true;
    return HGKS_OK;
}

hgks_status hgks_sync(hgks_ctx *c) {
    if (!c) return HGKS_E_INVALID_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->pool_refs) HIPCHK(c, hipStreamSynchronize(c->pool_stream));
    if (!c->has_state) return HGKS_OK;
    int32_t flag = 0;
    HIPCHK(c, hipMemcpy(&flag, c->desc.flag, 4, hipMemcpyDeviceToHost));
    if (flag) return fail(c, HGKS_E_NONPHYSICAL, "a step produced rho <= 0, p <= 0 or a non-finite value");
    return HGKS_OK;
}

hgks_status hgks_step_s2o4(hgks_ctx *c, int32_t nsteps, double dt_fixed, double *dt_last) {
    if (!c) return HGKS_E_INVALID_ARG;
    if (!c->has_state) return fail(c, HGKS_E_STATE, "step before init_state");
    if (c->pool_refs) return fail(c, HGKS_E_STATE, "context is in a pool: step it with hgks_pool_step");
    if (nsteps < 0 || !std::isfinite(dt_fixed)) return fail(c, HGKS_E_INVALID_ARG, "bad step arguments");
    HIPCHK(c, hipSetDevice(c->device));
    for (int32_t k = 0; k < nsteps; ++k) {
        enqueue_step(c, dt_fixed);
        // profiling: fold finished event pairs back into the pool so that a long
        // run keeps a bounded number of events in flight
        if (c->pending.size() > 512) collect_profile(c);
    }
    HIPCHK(c, hipGetLastError());
    if (dt_last) {
        hgks_status st = hgks_sync(c);
        HIPCHK(c, hipMemcpy(dt_last, c->desc.dt, 8, hipMemcpyDeviceToHost));
        if (st != HGKS_OK) return st;
    }
    return HGKS_OK;
}

hgks_status hgks_get_state(hgks_ctx *c, double *q_out, double *t_out) {
    if (!c) return HGKS_E_INVALID_ARG;
    if (!c->has_state) return fail(c, HGKS_E_STATE, "get_state before init_state");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->pool_refs) HIPCHK(c, hipStreamSynchronize(c->pool_stream));
    const int64_t nc = c->nc;
    if (q_out) {
        std::vector<double> soa((size_t)5 * nc);
        if (c->prm.precision == HGKS_FP32) {
            std::vector<float> soa32((size_t)5 * nc);
            HIPCHK(c, hipMemcpy(soa32.data(), c->desc.Q, soa32.size() * 4, hipMemcpyDeviceToHost));
            soa.assign(soa32.begin(), soa32.end());
        } else {
            HIPCHK(c, hipMemcpy(soa.data(), c->desc.Q, soa.size() * 8, hipMemcpyDeviceToHost));
        }
        for (int64_t i = 0; i < nc; ++i)
            for (int v = 0; v < 5; ++v) q_out[5 * c->perm[i] + v] = soa[(size_t)v * nc + i];
    }
    double tt = 0.0;
    int32_t flag = 0;
    HIPCHK(c, hipMemcpy(&tt, c->desc.time, 8, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&flag, c->desc.flag, 4, hipMemcpyDeviceToHost));
    if (t_out) *t_out = tt;
    if (flag) return fail(c, HGKS_E_NONPHYSICAL, "a step produced rho <= 0, p <= 0 or a non-finite value");
    return HGKS_OK;
}

hgks_status hgks_mesh_info(const hgks_ctx *c, int64_t *n_cells, int64_t *n_faces, int32_t *slots, int32_t *ncol) {
    if (!c) return HGKS_E_INVALID_ARG;
    if (!c->has_mesh) return HGKS_E_STATE;
    if (n_cells) *n_cells = c->nc;
    if (n_faces) *n_faces = c->nf;
    if (slots) *slots = c->ns;
    if (ncol) *ncol = (int32_t)c->colour_offsets.size() - 1;
    return HGKS_OK;
}

hgks_status hgks_footprint(const hgks_ctx *c, size_t *bytes) {
    if (!c || !bytes) return HGKS_E_INVALID_ARG;
    *bytes = c->bytes;
    return HGKS_OK;
}

hgks_status hgks_profile_enable(hgks_ctx *c, int on) {
    if (!c) return HGKS_E_INVALID_ARG;
    c->prof = on != 0;
    return HGKS_OK;
}

hgks_status hgks_profile_read(hgks_ctx *c, int id, double *ms, int64_t *n) {
    if (!c || id < 0 || id > 3) return HGKS_E_INVALID_ARG;
    collect_profile(c);
    if (ms) *ms = c->prof_ms[id];
    if (n) *n = c->prof_n[id];
    return HGKS_OK;
}

hgks_status hgks_profile_reset(hgks_ctx *c) {
    if (!c) return HGKS_E_INVALID_ARG;
    collect_profile(c);
    for (int k = 0; k < 4; ++k) {
        c->prof_ms[k] = 0;
        c->prof_n[k] = 0;
    }
    return HGKS_OK;
}

const char *hgks_last_error(const hgks_ctx *c) { return c ? c->err.c_str() : "null context"; }

void hgks_destroy(hgks_ctx *c) {
    if (!c) return;
    // A pooled context leaves its pool first (which waits for the pool's queued
    // steps), so the pool never launches on memory freed here.
    if (c->pool) pool_detach(c->pool, c);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    collect_profile(c);
    for (auto e : c->spare) (void)hipEventDestroy(e);
    release(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

hgks_status hgks_inspect_mesh(const hgks_params *params, int64_t n_nodes, const double *xyz, int64_t n_cells, int npc,
                              const int64_t *cell_nodes, const double *period, double *stats, int64_t *perm,
                              int32_t *sten) {
    hgks_params p;
    if (params) p = *params; else hgks_default_params(&p);
    if (check_params(&p) != HGKS_OK) return HGKS_E_INVALID_ARG;
    if (npc == 8) {
        HexMesh hx;
        std::string err;
        hgks_status st = build_hex_mesh(p, n_nodes, xyz, n_cells, cell_nodes, period, 0, nullptr, nullptr, hx, err, true);
        if (st != HGKS_OK) return st;
        if (stats) {
            stats[0] = (double)hx.nf;
            stats[1] = hx.ns;
            stats[2] = hx.max_members;
            stats[3] = hx.min_members;
            stats[4] = 1;
            stats[5] = hx.pinv_residual;
            stats[6] = hx.closure;
            stats[7] = 0;
        }
        if (perm) std::memcpy(perm, hx.perm.data(), hx.perm.size() * 8);
        if (sten) std::memcpy(sten, hx.sten.data(), hx.sten.size() * 4);
        return HGKS_OK;
    }
    HostMesh hm;
    std::string err;
    hgks_status st = build_mesh(p, n_nodes, xyz, n_cells, npc, cell_nodes, period, hm, err, true);
    if (st != HGKS_OK) return st;
    if (stats) {
        stats[0] = (double)hm.nf;
        stats[1] = SLOTS;
        stats[2] = hm.max_members;
        stats[3] = hm.min_members;
        stats[4] = (double)hm.colour_offsets.size() - 1;
        stats[5] = hm.pinv_residual;
        stats[6] = hm.closure;
        stats[7] = hm.dup_slots;
    }
    if (perm) std::memcpy(perm, hm.perm.data(), hm.perm.size() * 8);
    if (sten) std::memcpy(sten, hm.sten.data(), hm.sten.size() * 4);
    return HGKS_OK;
}

// ----------------------------------------------------------------------------
// pool
// ----------------------------------------------------------------------------
}  // extern "C"

struct hgks_pool {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0, used = 0;
    std::vector<hgks_ctx *> slot;
    // device tables for the current batch
    char *tab = nullptr;
    size_t tab_bytes = 0;
    std::vector<int> last_key;
    // launch plan of the current batch
    ProbDesc *d_probs = nullptr;
    int nprobs = 0;
    Tile *d_ct = nullptr, *d_ft = nullptr;
    struct Group { int prec; bool tau0; int c0, c1, f0, f1; bool walls; };
    std::vector<Group> groups;
    int n_ct = 0;
    // the allocation-free step: its plan, and the serial of its last upload into
    // the device's static table (the table holds the last uploader's plan)
    std::vector<int> static_key;
    std::vector<Group> static_groups;
    int static_nprobs = 0, static_n_ct = 0;
    uint64_t static_serial = 0;
};

namespace {

size_t footprint_of(const hgks_params &p, int64_t nc) {
    const int64_t nf = 2 * nc;
    const int nct = n_cell_tiles(nc);
    // coloured accumulation rounds every colour class up to whole tiles (at most 8 classes)
    const bool col = p.accumulation == HGKS_ACC_COLOURED;
    const int fw = (col || p.tau_mode == 0) ? FACE_TILE : 3 * GP_FACES;
    const int nft = (int)((nf + fw - 1) / fw) + (col ? 8 : 0);
    Layout L = layout_for(nc, nf, nct, nft, p.precision, p.accumulation == HGKS_ACC_COLOURED);
    return L.total;
}

// The launch tables of a batch, built on the host: problem descriptors, cell and
// face tiles grouped by kernel variant (FP64 first, then FP32-mixed, then FP32).
struct Plan {
    std::vector<ProbDesc> probs;
    std::vector<Tile> ct, ft;
    std::vector<hgks_pool::Group> groups;
    size_t bytes() const {
        return up(probs.size() * sizeof(ProbDesc)) + up(ct.size() * sizeof(Tile)) + up(ft.size() * sizeof(Tile));
    }
};

Plan make_plan(const hgks_pool *P, const std::vector<int> &key) {
    Plan pl;
    std::vector<int> order(key);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        auto ka = std::make_pair(P->slot[a]->prm.precision, P->slot[a]->prm.tau_mode);
        auto kb = std::make_pair(P->slot[b]->prm.precision, P->slot[b]->prm.tau_mode);
        return ka < kb;
    });
    for (size_t k = 0; k < order.size(); ++k) {
        hgks_ctx *c = P->slot[order[k]];
        const int prec = c->prm.precision;
        const bool tau0 = c->prm.tau_mode == 0;
        if (pl.groups.empty() || pl.groups.back().prec != prec || pl.groups.back().tau0 != tau0)
            pl.groups.push_back({prec, tau0, (int)pl.ct.size(), (int)pl.ct.size(), (int)pl.ft.size(),
                                 (int)pl.ft.size(), false});
        pl.groups.back().walls = pl.groups.back().walls || c->walls;
        const int pid = (int)pl.probs.size();
        pl.probs.push_back(c->desc);
        for (Tile t : c->h_ctiles) { t.prob = pid; pl.ct.push_back(t); }
        for (Tile t : c->h_ftiles) { t.prob = pid; pl.ft.push_back(t); }
        pl.groups.back().c1 = (int)pl.ct.size();
        pl.groups.back().f1 = (int)pl.ft.size();
    }
    for (auto &g : pl.groups) {
        xcd_order(pl.ct, g.c0, g.c1);
        xcd_order(pl.ft, g.f0, g.f1);
    }
    return pl;
}

// Copies a plan's tables to device memory at `dev` (synchronous; the caller has
// made sure that no queued launch still reads that memory).
hgks_status upload_plan(const Plan &pl, char *dev, ProbDesc **probs, Tile **ct, Tile **ft) {
    *probs = (ProbDesc *)dev;
    *ct = (Tile *)(dev + up(pl.probs.size() * sizeof(ProbDesc)));
    *ft = (Tile *)((char *)*ct + up(pl.ct.size() * sizeof(Tile)));
    if (hipMemcpy(*probs, pl.probs.data(), pl.probs.size() * sizeof(ProbDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(*ct, pl.ct.data(), pl.ct.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(*ft, pl.ft.data(), pl.ft.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess)
        return HGKS_E_DEVICE;
    return HGKS_OK;
}

hgks_status pool_plan(hgks_pool *P, const int *slots, int n) {
    std::vector<int> key(slots, slots + n);
    if (key == P->last_key && P->tab) return HGKS_OK;
    Plan pl = make_plan(P, key);
    const size_t need = pl.bytes();
    if (need > P->tab_bytes) {
        if (P->tab) {
            (void)hipStreamSynchronize(P->stream);
            (void)hipFree(P->tab);
        }
        P->tab = nullptr;
        if (hipMalloc((void **)&P->tab, need * 2) != hipSuccess) return HGKS_E_OOM;
        P->tab_bytes = need * 2;
    }
    (void)hipStreamSynchronize(P->stream);
    hgks_status st = upload_plan(pl, P->tab, &P->d_probs, &P->d_ct, &P->d_ft);
    if (st != HGKS_OK) return st;
    P->groups = pl.groups;
    P->nprobs = (int)pl.probs.size();
    P->n_ct = (int)pl.ct.size();
    P->last_key = key;
    return HGKS_OK;
}

// Serial of the plan each device's static table holds (0: none), and the counter
// that hands out serials.
std::mutex g_static_mu;
std::vector<uint64_t> g_static_serial;
uint64_t g_static_next = 0;

void enqueue_pool_steps(const ProbDesc *probs, int nprobs, const Tile *ct, int n_ct, const Tile *ft,
                        const std::vector<hgks_pool::Group> &groups, int32_t nsteps, hipStream_t s) {
    for (int32_t it = 0; it < nsteps; ++it) {
        launch_dt_final(probs, nprobs, 0.0, s);
        for (int stage = 1; stage <= 2; ++stage) {
            for (auto &g : groups) launch_weno(probs, ct + g.c0, g.c1 - g.c0, stage, g.prec, g.walls, s);
            for (auto &g : groups)
                launch_flux(probs, nprobs, ft + g.f0, g.f1 - g.f0, stage, g.prec, g.tau0, false, g.walls, s);
            // groups run FP64, FP32-mixed, FP32: the FP32 form's cells (FP32 storage) are
            // the last tiles, updated by their own launch
            int c32 = n_ct;
            for (auto &g : groups)
                if (g.prec == HGKS_FP32) c32 = std::min(c32, g.c0);
            launch_update(probs, ct, c32, stage, false, false, s);
            launch_update(probs, ct + c32, n_ct - c32, stage, false, true, s);
        }
    }
}

hgks_status check_slots(const hgks_pool *p, const int *slots, int n) {
    for (int k = 0; k < n; ++k) {
        if (slots[k] < 0 || slots[k] >= (int)p->slot.size() || !p->slot[slots[k]]) return HGKS_E_INVALID_ARG;
        for (int j = 0; j < k; ++j)
            if (slots[j] == slots[k]) return HGKS_E_INVALID_ARG;
    }
    return HGKS_OK;
}

}  // namespace

// Removes context c from pool p after the pool's queued work is done.
void pool_detach(hgks_pool *p, hgks_ctx *c) {
    (void)hipSetDevice(p->device);
    (void)hipStreamSynchronize(p->stream);
    for (auto &x : p->slot)
        if (x == c) {
            x = nullptr;
            p->used -= c->bytes;
        }
    c->pool_refs = 0;
    c->pool = nullptr;
    c->pool_stream = nullptr;
    p->last_key.clear();
    p->static_key.clear();
}

extern "C" {

hgks_status hgks_pool_create(int device, void *hip_stream, size_t hbm_budget, hgks_pool **out) {
    if (!out) return HGKS_E_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HGKS_E_INVALID_ARG;
    hgks_pool *p = new (std::nothrow) hgks_pool;
    if (!p) return HGKS_E_OOM;
    p->device = device;
    p->stream = (hipStream_t)hip_stream;
    p->budget = hbm_budget;
    if (hip_stream == HGKS_OWN_STREAM) {
        p->stream = nullptr;
        if (hipSetDevice(device) != hipSuccess ||
            hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return HGKS_E_DEVICE;
        }
        p->own_stream = true;
    }
    *out = p;
    return HGKS_OK;
}

hgks_status hgks_pool_footprint(const hgks_params *params, int64_t n_cells, int npc, size_t *bytes) {
    if (!params || !bytes || n_cells <= 0 || npc != 4) return HGKS_E_INVALID_ARG;
    if (check_params(params) != HGKS_OK) return HGKS_E_INVALID_ARG;
    *bytes = footprint_of(*params, n_cells);
    return HGKS_OK;
}

hgks_status hgks_pool_add(hgks_pool *p, hgks_ctx *c, int *slot) {
    if (!p || !c || !slot) return HGKS_E_INVALID_ARG;
    if (!c->has_state) return HGKS_E_STATE;
    if (c->device != p->device || c->prm.accumulation != HGKS_ACC_GATHER || c->hex) return HGKS_E_INVALID_ARG;
    if (p->budget && p->used + c->bytes > p->budget) return HGKS_E_OOM;
    if (c->pool) return HGKS_E_INVALID_ARG;     // a context belongs to one pool at a time
    // the pool runs on its own stream: finish the context's queued work first
    (void)hipSetDevice(p->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return HGKS_E_DEVICE;
    int s = -1;
    for (size_t k = 0; k < p->slot.size(); ++k)
        if (!p->slot[k]) { s = (int)k; break; }
    if (s < 0) { s = (int)p->slot.size(); p->slot.push_back(nullptr); }
    p->slot[s] = c;
    p->used += c->bytes;
    c->pool_refs++;
    c->pool = p;
    c->pool_stream = p->stream;
    p->last_key.clear();
    p->static_key.clear();
    *slot = s;
    return HGKS_OK;
}

hgks_status hgks_pool_step(hgks_pool *p, const int *slots, int n, int32_t nsteps) {
    if (!p || (n > 0 && !slots) || n < 0 || nsteps < 0) return HGKS_E_INVALID_ARG;
    if (n == 0 || nsteps == 0) return HGKS_OK;
    if (check_slots(p, slots, n) != HGKS_OK) return HGKS_E_INVALID_ARG;
    if (hipSetDevice(p->device) != hipSuccess) return HGKS_E_DEVICE;
    hgks_status st = pool_plan(p, slots, n);
    if (st != HGKS_OK) return st;
    enqueue_pool_steps(p->d_probs, p->nprobs, p->d_ct, p->n_ct, p->d_ft, p->groups, nsteps, p->stream);
    if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
    return HGKS_OK;
}

hgks_status hgks_pool_step_static(hgks_pool *p, const int *slots, int n, int32_t nsteps) {
    if (!p || (n > 0 && !slots) || n < 0 || nsteps < 0) return HGKS_E_INVALID_ARG;
    if (n == 0 || nsteps == 0) return HGKS_OK;
    if (check_slots(p, slots, n) != HGKS_OK) return HGKS_E_INVALID_ARG;
    if (hipSetDevice(p->device) != hipSuccess) return HGKS_E_DEVICE;
    void *table = nullptr;
    if (static_table_ptr(p->device, &table) != hipSuccess) return HGKS_E_DEVICE;
    std::vector<int> key(slots, slots + n);
    std::lock_guard<std::mutex> g(g_static_mu);
    if (g_static_serial.size() <= (size_t)p->device) g_static_serial.resize((size_t)p->device + 1, 0);
    ProbDesc *probs = nullptr;
    Tile *ct = nullptr, *ft = nullptr;
    if (key != p->static_key || g_static_serial[(size_t)p->device] != p->static_serial) {
        Plan pl = make_plan(p, key);
        if (pl.bytes() > STATIC_TABLE_BYTES) {
            const std::string m = "allocation-free pool step: the launch tables need " + std::to_string(pl.bytes()) +
                                  " bytes, beyond the static table of " + std::to_string(STATIC_TABLE_BYTES);
            for (int k = 0; k < n; ++k) p->slot[slots[k]]->err = m;
            return HGKS_E_INVALID_ARG;
        }
        // the table may still feed queued steps: this pool's, or another pool's when
        // that one uploaded last (then the whole device is waited for)
        const bool other = g_static_serial[(size_t)p->device] != 0 &&
                           g_static_serial[(size_t)p->device] != p->static_serial;
        if ((other ? hipDeviceSynchronize() : hipStreamSynchronize(p->stream)) != hipSuccess) return HGKS_E_DEVICE;
        hgks_status st = upload_plan(pl, (char *)table, &probs, &ct, &ft);
        if (st != HGKS_OK) return st;
        p->static_key = key;
        p->static_groups = pl.groups;
        p->static_nprobs = (int)pl.probs.size();
        p->static_n_ct = (int)pl.ct.size();
        p->static_serial = ++g_static_next;
        g_static_serial[(size_t)p->device] = p->static_serial;
    } else {
        // the table still holds this pool's plan for these slots
        probs = (ProbDesc *)table;
        ct = (Tile *)((char *)table + up((size_t)p->static_nprobs * sizeof(ProbDesc)));
        ft = (Tile *)((char *)ct + up((size_t)p->static_n_ct * sizeof(Tile)));
    }
    enqueue_pool_steps(probs, p->static_nprobs, ct, p->static_n_ct, ft, p->static_groups, nsteps, p->stream);
    if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
    return HGKS_OK;
}

hgks_status hgks_pool_remove(hgks_pool *p, int slot) {
    if (!p || slot < 0 || slot >= (int)p->slot.size() || !p->slot[slot]) return HGKS_E_INVALID_ARG;
    pool_detach(p, p->slot[slot]);
    return HGKS_OK;
}

hgks_status hgks_pool_used(const hgks_pool *p, size_t *bytes, int *n_slots) {
    if (!p) return HGKS_E_INVALID_ARG;
    if (bytes) *bytes = p->used;
    if (n_slots) {
        int k = 0;
        for (auto *x : p->slot) k += x != nullptr;
        *n_slots = k;
    }
    return HGKS_OK;
}

void hgks_pool_destroy(hgks_pool *p) {
    if (!p) return;
    for (auto *c : p->slot)
        if (c) pool_detach(p, c);
    (void)hipSetDevice(p->device);
    (void)hipStreamSynchronize(p->stream);
    if (p->tab) (void)hipFree(p->tab);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

}  // extern "C"
