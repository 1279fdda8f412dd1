// Host precompute of hexahedral meshes (Sec. 3.1 connectivity, Algorithm 1
// stencils, Sec. 2.3 hexahedral sub-stencils): cell geometry by Gauss quadrature
// of the trilinear map, bilinear faces with 2x2 Gauss points (each with its own
// normal and weight), ghosts of listed boundary faces, the big-stencil
// pseudo-inverses and the inverses of the eight exactly determined linear
// sub-stencil fits, all laid out for the device.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hgks_internal.h"

namespace hgks {

namespace {

struct P3 {
    double v[3];
    double &operator[](int a) { return v[a]; }
    double operator[](int a) const { return v[a]; }
};
inline P3 sub(const P3 &a, const P3 &b) { return {{a[0] - b[0], a[1] - b[1], a[2] - b[2]}}; }
inline P3 add(const P3 &a, const P3 &b) { return {{a[0] + b[0], a[1] + b[1], a[2] + b[2]}}; }
inline P3 scale(double s, const P3 &a) { return {{s * a[0], s * a[1], s * a[2]}}; }
inline double dot(const P3 &a, const P3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline P3 cross(const P3 &a, const P3 &b) {
    return {{a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]}};
}

// reference corner of node k on [0,1]^3
constexpr int CORNER[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
constexpr int FACE[6][4] = {{0, 1, 2, 3}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}};
// symmetric pairs (xx, yy, zz, xy, xz, yz)
constexpr int PA[6] = {0, 1, 2, 0, 0, 1};
constexpr int PB[6] = {0, 1, 2, 1, 2, 2};

// Gauss-Legendre on [0, 1]: three points (cells) and two points (faces)
const double G3X[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
const double G3W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
const double G2X[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};

struct CellGeo {
    double vol;
    P3 cen;
    double m2[6];      // central second moments: mean of (x-c)_a (x-c)_b
    bool ok;
};

// Volume, centroid and central second moments by the 3x3x3 product rule over the
// trilinear map x(r) = sum_k N_k(r) x_k (exact: the integrands are polynomials of
// degree <= 4 per reference direction).  ok = false when the map folds (Jacobians
// of both signs) or degenerates.
CellGeo cell_geometry(const P3 v[8]) {
    CellGeo g{};
    double jmin = HUGE_VAL, jmax = -HUGE_VAL;
    double s0 = 0.0, s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
    P3 pts[27];
    double wts[27];
    int n = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c, ++n) {
                const double r[3] = {G3X[a], G3X[b], G3X[c]};
                P3 x{{0, 0, 0}}, d[3] = {{{0, 0, 0}}, {{0, 0, 0}}, {{0, 0, 0}}};
                for (int k = 0; k < 8; ++k) {
                    double f[3], df[3];
                    for (int e = 0; e < 3; ++e) {
                        f[e] = CORNER[k][e] ? r[e] : 1.0 - r[e];
                        df[e] = CORNER[k][e] ? 1.0 : -1.0;
                    }
                    const double N = f[0] * f[1] * f[2];
                    const double dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
                    for (int e = 0; e < 3; ++e) {
                        x[e] += N * v[k][e];
                        for (int q = 0; q < 3; ++q) d[q][e] += dN[q] * v[k][e];
                    }
                }
                const double J = dot(d[0], cross(d[1], d[2]));
                jmin = std::min(jmin, J);
                jmax = std::max(jmax, J);
                pts[n] = x;
                wts[n] = G3W[a] * G3W[b] * G3W[c] * std::fabs(J);
            }
    double ext = 0.0;
    for (int k = 1; k < 8; ++k)
        for (int e = 0; e < 3; ++e) ext = std::max(ext, std::fabs(v[k][e] - v[0][e]));
    g.ok = jmin * jmax > 0.0 && std::min(std::fabs(jmin), std::fabs(jmax)) > 1e-12 * ext * ext * ext;
    for (int q = 0; q < 27; ++q) {
        s0 += wts[q];
        for (int e = 0; e < 3; ++e) s1[e] += wts[q] * pts[q][e];
    }
    g.vol = s0;
    for (int e = 0; e < 3; ++e) g.cen[e] = s1[e] / s0;
    for (int q = 0; q < 27; ++q) {
        const P3 y = sub(pts[q], g.cen);
        for (int m = 0; m < 6; ++m) s2[m] += wts[q] * y[PA[m]] * y[PB[m]];
    }
    for (int m = 0; m < 6; ++m) g.m2[m] = s2[m] / s0;
    return g;
}

// 2x2 Gauss points of the bilinear patch through corners c[0..3] (cyclic):
// positions, unit normals (x_s x x_t) and weights |x_s x x_t| / 4.
void face_points(const P3 c[4], P3 x[4], P3 n[4], double w[4]) {
    int g = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j, ++g) {
            const double s = G2X[i], t = G2X[j];
            P3 xs, xt;
            for (int e = 0; e < 3; ++e) {
                x[g][e] = (1 - s) * (1 - t) * c[0][e] + s * (1 - t) * c[1][e] + s * t * c[2][e] + (1 - s) * t * c[3][e];
                xs[e] = (1 - t) * (c[1][e] - c[0][e]) + t * (c[2][e] - c[3][e]);
                xt[e] = (1 - s) * (c[3][e] - c[0][e]) + s * (c[2][e] - c[1][e]);
            }
            const P3 cr = cross(xs, xt);
            const double len = std::sqrt(dot(cr, cr));
            n[g] = scale(1.0 / len, cr);
            w[g] = 0.25 * len;
        }
}

uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
    v &= 0x1FFFFF;
    v = (v | v << 32) & 0x1F00000000FFFFull;
    v = (v | v << 16) & 0x1F0000FF0000FFull;
    v = (v | v << 8) & 0x100F00F00F00F00Full;
    v = (v | v << 4) & 0x10C30C30C30C30C3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// 3x3 inverse through the adjugate; false when singular against the entries' scale
bool inv3(const double A[3][3], double X[3][3]) {
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1], c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2],
                 c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    double sc = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) sc = std::max(sc, std::fabs(A[i][j]));
    if (!(std::fabs(det) > 1e-10 * sc * sc * sc)) return false;
    const double id = 1.0 / det;
    X[0][0] = c00 * id;
    X[1][0] = c01 * id;
    X[2][0] = c02 * id;
    X[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    X[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    X[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    X[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    X[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    X[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return true;
}

// A stencil member: a cell with an integer periodic image shift, or a ghost
// (cell = nc + ghost id, no shift).
struct Mem {
    int32_t id;
    int8_t s[3];
    bool operator==(const Mem &o) const { return id == o.id && s[0] == o.s[0] && s[1] == o.s[1] && s[2] == o.s[2]; }
};

}  // namespace

hgks_status build_hex_mesh(const hgks_params &prm, int64_t nn, const double *xyz, int64_t nc, const int64_t *cn,
                           const double *period_in, int64_t nbf, const int64_t *bfn, const int32_t *bkind,
                           HexMesh &out, std::string &err, bool diagnostics) {
    if (nn <= 0 || nc <= 0 || !xyz || !cn) {
        err = "empty mesh";
        return HGKS_E_INVALID_ARG;
    }
    if (nc >= (int64_t)1 << 29) {
        err = "too many cells";
        return HGKS_E_INVALID_ARG;
    }
    double per[3];
    bool any_per = false;
    for (int a = 0; a < 3; ++a) {
        per[a] = period_in ? period_in[a] : 0.0;
        if (!(per[a] >= 0.0) || !std::isfinite(per[a])) {
            err = "bad period";
            return HGKS_E_INVALID_ARG;
        }
        any_per = any_per || per[a] > 0.0;
    }
    if (nbf < 0 || (nbf > 0 && (!bfn || !bkind))) {
        err = "boundary faces without nodes or kinds";
        return HGKS_E_INVALID_ARG;
    }
    if (nbf > 0 && any_per) {
        err = "listed boundary faces need a mesh without periodic axes";
        return HGKS_E_INVALID_ARG;
    }
    for (int64_t k = 0; k < nbf; ++k)
        if (bkind[k] != HGKS_BC_WALL && bkind[k] != HGKS_BC_FAR) {
            err = "unknown boundary kind";
            return HGKS_E_INVALID_ARG;
        }
    for (int64_t k = 0; k < nc * 8; ++k)
        if (cn[k] < 0 || cn[k] >= nn) {
            err = "node id out of range";
            return HGKS_E_INVALID_ARG;
        }
    for (int64_t k = 0; k < nbf * 4; ++k)
        if (bfn[k] < 0 || bfn[k] >= nn) {
            err = "boundary-face node id out of range";
            return HGKS_E_INVALID_ARG;
        }

    // ---- 1. unwrapped vertices and cell geometry -------------------------------
    std::vector<std::array<P3, 8>> vert(nc);
    std::vector<CellGeo> geo(nc);
    std::atomic<int> bad{0};
    parallel_range(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            const double *x0 = xyz + 3 * cn[8 * c];
            for (int q = 0; q < 8; ++q) {
                const double *xq = xyz + 3 * cn[8 * c + q];
                for (int a = 0; a < 3; ++a) {
                    double d = xq[a] - x0[a];
                    if (per[a] > 0) d -= per[a] * std::nearbyint(d / per[a]);
                    vert[c][q][a] = x0[a] + d;
                }
            }
            geo[c] = cell_geometry(vert[c].data());
            if (!geo[c].ok) bad = 1;
        }
    });
    if (bad) {
        err = "degenerate or folded hexahedron";
        return HGKS_E_BAD_MESH;
    }

    // ---- 2. faces: sort every cell face by its node set ------------------------
    using Key = std::array<int64_t, 4>;
    auto face_key = [&](int64_t c, int p) {
        Key k;
        for (int q = 0; q < 4; ++q) k[q] = cn[8 * c + FACE[p][q]];
        std::sort(k.begin(), k.end());
        return k;
    };
    std::vector<std::pair<Key, int64_t>> recs((size_t)nc * 6);
    parallel_range(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c)
            for (int p = 0; p < 6; ++p) recs[c * 6 + p] = {face_key(c, p), c * 6 + p};
    });
    std::sort(recs.begin(), recs.end());
    std::vector<std::pair<Key, int32_t>> blist((size_t)nbf);
    for (int64_t k = 0; k < nbf; ++k) {
        Key key;
        for (int q = 0; q < 4; ++q) key[q] = bfn[4 * k + q];
        std::sort(key.begin(), key.end());
        blist[k] = {key, bkind[k]};
    }
    std::sort(blist.begin(), blist.end());
    std::vector<char> bused((size_t)nbf, 0);
    std::vector<int64_t> partner((size_t)nc * 6, -1);   // (c*6+p) -> (c'*6+p'), or -1 - kind
    for (size_t s = 0; s < recs.size();) {
        size_t t = s + 1;
        while (t < recs.size() && recs[t].first == recs[s].first) ++t;
        if (t - s == 2) {
            partner[recs[s].second] = recs[s + 1].second;
            partner[recs[s + 1].second] = recs[s].second;
        } else if (t - s == 1) {
            auto it = std::lower_bound(blist.begin(), blist.end(), std::make_pair(recs[s].first, (int32_t)-1));
            if (it == blist.end() || it->first != recs[s].first) {
                err = "a face of one cell is not in the boundary-face list (hexahedral meshes need every "
                      "unshared face listed)";
                return HGKS_E_BAD_MESH;
            }
            bused[it - blist.begin()] = 1;
            partner[recs[s].second] = -1 - it->second;
        } else {
            err = "non-conforming face";
            return HGKS_E_BAD_MESH;
        }
        s = t;
    }
    for (int64_t k = 0; k < nbf; ++k)
        if (!bused[k]) {
            err = "a listed boundary face is not a face of exactly one cell";
            return HGKS_E_BAD_MESH;
        }

    // ---- 3. renumbering (Morton order of the centroids) ------------------------
    std::vector<int64_t> perm(nc);
    for (int64_t c = 0; c < nc; ++c) perm[c] = c;
    if (prm.reorder) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        auto wrapped = [&](int64_t c, int a) {
            double x = geo[c].cen[a];
            if (per[a] > 0) x -= per[a] * std::floor(x / per[a]);
            return x;
        };
        for (int64_t c = 0; c < nc; ++c)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], wrapped(c, a));
                hi[a] = std::max(hi[a], wrapped(c, a));
            }
        std::vector<std::pair<uint64_t, int64_t>> key(nc);
        parallel_range(nc, [&](int64_t b, int64_t e) {
            for (int64_t c = b; c < e; ++c) {
                uint64_t code = 0;
                for (int a = 0; a < 3; ++a) {
                    const double t = hi[a] > lo[a] ? (wrapped(c, a) - lo[a]) / (hi[a] - lo[a]) : 0.0;
                    code |= spread3((uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0))) << a;
                }
                key[c] = {code, c};
            }
        });
        std::sort(key.begin(), key.end());
        for (int64_t c = 0; c < nc; ++c) perm[c] = key[c].second;
    }
    std::vector<int32_t> inv(nc);
    for (int64_t c = 0; c < nc; ++c) inv[perm[c]] = (int32_t)c;

    // ---- 4. face list in internal order: a face belongs to its lower internal cell
    // (the left one); ghosts numbered in face order ------------------------------
    std::vector<std::array<int32_t, 6>> cface(nc);
    std::vector<std::array<int32_t, 2>> fcell;
    std::vector<int32_t> fside;     // left cell's local face
    fcell.reserve((size_t)nc * 3 + nbf);
    fside.reserve((size_t)nc * 3 + nbf);
    for (int64_t ci = 0; ci < nc; ++ci) {
        const int64_t c = perm[ci];
        for (int p = 0; p < 6; ++p) {
            const int64_t o = partner[c * 6 + p];
            if (o >= 0 && inv[o / 6] < ci) continue;   // the other cell owns it
            const int32_t f = (int32_t)fcell.size();
            fcell.push_back({(int32_t)ci, o >= 0 ? (int32_t)inv[o / 6] : (int32_t)(-(-1 - o))});
            fside.push_back(p);
            cface[ci][p] = f << 1;
            if (o >= 0) cface[inv[o / 6]][o % 6] = (f << 1) | 1;
        }
    }
    const int64_t nf = (int64_t)fcell.size();
    {   // within each block of 64 faces (a flux workgroup's tile), order by the right
        // cell (listed faces first): the update's gathers of the faces a cell sees as
        // the right cell then come in cell order
        std::vector<int32_t> order(nf), newid(nf);
        for (int64_t f = 0; f < nf; ++f) order[f] = (int32_t)f;
        for (int64_t b = 0; b < nf; b += 64)
            std::stable_sort(order.begin() + b, order.begin() + std::min<int64_t>(nf, b + 64),
                             [&](int32_t x, int32_t y) { return fcell[x][1] < fcell[y][1]; });
        std::vector<std::array<int32_t, 2>> fc2(nf);
        std::vector<int32_t> fs2(nf);
        for (int64_t k = 0; k < nf; ++k) {
            newid[order[k]] = (int32_t)k;
            fc2[k] = fcell[order[k]];
            fs2[k] = fside[order[k]];
        }
        fcell.swap(fc2);
        fside.swap(fs2);
        for (int64_t ci = 0; ci < nc; ++ci)
            for (int p = 0; p < 6; ++p) {
                const int32_t code = cface[ci][p];
                cface[ci][p] = (newid[code >> 1] << 1) | (code & 1);
            }
    }

    // neighbours (internal ids; ghosts nc + g) with image shifts
    std::vector<std::array<Mem, 6>> nb(nc);
    std::vector<int32_t> gcell, gkind, gface;
    std::vector<int32_t> fghost(nf, -1);
    for (int64_t f = 0; f < nf; ++f)
        if (fcell[f][1] < 0) {
            fghost[f] = (int32_t)gcell.size();
            gcell.push_back(fcell[f][0]);
            gkind.push_back(-fcell[f][1]);
            gface.push_back((int32_t)f);
        }
    const int64_t ng = (int64_t)gcell.size();

    // ---- 5. face geometry (left cell's frame) and neighbour shifts --------------
    out.fgeo.resize((size_t)HEX_FGEO * nf);
    std::vector<double> asum(nc, 0.0);
    std::vector<P3> gpt(ng), gn(ng);
    std::vector<std::array<int8_t, 3>> fsh(nf);     // right cell's image shift in the left frame
    double closure = 0.0;
    std::mutex mu;
    parallel_range(nf, [&](int64_t b, int64_t e) {
        for (int64_t f = b; f < e; ++f) {
            const int32_t li = fcell[f][0];
            const int64_t l = perm[li];
            const int p = fside[f];
            P3 corners[4], x[4], n[4];
            double w[4];
            for (int q = 0; q < 4; ++q) corners[q] = vert[l][FACE[p][q]];
            face_points(corners, x, n, w);
            P3 va{{0, 0, 0}}, fc{{0, 0, 0}};
            for (int g = 0; g < 4; ++g) {
                va = add(va, scale(w[g], n[g]));
                fc = add(fc, scale(0.25, x[g]));
            }
            const double sg = dot(va, sub(fc, geo[l].cen)) < 0.0 ? -1.0 : 1.0;
            const double vlen = std::sqrt(dot(va, va));
            double *F = out.fgeo.data();
            auto put = [&](int v, double val) { F[(size_t)v * nf + f] = val; };
            for (int g = 0; g < 4; ++g) {
                for (int a = 0; a < 3; ++a) put(7 * g + a, sg * n[g][a]);
                put(7 * g + 3, w[g]);
                for (int a = 0; a < 3; ++a) put(7 * g + 4 + a, x[g][a] - geo[l].cen[a]);
            }
            for (int a = 0; a < 3; ++a) put(31 + a, sg * va[a] / vlen);
            const int32_t ri = fcell[f][1];
            if (ri >= 0) {
                // image shift of the right cell: a shared node's positions in both frames
                const int64_t r = perm[ri];
                const int64_t node = cn[8 * l + FACE[p][0]];
                int qr = 0;
                while (cn[8 * r + qr] != node) ++qr;
                const P3 d = sub(corners[0], vert[r][qr]);
                for (int a = 0; a < 3; ++a) {
                    const double k = per[a] > 0 ? std::nearbyint(d[a] / per[a]) : 0.0;
                    fsh[f][a] = (int8_t)k;
                    put(28 + a, geo[l].cen[a] - (geo[r].cen[a] + k * per[a]));
                }
            } else {
                for (int a = 0; a < 3; ++a) {
                    fsh[f][a] = 0;
                    put(28 + a, 0.0);
                }
                const int32_t g = fghost[f];
                gpt[g] = fc;
                gn[g] = scale(sg / vlen, va);
            }
        }
    });
    for (int64_t f = 0; f < nf; ++f) {
        double w = 0.0;
        for (int g = 0; g < 4; ++g) w += out.fgeo[(size_t)(7 * g + 3) * nf + f];
        asum[perm[fcell[f][0]]] += w;
        if (fcell[f][1] >= 0) asum[perm[fcell[f][1]]] += w;
    }
    for (int64_t ci = 0; ci < nc; ++ci)
        for (int p = 0; p < 6; ++p) {
            const int32_t code = cface[ci][p], f = code >> 1;
            const bool right = code & 1;
            Mem m;
            if (right) {
                m.id = fcell[f][0];
                for (int a = 0; a < 3; ++a) m.s[a] = (int8_t)-fsh[f][a];
            } else if (fcell[f][1] >= 0) {
                m.id = fcell[f][1];
                for (int a = 0; a < 3; ++a) m.s[a] = fsh[f][a];
            } else {
                m.id = (int32_t)(nc + fghost[f]);
                m.s[0] = m.s[1] = m.s[2] = 0;
            }
            nb[ci][p] = m;
        }
    if (diagnostics) {
        // closure: sum over a cell's faces of the outward weighted normals
        std::vector<P3> acc(nc, P3{{0, 0, 0}});
        for (int64_t f = 0; f < nf; ++f) {
            P3 va{{0, 0, 0}};
            for (int g = 0; g < 4; ++g)
                for (int a = 0; a < 3; ++a)
                    va[a] += out.fgeo[(size_t)(7 * g + 3) * nf + f] * out.fgeo[(size_t)(7 * g + a) * nf + f];
            acc[fcell[f][0]] = add(acc[fcell[f][0]], va);
            if (fcell[f][1] >= 0) acc[fcell[f][1]] = sub(acc[fcell[f][1]], va);
        }
        for (int64_t c = 0; c < nc; ++c)
            for (int a = 0; a < 3; ++a) closure = std::max(closure, std::fabs(acc[c][a]));
    }

    // ---- 6. stencils (Algorithm 1) and their fits, internal order ---------------
    // member geometry in cell i's frame: centroid and central second moments
    auto member_geo = [&](const Mem &m, P3 &c, double m2[6]) {
        if (m.id < nc) {
            const CellGeo &G = geo[perm[m.id]];
            for (int a = 0; a < 3; ++a) c[a] = G.cen[a] + m.s[a] * per[a];
            for (int q = 0; q < 6; ++q) m2[q] = G.m2[q];
            return;
        }
        // the ghost: the cell's mirror image in its face plane, x -> x - 2 ((x - p).n) n
        const int32_t g = m.id - (int32_t)nc;
        const CellGeo &G = geo[perm[gcell[g]]];
        const P3 &n = gn[g];
        const double d = dot(sub(G.cen, gpt[g]), n);
        c = sub(G.cen, scale(2.0 * d, n));
        double R[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b2 = 0; b2 < 3; ++b2) R[a][b2] = (a == b2 ? 1.0 : 0.0) - 2.0 * n[a] * n[b2];
        double S[3][3];
        for (int q = 0; q < 6; ++q) S[PA[q]][PB[q]] = S[PB[q]][PA[q]] = G.m2[q];
        for (int q = 0; q < 6; ++q) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b2 = 0; b2 < 3; ++b2) s += R[PA[q]][a] * S[a][b2] * R[PB[q]][b2];
            m2[q] = s;
        }
    };
    std::vector<std::vector<Mem>> sten(nc);
    std::atomic<int> smax{0}, smin{1 << 30};
    parallel_range(nc, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            std::vector<Mem> &S = sten[i];
            S.clear();
            const Mem self{(int32_t)i, {0, 0, 0}};
            for (int p = 0; p < 6; ++p) {
                if (nb[i][p] == self || std::find(S.begin(), S.end(), nb[i][p]) != S.end()) bad = 2;
                S.push_back(nb[i][p]);
            }
            for (int p = 0; p < 6; ++p) {
                const Mem j = nb[i][p];
                if (j.id >= nc) continue;                      // a ghost has no neighbours
                for (int q = 0; q < 6; ++q) {
                    Mem x = nb[j.id][q];
                    if (x.id < nc)
                        for (int a = 0; a < 3; ++a) x.s[a] = (int8_t)(x.s[a] + j.s[a]);
                    if (x == self || std::find(S.begin(), S.end(), x) != S.end()) continue;
                    S.push_back(x);
                }
            }
            int cur = smax.load();
            while ((int)S.size() > cur && !smax.compare_exchange_weak(cur, (int)S.size())) {}
            cur = smin.load();
            while ((int)S.size() < cur && !smin.compare_exchange_weak(cur, (int)S.size())) {}
        }
    });
    if (bad == 2) {
        err = "a hexahedron's six face neighbours must be distinct cells (a periodic axis needs at least "
              "five cells)";
        return HGKS_E_BAD_MESH;
    }
    if (smax.load() > HEX_SLOTS) {
        err = "a hexahedral stencil has more than " + std::to_string(HEX_SLOTS) +
              " members (an edge shared by more than four cells)";
        return HGKS_E_BAD_MESH;
    }
    const int ns = HEX_SLOTS;
    out.sten.resize((size_t)ns * nc);
    out.pinv.resize((size_t)9 * ns * nc);
    out.binv.resize((size_t)HEX_BINV * nc);
    out.cgeo.resize((size_t)CGEO * nc);
    double resid_max = 0.0;
    parallel_range(nc, [&](int64_t b, int64_t e) {
        double lres = 0.0;
        std::vector<double> A, Pm;
        for (int64_t i = b; i < e; ++i) {
            const CellGeo &Gi = geo[perm[i]];
            const double h = std::cbrt(Gi.vol), ih = 1.0 / h;
            const std::vector<Mem> &S = sten[i];
            const int K = (int)S.size();
            A.assign((size_t)K * 9, 0.0);
            Pm.assign((size_t)K * 9, 0.0);
            for (int k = 0; k < K; ++k) {
                P3 c;
                double m2[6];
                member_geo(S[k], c, m2);
                const P3 d = sub(c, Gi.cen);
                for (int a = 0; a < 3; ++a) A[k * 9 + a] = d[a] * ih;
                for (int q = 0; q < 6; ++q) A[k * 9 + 3 + q] = (m2[q] + d[PA[q]] * d[PB[q]] - Gi.m2[q]) * ih * ih;
            }
            if (!pinv_normal(K, 9, A.data(), Pm.data())) {
                bad = 3;
                continue;
            }
            for (int s = 0; s < ns; ++s) {
                out.sten[(size_t)s * nc + i] = s < K ? S[s].id : (int32_t)i;
                for (int r = 0; r < 9; ++r)
                    out.pinv[(((size_t)r * (ns / 2) + s / 2) * nc + i) * 2 + (s & 1)] = s < K ? Pm[(size_t)r * K + s] : 0.0;
            }
            if (diagnostics) {
                for (int r = 0; r < 9; ++r)
                    for (int c2 = 0; c2 < 9; ++c2) {
                        double t = 0.0;
                        for (int k = 0; k < K; ++k) t += Pm[(size_t)r * K + k] * A[k * 9 + c2];
                        lres = std::max(lres, std::fabs(t - (r == c2 ? 1.0 : 0.0)));
                    }
            }
            // sub-stencil m: rows (c_t - c_i)/h of its three face neighbours, inverted
            for (int m = 0; m < 8; ++m) {
                double Am[3][3], X[3][3];
                for (int t = 0; t < 3; ++t) {
                    P3 c;
                    double m2[6];
                    member_geo(S[HEXSUB[m][t]], c, m2);
                    for (int a = 0; a < 3; ++a) Am[t][a] = (c[a] - Gi.cen[a]) * ih;
                }
                if (!inv3(Am, X)) bad = 4;
                for (int k = 0; k < 3; ++k)
                    for (int t = 0; t < 3; ++t) out.binv[((size_t)(m * 3 + k) * 3 + t) * nc + i] = X[k][t];
            }
            double *cg = out.cgeo.data();
            cg[0 * nc + i] = ih;
            for (int q = 0; q < 6; ++q) cg[(size_t)(1 + q) * nc + i] = Gi.m2[q] * ih * ih;
            cg[7 * nc + i] = 1.0 / Gi.vol;
            cg[8 * nc + i] = 6.0 * Gi.vol / asum[perm[i]];
        }
        std::lock_guard<std::mutex> lk(mu);
        resid_max = std::max(resid_max, lres);
    });
    if (bad == 3 || bad == 4) {
        err = bad == 3 ? "rank-deficient least-squares stencil" : "singular hexahedral sub-stencil (coplanar centroids)";
        return HGKS_E_BAD_MESH;
    }

    // ---- 7. remaining arrays ------------------------------------------------------
    out.cface.resize((size_t)6 * nc);
    for (int64_t i = 0; i < nc; ++i)
        for (int p = 0; p < 6; ++p) out.cface[(size_t)p * nc + i] = cface[i][p];
    out.fcell.resize((size_t)2 * nf);
    for (int64_t f = 0; f < nf; ++f) {
        out.fcell[f] = fcell[f][0];
        out.fcell[nf + f] = fcell[f][1];
    }
    out.gcell.assign(gcell.begin(), gcell.end());
    out.gkind.assign(gkind.begin(), gkind.end());
    out.gnrm.resize((size_t)3 * std::max<int64_t>(ng, 1));
    for (int64_t g = 0; g < ng; ++g)
        for (int a = 0; a < 3; ++a) out.gnrm[(size_t)a * ng + g] = gn[g][a];
    out.nc = nc;
    out.nf = nf;
    out.ng = ng;
    out.ns = ns;
    out.perm = std::move(perm);
    out.max_members = smax.load();
    out.min_members = smin.load();
    out.pinv_residual = resid_max;
    out.closure = closure;
    return HGKS_OK;
}

}  // namespace hgks
