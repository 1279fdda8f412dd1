// Host precompute of everything the GPU step needs for a tetrahedral mesh
// (Sec. 3.1 "Generation of geometric information" and Algorithm 1), laid out
// for the gfx950 kernels.  Runs once per mesh on the host, multithreaded.
//
//  1. unwrap every cell around its first node (periodic axes), volume, centroid,
//     central second moments by the vertex formula
//        int_T (x-c)_a (x-c)_b dV = |T|/20 sum_q (v_q-c)_a (v_q-c)_b;
//  2. faces: cell faces bucketed by their smallest node id and matched on the
//     other two (face p of a cell is opposite its node p, Sec. 3.1 item 1);
//  3. first-layer neighbours with integer periodic image shifts, then the
//     16-slot two-layer stencil (Algorithm 1; the paper's tetrahedral
//     sub-stencils of Sec. 2.3 then sit at fixed slots);
//  4. least-squares rows of each stencil member in the cell's scaled, centred
//     coordinates and their pseudo-inverses by Householder QR (Sec. 2.3:
//     constraints (1/|Omega_k|) int P = Q_k, solved in the least-squares sense);
//  5. Morton renumbering of the cells, faces ordered by left cell, Gauss points.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <memory>
#include <thread>

#include "hgks_internal.h"

namespace hgks {

int host_threads() {
    int n = 0;
    if (const char *e = std::getenv("OMP_NUM_THREADS")) n = std::atoi(e);
    if (n <= 0) n = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 32));
}

template <class F>
static void parallel_for(int64_t n, F &&f) {
    int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / 2048));
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([&f, b, e] { f(b, e); });
    }
    for (auto &x : th) x.join();
}

void parallel_range(int64_t n, const std::function<void(int64_t, int64_t)> &f) { parallel_for(n, f); }

void pinv0_quads_f32(const HostMesh &hm, float *out) {
    const int64_t n = hm.nc;
    const double *p = hm.pinv0.data();
    parallel_for(n, [&](int64_t b, int64_t e) {
        for (int64_t k = 0; k < 36; ++k)
            for (int64_t i = b; i < e; ++i)
                for (int64_t q = 0; q < 4; ++q)
                    out[(k * n + i) * 4 + q] = (float)p[((2 * k + q / 2) * n + i) * 2 + q % 2];
    });
}

// Pseudo-inverse of a full-column-rank m x n matrix (row-major, any m; n = 9 or 3) by
// the normal equations: P (n x m, row-major) = (A^T A)^{-1} A^T with a Cholesky
// factor of A^T A (the least-squares fit the oracle solves the same way).  Returns
// false when a pivot of the factor is negligible against the largest (rank
// deficiency; the squared form of the test |R_jj| > 1e-9 max |R| on a QR factor).
// With P == nullptr only the rank test runs.
namespace {
// the same with the column count fixed at compile time (the loops unroll)
template <int N>
bool pinv_normal_n(int m, const double *A, double *P) {
    double L[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += A[k * N + i] * A[k * N + j];
            L[i][j] = s;
        }
    double dmax = 0.0;
    for (int i = 0; i < N; ++i) dmax = std::max(dmax, L[i][i]);
    double id[N];                           // one division per pivot, not per column
    for (int j = 0; j < N; ++j) {
        double d = L[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 1e-18 * dmax)) return false;
        const double ljj = std::sqrt(d);
        L[j][j] = ljj;
        id[j] = 1.0 / ljj;
        for (int i = j + 1; i < N; ++i) {
            double s = L[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s * id[j];
        }
    }
    if (!P) return true;
    for (int c = 0; c < m; ++c) {          // column c of P solves (L L^T) x = row c of A
        double y[N];
        for (int i = 0; i < N; ++i) {
            double s = A[c * N + i];
            for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
            y[i] = s * id[i];
        }
        for (int i = N - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < N; ++k) s -= L[k][i] * y[k];
            y[i] = s * id[i];
            P[i * m + c] = y[i];
        }
    }
    return true;
}
}  // namespace

bool pinv_normal(int m, int n, const double *A, double *P) {
    if (n == 9) return pinv_normal_n<9>(m, A, P);
    if (n == 3) return pinv_normal_n<3>(m, A, P);
    return false;
}

namespace {

struct V3 {
    double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// A stencil member: cell id and, per axis, its placement: on a periodic axis the
// image shift k (x + k * period), on a non-periodic axis 0 (the cell itself), -1 or
// +1 (its mirror image in the low or high wall: 2 lo - x or 2 hi - x).
struct Member {
    int32_t cell;
    int8_t s[3];
    bool operator==(const Member &o) const {
        return cell == o.cell && s[0] == o.s[0] && s[1] == o.s[1] && s[2] == o.s[2];
    }
};

// Quadratic basis order: xx, yy, zz, xy, xz, yz (indices into a symmetric 3x3)
constexpr int QA[6] = {0, 1, 2, 0, 0, 1};
constexpr int QB[6] = {0, 1, 2, 1, 2, 2};

// Proper edge colouring of a graph with n vertices, edges (eu[e], ev[e]) and largest
// degree at most 4 (faces of tetrahedra): colour[e] in [0, k), no two edges of one
// colour at a vertex.  A bipartite graph gets k = 4 colours: an edge takes a colour
// free at both ends, or else the alternating path of the two colours free at either
// end is swapped first (it cannot return to the edge in a bipartite graph).  Any
// other graph gets at most 5 by the fan-rotation method of Misra and Gries.  Returns
// the number of colours used, or -1 if the result fails the final check.
int colour_edges(int32_t n, const std::vector<int32_t> &eu, const std::vector<int32_t> &ev,
                 std::vector<int8_t> &colour) {
    const int64_t m = (int64_t)eu.size();
    constexpr int MAXC = 5;
    std::vector<std::array<int32_t, 4>> inc(n);          // incident edges of each vertex
    std::vector<int8_t> deg(n, 0);
    for (int64_t e = 0; e < m; ++e) {
        for (int32_t x : {eu[e], ev[e]}) {
            if (deg[x] >= 4) return -1;
            inc[x][deg[x]++] = (int32_t)e;
        }
    }
    // two-colour the vertices: bipartite or not
    std::vector<int8_t> side(n, -1);
    bool bip = true;
    {
        std::vector<int32_t> stack;
        for (int32_t s0 = 0; s0 < n && bip; ++s0) {
            if (side[s0] >= 0) continue;
            side[s0] = 0;
            stack.push_back(s0);
            while (!stack.empty() && bip) {
                const int32_t x = stack.back();
                stack.pop_back();
                for (int k = 0; k < deg[x]; ++k) {
                    const int64_t e = inc[x][k];
                    const int32_t y = eu[e] == x ? ev[e] : eu[e];
                    if (side[y] < 0) {
                        side[y] = (int8_t)(1 - side[x]);
                        stack.push_back(y);
                    } else if (side[y] == side[x]) {
                        bip = false;
                    }
                }
            }
        }
    }
    const int K = bip ? 4 : 5;
    std::vector<std::array<int32_t, MAXC>> at(n);         // at[x][c]: edge of colour c at x, or -1
    for (auto &a : at) a.fill(-1);
    for (int64_t e = 0; e < m; ++e) colour[e] = -1;
    auto other = [&](int64_t e, int32_t x) { return eu[e] == x ? ev[e] : eu[e]; };
    auto free_at = [&](int32_t x, int c) { return at[x][c] < 0; };
    auto first_free = [&](int32_t x) {
        for (int c = 0; c < K; ++c)
            if (at[x][c] < 0) return c;
        return -1;
    };
    auto set = [&](int64_t e, int c) {
        colour[e] = (int8_t)c;
        at[eu[e]][c] = (int32_t)e;
        at[ev[e]][c] = (int32_t)e;
    };
    auto unset = [&](int64_t e) {
        const int c = colour[e];
        if (c < 0) return;
        if (at[eu[e]][c] == e) at[eu[e]][c] = -1;
        if (at[ev[e]][c] == e) at[ev[e]][c] = -1;
        colour[e] = -1;
    };
    // swap colours a and b along the maximal path that leaves x on its a-edge
    std::vector<int64_t> path;
    auto swap_path = [&](int32_t x, int a, int b) {
        path.clear();
        int c = a, d = b;
        int32_t y = x;
        while (at[y][c] >= 0) {
            const int64_t e = at[y][c];
            path.push_back(e);
            y = other(e, y);
            std::swap(c, d);
        }
        for (int64_t e : path) unset(e);
        for (size_t k = 0; k < path.size(); ++k) set(path[k], k % 2 == 0 ? b : a);
    };
    for (int64_t e = 0; e < m; ++e) {
        const int32_t u = eu[e], v = ev[e];
        if (bip) {
            const int a = first_free(u), b = first_free(v);
            if (a < 0 || b < 0) return -1;
            if (free_at(v, a)) {
                set(e, a);
                continue;
            }
            swap_path(v, a, b);          // v's a-edge becomes b: a is free at v, still at u
            if (!free_at(u, a) || !free_at(v, a)) return -1;
            set(e, a);
            continue;
        }
        // Misra-Gries: a maximal fan of u starting at v
        std::vector<int32_t> fan{v};
        while (true) {
            const int32_t last = fan.back();
            int32_t next = -1;
            for (int k = 0; k < deg[u] && next < 0; ++k) {
                const int64_t f = inc[u][k];
                if (colour[f] < 0) continue;
                const int32_t w = other(f, u);
                if (std::find(fan.begin(), fan.end(), w) != fan.end()) continue;
                if (free_at(last, colour[f])) next = w;
            }
            if (next < 0) break;
            fan.push_back(next);
        }
        const int c = first_free(u), d = first_free(fan.back());
        if (c < 0 || d < 0) return -1;
        if (c != d) swap_path(u, d, c);  // the cd-path from u, starting on its d-edge
        // the first fan vertex w at which d is free; the fan up to w stays a fan
        size_t wi = 0;
        while (wi < fan.size() && !free_at(fan[wi], d)) ++wi;
        if (wi == fan.size()) return -1;
        auto edge_to = [&](int32_t w) {
            for (int k = 0; k < deg[u]; ++k)
                if (other(inc[u][k], u) == w) return (int64_t)inc[u][k];
            return (int64_t)-1;
        };
        // rotate: (u, fan[i]) takes the colour of (u, fan[i+1]); (u, w) takes d
        for (size_t i = 0; i < wi; ++i) {
            const int64_t fi = edge_to(fan[i]), fj = edge_to(fan[i + 1]);
            const int cj = colour[fj];
            unset(fj);
            unset(fi);
            set(fi, cj);
        }
        const int64_t fw = edge_to(fan[wi]);
        unset(fw);
        if (!free_at(u, d) || !free_at(fan[wi], d)) return -1;
        set(fw, d);
    }
    // check: every edge coloured, no colour twice at a vertex
    int used = 0;
    for (int32_t x = 0; x < n; ++x) {
        int mask = 0;
        for (int k = 0; k < deg[x]; ++k) {
            const int c = colour[inc[x][k]];
            if (c < 0 || c >= K || (mask >> c) & 1) return -1;
            mask |= 1 << c;
            used = std::max(used, c + 1);
        }
    }
    return used;
}

uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

}  // namespace

hgks_status build_mesh(const hgks_params &prm, int64_t nn, const double *xyz, int64_t nc, int npc,
                       const int64_t *cn, const double *period_in, HostMesh &out, std::string &err,
                       bool diagnostics) {
    if (nn <= 0 || nc <= 0 || !xyz || !cn) {
        err = "empty mesh";
        return HGKS_E_INVALID_ARG;
    }
    if (npc != 4) {
        err = "only tetrahedral cells (nodes_per_cell = 4) are supported";
        return HGKS_E_INVALID_ARG;
    }
    if (nc >= (int64_t)1 << 30) {
        err = "too many cells";
        return HGKS_E_INVALID_ARG;
    }
    double per[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        per[a] = period_in ? period_in[a] : 0.0;
        if (!(per[a] >= 0.0) || !std::isfinite(per[a])) {
            err = "bad period";
            return HGKS_E_INVALID_ARG;
        }
    }
    for (int64_t k = 0; k < nc * 4; ++k)
        if (cn[k] < 0 || cn[k] >= nn) {
            err = "node id out of range";
            return HGKS_E_INVALID_ARG;
        }

    // extent of the nodes per axis: the walls of the non-periodic axes
    double wlo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, whi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t k = 0; k < nn; ++k)
        for (int a = 0; a < 3; ++a) {
            wlo[a] = std::min(wlo[a], xyz[3 * k + a]);
            whi[a] = std::max(whi[a], xyz[3 * k + a]);
        }

    // ---- 1. unwrapped vertices, volume, centroid, central second moments --------
    std::vector<std::array<V3, 4>> vert(nc);
    std::vector<V3> cen(nc);
    std::vector<double> vol(nc);
    std::vector<std::array<double, 6>> smom(nc);  // central second moments (xx,yy,zz,xy,xz,yz)
    std::atomic<int> bad{0};
    parallel_for(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            const double *x0 = xyz + 3 * cn[4 * c];
            for (int q = 0; q < 4; ++q) {
                const double *xq = xyz + 3 * cn[4 * c + q];
                double d[3];
                for (int a = 0; a < 3; ++a) {
                    d[a] = xq[a] - x0[a];
                    if (per[a] > 0) d[a] -= per[a] * std::nearbyint(d[a] / per[a]);
                }
                vert[c][q] = {x0[0] + d[0], x0[1] + d[1], x0[2] + d[2]};
            }
            V3 e1 = vert[c][1] - vert[c][0], e2 = vert[c][2] - vert[c][0], e3 = vert[c][3] - vert[c][0];
            double v6 = std::fabs(dot(e1, cross(e2, e3)));
            double ext = std::max({std::fabs(e1.x) + std::fabs(e2.x) + std::fabs(e3.x),
                                   std::fabs(e1.y) + std::fabs(e2.y) + std::fabs(e3.y),
                                   std::fabs(e1.z) + std::fabs(e2.z) + std::fabs(e3.z)});
            if (!(v6 > 6e-12 * ext * ext * ext)) bad = 1;
            vol[c] = v6 / 6.0;
            cen[c] = 0.25 * (vert[c][0] + vert[c][1] + vert[c][2] + vert[c][3]);
            for (int d = 0; d < 6; ++d) {
                double s = 0.0;
                for (int q = 0; q < 4; ++q) {
                    V3 w = vert[c][q] - cen[c];
                    s += comp(w, QA[d]) * comp(w, QB[d]);
                }
                smom[c][d] = s / 20.0;
            }
        }
    });
    if (bad) {
        err = "degenerate tetrahedron";
        return HGKS_E_BAD_MESH;
    }

    // ---- 2. faces: bucket every cell face by its smallest node ------------------
    std::vector<int64_t> bstart(nn + 1, 0);
    auto face_nodes = [&](int64_t c, int p, int64_t k[3]) {
        int t = 0;
        for (int q = 0; q < 4; ++q)
            if (q != p) k[t++] = cn[4 * c + q];
        std::sort(k, k + 3);
    };
    for (int64_t c = 0; c < nc; ++c)
        for (int p = 0; p < 4; ++p) {
            int64_t k[3];
            face_nodes(c, p, k);
            bstart[k[0] + 1]++;
        }
    for (int64_t i = 0; i < nn; ++i) bstart[i + 1] += bstart[i];
    std::vector<int64_t> bfill(bstart.begin(), bstart.end() - 1);
    std::vector<int64_t> bent(nc * 4);  // entries: c*4+p
    for (int64_t c = 0; c < nc; ++c)
        for (int p = 0; p < 4; ++p) {
            int64_t k[3];
            face_nodes(c, p, k);
            bent[bfill[k[0]]++] = c * 4 + p;
        }
    std::vector<int64_t> partner(nc * 4, -1);  // (c*4+p) -> (c'*4+p')
    parallel_for(nn, [&](int64_t b, int64_t e) {
        std::vector<std::pair<std::pair<int64_t, int64_t>, int64_t>> buf;
        for (int64_t node = b; node < e; ++node) {
            buf.clear();
            for (int64_t s = bstart[node]; s < bstart[node + 1]; ++s) {
                int64_t cp = bent[s], k[3];
                face_nodes(cp / 4, (int)(cp % 4), k);
                buf.push_back({{k[1], k[2]}, cp});
            }
            std::sort(buf.begin(), buf.end());
            for (size_t s = 0; s < buf.size();) {
                size_t t = s + 1;
                while (t < buf.size() && buf[t].first == buf[s].first) ++t;
                if (t - s == 2) {
                    partner[buf[s].second] = buf[s + 1].second;
                    partner[buf[s + 1].second] = buf[s].second;
                } else if (t - s == 1) {
                    // a wall face: all three nodes on the lowest or highest coordinate of a
                    // non-periodic axis; partner = -2 - (2 axis + side)
                    int64_t cp = buf[s].second, k[3];
                    face_nodes(cp / 4, (int)(cp % 4), k);
                    int code = -1;
                    for (int a = 0; a < 3 && code < 0; ++a) {
                        if (per[a] > 0) continue;
                        const double x0 = xyz[3 * k[0] + a], x1 = xyz[3 * k[1] + a], x2 = xyz[3 * k[2] + a];
                        if (x0 == x1 && x1 == x2 && (x0 == wlo[a] || x0 == whi[a])) code = 2 * a + (x0 == whi[a] ? 1 : 0);
                    }
                    if (code < 0) bad = 1;
                    partner[cp] = -2 - code;
                } else {
                    bad = 2;
                }
                s = t;
            }
        }
    });
    if (bad) {
        err = bad == 1 ? "boundary face off the walls (an unshared face must lie on the lowest or highest "
                         "coordinate of a non-periodic axis)"
                       : "non-conforming face";
        return HGKS_E_BAD_MESH;
    }

    // ---- 3. neighbours with integer image shifts --------------------------------
    // nb[c][p] = cell across face p; nsh[c][p] = shift k such that that cell's
    // coordinates + k*period are in c's frame.
    std::vector<std::array<int32_t, 4>> nb(nc);
    std::vector<std::array<std::array<int8_t, 3>, 4>> nsh(nc);
    std::vector<double> asum(nc, 0.0);
    parallel_for(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            double as = 0.0;
            for (int p = 0; p < 4; ++p) {
                int64_t o = partner[c * 4 + p];
                if (o < 0) {                    // wall face: the neighbour is the cell's mirror image
                    const int code = (int)(-2 - o), a = code / 2;
                    nb[c][p] = (int32_t)c;
                    for (int d = 0; d < 3; ++d) nsh[c][p][d] = 0;
                    nsh[c][p][a] = (int8_t)(code % 2 ? 1 : -1);
                    V3 t0 = vert[c][(p + 1) % 4], t1 = vert[c][(p + 2) % 4], t2 = vert[c][(p + 3) % 4];
                    as += 0.5 * std::sqrt(dot(cross(t1 - t0, t2 - t0), cross(t1 - t0, t2 - t0)));
                    continue;
                }
                int64_t c2 = o / 4;
                nb[c][p] = (int32_t)c2;
                int q0 = p == 0 ? 1 : 0;
                int64_t node = cn[4 * c + q0];
                int q2 = 0;
                while (cn[4 * c2 + q2] != node) ++q2;
                V3 d = vert[c][q0] - vert[c2][q2];
                for (int a = 0; a < 3; ++a) {
                    double k = per[a] > 0 ? std::nearbyint(comp(d, a) / per[a]) : 0.0;
                    nsh[c][p][a] = (int8_t)k;
                }
                V3 t0 = vert[c][(p + 1) % 4], t1 = vert[c][(p + 2) % 4], t2 = vert[c][(p + 3) % 4];
                as += 0.5 * std::sqrt(dot(cross(t1 - t0, t2 - t0), cross(t1 - t0, t2 - t0)));
            }
            asum[c] = as;
        }
    });

    // ---- 4. renumbering ---------------------------------------------------------
    std::vector<int64_t> perm(nc);
    for (int64_t c = 0; c < nc; ++c) perm[c] = c;
    if (prm.reorder) {
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = 1e300;
            hi[a] = -1e300;
        }
        for (int64_t c = 0; c < nc; ++c)
            for (int a = 0; a < 3; ++a) {
                double x = comp(cen[c], a);
                if (per[a] > 0) x -= per[a] * std::floor(x / per[a]);
                lo[a] = std::min(lo[a], x);
                hi[a] = std::max(hi[a], x);
            }
        std::vector<std::pair<uint64_t, int64_t>> key(nc);
        parallel_for(nc, [&](int64_t b, int64_t e) {
            for (int64_t c = b; c < e; ++c) {
                uint64_t code = 0;
                for (int a = 0; a < 3; ++a) {
                    double x = comp(cen[c], a);
                    if (per[a] > 0) x -= per[a] * std::floor(x / per[a]);
                    double t = hi[a] > lo[a] ? (x - lo[a]) / (hi[a] - lo[a]) : 0.0;
                    uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
                    code |= spread3(q) << a;
                }
                key[c] = {code, c};
            }
        });
        std::sort(key.begin(), key.end());
        for (int64_t c = 0; c < nc; ++c) perm[c] = key[c].second;
    }
    std::vector<int32_t> inv(nc);
    for (int64_t c = 0; c < nc; ++c) inv[perm[c]] = (int32_t)c;

    // ---- 5. stencils and pseudo-inverses, written in internal numbering --------
    // the per-cell data in internal (Morton) order first, so that a stencil's members
    // are read from nearby memory rather than from all over the caller's order
    std::vector<V3> cenI(nc);
    std::vector<std::array<double, 6>> smomI(nc);
    std::vector<double> hI(nc);
    std::vector<std::array<int32_t, 4>> nbI(nc);
    std::vector<std::array<std::array<int8_t, 3>, 4>> nshI(nc);
    parallel_for(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            const int64_t o = perm[c];
            cenI[c] = cen[o];
            smomI[c] = smom[o];
            hI[c] = std::cbrt(vol[o]);
            for (int p = 0; p < 4; ++p) nbI[c][p] = inv[nb[o][p]];
            nshI[c] = nsh[o];
        }
    });
    // centroid of a member in the frame of the cell whose stencil holds it
    auto place = [&](const Member &x) {
        V3 c = cenI[x.cell];
        double v[3] = {c.x, c.y, c.z};
        for (int a = 0; a < 3; ++a) {
            if (per[a] > 0)
                v[a] += x.s[a] * per[a];
            else if (x.s[a] != 0)
                v[a] = 2.0 * (x.s[a] < 0 ? wlo[a] : whi[a]) - v[a];
        }
        return V3{v[0], v[1], v[2]};
    };
    auto mirror_sign = [&](const Member &x, int a) { return per[a] <= 0 && x.s[a] != 0 ? -1.0 : 1.0; };
    // every entry of these arrays is written below (no fill on resize)
    out.sten.resize((size_t)SLOTS * nc);
    out.pinv0.resize((size_t)144 * nc);
    out.sshift.resize((size_t)4 * nc);
    std::atomic<int> members_max{0}, members_min{1 << 30}, dups{0};
    std::mutex mu;
    double resid_max = 0.0;
    parallel_for(nc, [&](int64_t b, int64_t e) {
        double local_resid = 0.0;
        int lmax = 0, lmin = 1 << 30, ldup = 0;
        for (int64_t c = b; c < e; ++c) {
            const int64_t i = c;                // internal ids throughout
            Member S[SLOTS];
            for (int p = 0; p < 4; ++p) S[p] = {nbI[i][p], {nshI[i][p][0], nshI[i][p][1], nshI[i][p][2]}};
            for (int m = 0; m < 4; ++m) {
                int32_t j = nbI[i][m];
                int t = 0;
                for (int q = 0; q < 4; ++q) {
                    Member x{nbI[j][q], {0, 0, 0}};
                    for (int a = 0; a < 3; ++a) {
                        const int s1 = nshI[i][m][a], s2 = nshI[j][q][a];
                        if (per[a] > 0) {
                            x.s[a] = (int8_t)(s1 + s2);
                        } else {        // mirror images compose: the same wall twice is the identity
                            if (s1 != 0 && s2 != 0 && s1 != s2) bad = 6;   // both walls: a translation
                            x.s[a] = (int8_t)(s2 == 0 ? s1 : (s1 == 0 ? s2 : 0));
                        }
                    }
                    if (x.cell == i && x.s[0] == 0 && x.s[1] == 0 && x.s[2] == 0) continue;
                    if (t < 3) S[4 + 3 * m + t] = x;
                    ++t;
                }
                if (t != 3) bad = 3;
            }
            // least-squares rows in the scaled coordinates xi = (x - c_i)/h_i
            const double ih = 1.0 / hI[i], ih2 = ih * ih;
            auto row = [&](const Member &x, double r[9]) {
                V3 d = place(x) - cenI[i];
                r[0] = d.x * ih;
                r[1] = d.y * ih;
                r[2] = d.z * ih;
                for (int q = 0; q < 6; ++q) {
                    // a mirror flips the sign of the mixed moments that involve its axis
                    const double sg = mirror_sign(x, QA[q]) * mirror_sign(x, QB[q]);
                    r[3 + q] = (sg * smomI[x.cell][q] + comp(d, QA[q]) * comp(d, QB[q]) - smomI[i][q]) * ih2;
                }
            };
            // distinct members of the big stencil (self excluded by construction)
            int first[SLOTS], nm = 0;
            double A[SLOTS * 9];
            Member uniq[SLOTS];
            for (int s = 0; s < SLOTS; ++s) {
                first[s] = -1;
                for (int u = 0; u < nm; ++u)
                    if (uniq[u] == S[s]) first[s] = -2 - u;
                if (first[s] == -1) {
                    uniq[nm] = S[s];
                    row(S[s], &A[nm * 9]);
                    first[s] = nm++;
                } else {
                    ++ldup;
                }
            }
            lmax = std::max(lmax, nm);
            lmin = std::min(lmin, nm);
            double Pk[9 * SLOTS];
            if (!pinv_normal(nm, 9, A, Pk)) {
                bad = 4;
                continue;
            }
            // residual |P A - I| (a diagnostic of hgks_inspect_mesh, skipped at upload)
            if (diagnostics)
            for (int r = 0; r < 9; ++r)
                for (int c = 0; c < 9; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < nm; ++k) s += Pk[r * nm + k] * A[k * 9 + c];
                    local_resid = std::max(local_resid, std::fabs(s - (r == c ? 1.0 : 0.0)));
                }
            // slot s of a cell reached twice keeps its member but gets zero weight
            for (int r = 0; r < 9; ++r)
                for (int s = 0; s < SLOTS; ++s)
                    out.pinv0[(((size_t)(r * 8 + s / 2)) * nc + c) * 2 + (s & 1)] = first[s] >= 0 ? Pk[r * nm + first[s]] : 0.0;
            for (int s = 0; s < SLOTS; ++s) out.sten[(size_t)s * nc + c] = S[s].cell;
            for (int w = 0; w < 4; ++w) {
                uint32_t word = 0;
                for (int s = 4 * w; s < 4 * w + 4; ++s) {
                    const uint32_t code = (uint32_t)((S[s].s[0] + 2) + 5 * (S[s].s[1] + 2) + 25 * (S[s].s[2] + 2));
                    word |= code << (8 * (s % 4));
                }
                out.sshift[(size_t)w * nc + c] = word;
            }
            // the four linear sub-stencil fits (first-layer minus one, plus N(i_m)) are
            // formed on the device; here only their rank is checked
            for (int m = 0; m < 4; ++m) {
                int sl[6] = {SUBFIRST[m][0], SUBFIRST[m][1], SUBFIRST[m][2], 4 + 3 * m, 5 + 3 * m, 6 + 3 * m};
                double As[6 * 3];
                int ns = 0;
                Member us[6];
                for (int t = 0; t < 6; ++t) {
                    bool dup = false;
                    for (int u = 0; u < ns; ++u)
                        if (us[u] == S[sl[t]]) dup = true;
                    if (dup) continue;
                    us[ns] = S[sl[t]];
                    const V3 d = place(S[sl[t]]) - cenI[i];      // the linear part of the row
                    As[ns * 3 + 0] = d.x * ih;
                    As[ns * 3 + 1] = d.y * ih;
                    As[ns * 3 + 2] = d.z * ih;
                    ++ns;
                }
                if (ns < 3 || !pinv_normal(ns, 3, As, nullptr)) {
                    bad = 4;
                    continue;
                }
            }
        }
        std::lock_guard<std::mutex> g(mu);
        resid_max = std::max(resid_max, local_resid);
        members_max = std::max(members_max.load(), lmax);
        members_min = std::min(members_min.load(), lmin);
        dups += ldup;
    });
    if (bad == 3) {
        err = "a neighbour does not have three other neighbours";
        return HGKS_E_BAD_MESH;
    }
    if (bad == 6) {
        err = "a stencil reaches both walls of a non-periodic axis (too few cells across it)";
        return HGKS_E_BAD_MESH;
    }
    if (bad == 4) {
        err = "rank-deficient least-squares stencil";
        return HGKS_E_BAD_MESH;
    }

    // ---- 6. faces in internal numbering: left = smaller internal id -------------
    // counting sort by left cell, then by right cell; a wall face has the wall cell
    // on the left and right = -1 (the ghost)
    auto is_wall = [&](int64_t c, int p) { return partner[c * 4 + p] < 0; };
    std::vector<int64_t> fstart(nc + 1, 0);
    int64_t nwall = 0;
    for (int64_t c = 0; c < nc; ++c)
        for (int p = 0; p < 4; ++p) {
            int64_t c2 = nb[c][p];
            if (is_wall(c, p)) {
                fstart[inv[c] + 1]++;
                ++nwall;
            } else if (inv[c] < inv[c2]) {
                fstart[inv[c] + 1]++;
            }
        }
    for (int64_t c = 0; c < nc; ++c) fstart[c + 1] += fstart[c];
    const int64_t nf = fstart[nc];
    if (2 * nf != 4 * nc + nwall) {
        err = "face count mismatch";
        return HGKS_E_BAD_MESH;
    }
    struct FaceRec {
        int32_t l, r;      // internal ids
        int32_t cl;        // caller id of the left cell
        int8_t pl;         // local face index in the left cell
    };
    std::vector<FaceRec> faces(nf);
    {
        std::vector<int64_t> fill(fstart.begin(), fstart.end() - 1);
        for (int64_t c = 0; c < nc; ++c)
            for (int p = 0; p < 4; ++p) {
                int64_t c2 = nb[c][p];
                if (is_wall(c, p))
                    faces[fill[inv[c]]++] = {inv[c], -1, (int32_t)c, (int8_t)p};
                else if (inv[c] < inv[c2])
                    faces[fill[inv[c]]++] = {inv[c], inv[c2], (int32_t)c, (int8_t)p};
            }
        parallel_for(nc, [&](int64_t b, int64_t e) {
            for (int64_t c = b; c < e; ++c)
                std::sort(faces.begin() + fstart[c], faces.begin() + fstart[c + 1],
                          [](const FaceRec &x, const FaceRec &y) { return x.r < y.r || (x.r == y.r && x.pl < y.pl); });
        });
        // within each block of 64 faces (a flux workgroup's tile), order by the right
        // cell: the left cells stay the block's few consecutive cells, and the update's
        // gathers of the faces a cell sees as the right cell come in cell order (update
        // 113 -> 104 us at 6 64^3)
        parallel_for((nf + 63) / 64, [&](int64_t b, int64_t e) {
            for (int64_t k = b; k < e; ++k)
                std::stable_sort(faces.begin() + 64 * k, faces.begin() + std::min<int64_t>(nf, 64 * k + 64),
                                 [](const FaceRec &x, const FaceRec &y) { return x.r < y.r; });
        });
    }
    // colour classes for the coloured accumulation: no two faces of a class share a
    // cell.  Faces are the edges of the cell graph (a wall face an edge to a ghost of
    // its own), whose largest degree is 4; colour_edges uses 4 classes when the graph
    // is bipartite (Koenig's theorem) and at most 5 otherwise (Vizing's theorem).
    std::vector<int8_t> colour(nf, 0);
    int ncol = 1;
    if (prm.accumulation == HGKS_ACC_COLOURED) {
        std::vector<int32_t> eu(nf), ev(nf);
        int32_t ghost = (int32_t)nc;
        for (int64_t f = 0; f < nf; ++f) {
            eu[f] = faces[f].l;
            ev[f] = faces[f].r >= 0 ? faces[f].r : ghost++;
        }
        ncol = colour_edges(ghost, eu, ev, colour);
        if (ncol < 0) {
            err = "internal error: face colouring";
            return HGKS_E_BAD_MESH;
        }
    }
    std::vector<int64_t> forder(nf);
    for (int64_t f = 0; f < nf; ++f) forder[f] = f;
    out.colour_offsets.assign(ncol + 1, 0);
    if (prm.accumulation == HGKS_ACC_COLOURED) {
        std::stable_sort(forder.begin(), forder.end(), [&](int64_t a, int64_t b) { return colour[a] < colour[b]; });
    }
    for (int64_t f = 0; f < nf; ++f) out.colour_offsets[colour[f] + 1]++;
    for (int k = 0; k < ncol; ++k) out.colour_offsets[k + 1] += out.colour_offsets[k];

    // ---- 7. pack device arrays --------------------------------------------------
    out.nc = nc;
    out.nf = nf;
    out.perm = perm;
    // every entry of these arrays is written below (no fill on resize)
    out.cen.resize((size_t)3 * nc);
    out.cgeo.resize((size_t)CGEO * nc);
    out.cface.resize((size_t)4 * nc);
    out.fcell.resize((size_t)2 * nf);
    out.fgeo.resize((size_t)FGEO * nf);
    parallel_for(nc, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            int64_t o = perm[c];
            for (int a = 0; a < 3; ++a) out.cen[(size_t)a * nc + c] = comp(cen[o], a);
            double h = std::cbrt(vol[o]);
            out.cgeo[0 * (size_t)nc + c] = 1.0 / h;
            for (int q = 0; q < 6; ++q) out.cgeo[(size_t)(1 + q) * nc + c] = smom[o][q] / (h * h);
            out.cgeo[7 * (size_t)nc + c] = 1.0 / vol[o];
            out.cgeo[8 * (size_t)nc + c] = 6.0 * vol[o] / asum[o];
        }
    });
    // faces
    std::vector<int8_t> cfill(nc, 0);
    for (int64_t k = 0; k < nf; ++k) {
        const FaceRec &F = faces[forder[k]];
        out.fcell[k] = F.l;
        out.fcell[nf + k] = F.r;
        out.cface[(size_t)cfill[F.l]++ * nc + F.l] = (int32_t)(k << 1);
        if (F.r >= 0) out.cface[(size_t)cfill[F.r]++ * nc + F.r] = (int32_t)((k << 1) | 1);
    }
    parallel_for(nf, [&](int64_t b, int64_t e) {
        for (int64_t k = b; k < e; ++k) {
            const FaceRec &F = faces[forder[k]];
            int64_t lo = F.cl;       // caller id of the left cell
            int p = F.pl;
            int64_t ro = nb[lo][p];
            V3 tri[3];
            int t = 0;
            for (int q = 0; q < 4; ++q)
                if (q != p) tri[t++] = vert[lo][q];
            V3 nrm = cross(tri[1] - tri[0], tri[2] - tri[0]);
            double len = std::sqrt(dot(nrm, nrm));
            nrm = (1.0 / len) * nrm;
            V3 fc = (1.0 / 3.0) * (tri[0] + tri[1] + tri[2]);
            if (dot(nrm, fc - cen[lo]) < 0) nrm = -1.0 * nrm;
            // right centroid in the left frame; at a wall the ghost side is evaluated from
            // the wall cell's own record at the same point (its mirror image), so yr = yl
            V3 cr = cen[lo];
            if (F.r >= 0) {
                V3 shift = {nsh[lo][p][0] * per[0], nsh[lo][p][1] * per[1], nsh[lo][p][2] * per[2]};
                cr = cen[ro] + shift;
                if (!(dot(nrm, cr - fc) > 0.0)) bad = 5;   // both cells on one side: overlapping / folded
            }
            // value v of face k sits in pair row v/2, lane v%2
            auto put = [&](int v, double x) { out.fgeo[((size_t)(v / 2) * nf + k) * 2 + (v & 1)] = x; };
            put(0, nrm.x);
            put(1, nrm.y);
            put(2, nrm.z);
            put(3, 0.5 * len);
            for (int q = 0; q < 3; ++q) {
                // 3-point degree-2 rule: barycentric permutations of (2/3, 1/6, 1/6)
                V3 xg = (2.0 / 3.0) * tri[q] + (1.0 / 6.0) * (tri[(q + 1) % 3] + tri[(q + 2) % 3]);
                V3 yl = xg - cen[lo];
                for (int a = 0; a < 3; ++a) put(4 + 3 * q + a, comp(yl, a));
            }
            // left minus right centroid: a point's offset from the right centroid is its
            // left offset plus this (zero at a wall: cr is the wall cell's own centroid)
            V3 dlr = cen[lo] - cr;
            for (int a = 0; a < 3; ++a) put(13 + a, comp(dlr, a));
        }
    });
    if (bad == 5) {
        err = "overlapping or folded cells (a face does not separate its two cells)";
        return HGKS_E_BAD_MESH;
    }
    for (int64_t c = 0; c < nc; ++c)
        if (cfill[c] != 4) {
            err = "cell without four faces";
            return HGKS_E_BAD_MESH;
        }
    // closure: the outward n S of each cell's four faces sum to zero
    double closure = 0.0;
    parallel_for(nc, [&](int64_t b, int64_t e) {
        double lmax = 0.0;
        for (int64_t c = b; c < e; ++c) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int p = 0; p < 4; ++p) {
                const int32_t code = out.cface[(size_t)p * nc + c];
                const int64_t k = code >> 1;
                const double sS = (code & 1 ? -1.0 : 1.0) * out.fgeo[((size_t)1 * nf + k) * 2 + 1];
                for (int a = 0; a < 3; ++a) acc[a] += out.fgeo[((size_t)(a / 2) * nf + k) * 2 + (a & 1)] * sS;
            }
            for (int a = 0; a < 3; ++a) lmax = std::max(lmax, std::fabs(acc[a]));
        }
        std::lock_guard<std::mutex> g(mu);
        closure = std::max(closure, lmax);
    });
    out.max_members = members_max;
    out.min_members = members_min;
    out.dup_slots = dups;
    out.pinv_residual = resid_max;
    out.n_wall_faces = nwall;
    for (int a = 0; a < 3; ++a) {
        out.mir[a][0] = per[a] > 0 ? 0.0 : 2.0 * wlo[a];
        out.mir[a][1] = per[a] > 0 ? 0.0 : 2.0 * whi[a];
    }
    out.closure = closure;
    return HGKS_OK;
}

}  // namespace hgks
