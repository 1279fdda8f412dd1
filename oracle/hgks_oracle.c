/*
 * hgks_oracle.c -- plain FP64 CPU reference of one explicit
 * HGKS step (third-order unstructured WENO, Gauss-point gas-kinetic flux,
 * two-stage fourth-order update) on tetrahedral and hexahedral meshes.
 *
 * TEST INFRASTRUCTURE ONLY.  It is linked by the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product path, and it
 * shares no code with the GPU library.  It is written for obviousness, not speed:
 * every step follows the paper (arXiv 2407.00656, Sec. 2) in the paper's order:
 *
 *   geometry ............ Sec. 3.1 (areas, volumes, local frames)
 *   stencils ............ Sec. 3.1 item 4 / Algorithm 1, Sec. 2.3 (tet and hex
 *                         sub-stencils)
 *   WENO ................ Sec. 2.3, Eqs. (polys) and (weno), WENO-Z weights,
 *                         smoothness indicators beta_m, gamma_0 = 1 - M gamma
 *   gas-kinetic flux .... Sec. 2.1, Eqs. (flux-G), (flux), compatibility
 *                         condition for Q0, slope relations <a>, <a.u + A> = 0
 *   time fit ............ Sec. 2.2, Eq. (expansion-1) and its 2x2 system
 *   S2O4 update ......... Sec. 2.2
 *   viscous flow ........ Sec. 5.2 (mu = mu_inf (T/T_inf)^0.7, no-slip adiabatic
 *                         wall, far field by Riemann invariants)
 *
 * Readings where the paper is silent (all are parameters or documented choices):
 *   - 3-point degree-2 Gauss rule on each triangular face (weights 1/3); on a
 *     hexahedron's bilinear face the 2x2 Gauss-Legendre rule in the face's
 *     bilinear parameters, each point with its own unit normal and weight
 *     |x_s x x_t| / 4 (the weights sum to the face's area up to the rule's
 *     error, and the weighted normals to its exact vector area);
 *   - cell integrals: the 4-point degree-2 rule on a tetrahedron; the 3x3x3
 *     Gauss-Legendre rule over the trilinear map of a hexahedron (exact for the
 *     monomials of degree <= 2 times the map's Jacobian);
 *   - WENO-Z with exponent 1 and the epsilon given in the parameters;
 *   - unweighted least squares in cell-scaled centroid coordinates, solved by
 *     normal equations + Cholesky;
 *   - the slopes of the equilibrium state use dQ0 = (dQ_l + dQ_r)/2;
 *   - tau = 0 (smooth flow, Sec. 5.1), tau = eps*dt + C*|pl-pr|/(pl+pr)*dt, or
 *     (viscous) tau = mu(T0)/p0 + C*|pl-pr|/(pl+pr)*dt with T = p/rho;
 *   - Prandtl number: BGK has Pr = 1; for Pr != 1 (viscous mode only) the energy
 *     flux takes (1/Pr - 1) times the heat flux of the interface distribution,
 *     measured in the frame of the interface equilibrium velocity U0;
 *   - dt = CFL * min_i h_i / (|U_i| + c_i), h_i = 6|Omega_i| / sum_p S_ip;
 *   - positivity fallback at Gauss points (where a reconstructed side is
 *     non-physical the point is first order: zero gradients, cell averages for
 *     the non-physical sides), which acts only at discontinuities.
 *
 * Conventions: cells are 0-based.  Face p of a tetrahedron is the one opposite
 * its node p (Sec. 3.1 item 1).  A hexahedron lists nodes 0-3 around one face and
 * nodes 4-7 above them (node k+4 joined to node k); its faces, in the paper's
 * numbering 1..6 (Sec. 2.3, where faces 1 and 6 are opposite and 2..5 go around)
 * are, 0-based: 0 = (0,1,2,3), 1 = (0,1,5,4), 2 = (1,2,6,5), 3 = (2,3,7,6),
 * 4 = (3,0,4,7), 5 = (4,5,6,7).  The neighbour across face p is "i_{p+1}" of
 * Sec. 2.3.  Meshes may be periodic: period[a] > 0 identifies x_a with
 * x_a + period[a]; each cell is unwrapped around its first node.
 *
 * Boundaries (Algorithm 1 gives a boundary face a ghost neighbour "according to
 * the boundary condition").  Without a boundary-face list, an axis with period 0
 * ends in two planar transmissive walls at the extreme node coordinates.  The
 * ghost across such a wall face is the mirror image of the wall cell in the wall
 * plane and holds the wall cell's state.  A ghost's face neighbours are the
 * mirror images of the wall cell's neighbours (so a two-layer stencil near a
 * wall contains mirror images of interior cells, and near an edge images under
 * two mirrors), all holding the state of the cell they image.  Stencil members
 * are therefore (cell, x -> s*x + o per axis) pairs: s = 1 for periodic images,
 * s = -1 for mirrors.  Because a ghost's stencil and data are the mirror image of
 * the wall cell's, so is its reconstruction: at a wall Gauss point its value is
 * the wall cell's and its gradient the wall cell's reflected in the wall.
 *
 * With a boundary-face list (no periodic axis), each listed face is a no-slip
 * adiabatic wall or a far-field face.  Its ghost is the cell's mirror image in
 * the face's mean plane, has no neighbours of its own, and holds the ghost state
 * of the cell's average: at a wall (rho, -rho U, rho E), i.e. zero velocity and
 * the cell's temperature on the face; at the far field the Riemann-invariant
 * state of the cell and the free stream.  At a Gauss point of such a face the
 * right side is the same ghost map applied to the left reconstruction: at a wall
 * the value with its momentum negated and the gradient reflected in the plane
 * (momentum rows negated), at the far field the Riemann-invariant state of the
 * left point value with a zero gradient.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_MESH 2
#define ORC_E_NONPHYS 6

#define MAXSTEN 40
#define MAXSUB 8
#define MAXM 8              /* sub-stencils per cell: 4 (tet), 8 (hex) */
#define MAXFC 6             /* faces per cell */
#define MAXGP 4             /* Gauss points per face */
#define MAXCQ 27            /* cell quadrature points */

typedef struct {
    double gamma;
    double cfl;
    int tau_mode;          /* 0: tau = 0;  1: tau = tau_eps*dt + tau_C*|pl-pr|/(pl+pr)*dt;
                              2: tau = mu(T0)/p0 + tau_C*|pl-pr|/(pl+pr)*dt (viscous) */
    double tau_eps;
    double tau_C;
    double weno_eps;
    double gamma_lin;      /* linear weight of each sub-stencil; gamma_0 = 1 - M*gamma_lin */
    double mu_ref;         /* viscous mode: mu = mu_ref * (T / T_ref)^mu_exp, T = p / rho */
    double T_ref;
    double mu_exp;
    double prandtl;
    double farfield[5];    /* free stream (rho, U, V, W, p) of far-field faces */
} orc_params;

/* boundary kinds of listed boundary faces */
#define ORC_BC_WALL 1      /* no-slip adiabatic wall */
#define ORC_BC_FAR 2       /* far field (Riemann invariants) */

/* placement of a stencil member: x -> s*x + o on each axis */
typedef struct { double s[3], o[3]; } xform;
static const xform XID = {{1.0, 1.0, 1.0}, {0.0, 0.0, 0.0}};

typedef struct {
    int64_t nc, nn, nf;
    int npc, nfc, ngp, msub;       /* nodes per cell, faces per cell, Gauss points per face, sub-stencils */
    double period[3];
    double lo[3], hi[3];            /* node extent per axis (the walls of non-periodic axes) */
    double (*vert)[8][3];          /* unwrapped vertices of each cell */
    double *vol;
    double (*cen)[3];
    double *h;                      /* |Omega|^(1/3): length scale of the local coordinates */
    double *hdt;                    /* 6|Omega| / sum of face areas */
    /* faces */
    int64_t (*fcell)[2];            /* left, right (-1: a boundary face, the right side is the ghost) */
    int *fkind;                     /* 0 interior or transmissive wall, ORC_BC_WALL, ORC_BC_FAR */
    double (*fshift)[3];            /* right cell's image in the left cell's frame = right + fshift */
    double (*fnrm)[3];              /* mean unit normal (vector area / area), left -> right */
    double *farea;                  /* sum of the Gauss weights */
    double (*fgp)[MAXGP][3];        /* Gauss points, left cell's frame */
    double (*fpn)[MAXGP][3];        /* unit normal at each Gauss point */
    double (*fpw)[MAXGP];           /* weight of each Gauss point (area units) */
    int64_t (*cface)[MAXFC];        /* local face p of each cell */
    /* neighbours i_1..i_nfc; an id >= nc is ghost (id - nc) of a listed boundary face */
    int64_t (*nb)[MAXFC];           /* the cell itself across a transmissive wall face */
    xform (*nbx)[MAXFC];            /* placement of that neighbour (a mirror across a wall face) */
    /* ghosts of listed boundary faces */
    int64_t ng;
    int64_t *gcell, *gface;
    int *gkind;
    double (*gpt)[3], (*gnrm)[3];   /* mirror plane: a point and the unit normal */
    /* big stencil and the sub-stencils (members other than the cell itself) */
    int *nsten;
    int64_t (*sten)[MAXSTEN];
    xform (*stx)[MAXSTEN];
    int (*nsub)[MAXM];
    int64_t (*sub)[MAXM][MAXSUB];
    xform (*subx)[MAXM][MAXSUB];
} orc_mesh;

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static void sub3(const double *a, const double *b, double *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void set_err(char *err, int errlen, const char *msg) {
    if (err && errlen > 0) { strncpy(err, msg, (size_t)errlen - 1); err[errlen - 1] = 0; }
}

/* Degree-2 exact 4-point rule on a tetrahedron (points a*V_q + b*sum of others). */
static void tet_points(const double v[4][3], double pts[4][3]) {
    const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
    const double b = (5.0 - sqrt(5.0)) / 20.0;
    for (int q = 0; q < 4; ++q)
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int r = 0; r < 4; ++r) s += (r == q ? a : b) * v[r][d];
            pts[q][d] = s;
        }
}

/* Basis exponents for p_d, |d| = 1..2 (Eq. polys): x, y, z, xx, yy, zz, xy, xz, yz. */
static const int DEXP[9][3] = {{1,0,0},{0,1,0},{0,0,1},{2,0,0},{0,2,0},{0,0,2},{1,1,0},{1,0,1},{0,1,1}};

static double ipow(double x, int e) { double r = 1.0; for (int k = 0; k < e; ++k) r *= x; return r; }
static double mono(const int e[3], const double *xi) { return ipow(xi[0], e[0]) * ipow(xi[1], e[1]) * ipow(xi[2], e[2]); }
/* d/dxi_j of xi^e */
static double dmono(const int e[3], int j, const double *xi) {
    if (e[j] == 0) return 0.0;
    int f[3] = {e[0], e[1], e[2]};
    f[j] -= 1;
    return (double)e[j] * mono(f, xi);
}
/* d^2/(dxi_j dxi_k) of xi^e */
static double d2mono(const int e[3], int j, int k, const double *xi) {
    int f[3] = {e[0], e[1], e[2]};
    double c = (double)f[j];
    if (f[j] == 0) return 0.0;
    f[j] -= 1;
    c *= (double)f[k];
    if (f[k] == 0) return 0.0;
    f[k] -= 1;
    return c * mono(f, xi);
}

/* Mean over tetrahedron `v` (any frame) of the 9 monomials in the scaled coordinates
 * of a cell with centroid c and length h: xi = (x - c)/h. */
static void tet_monomial_means(const double v[4][3], const double *c, double h, double out[9]) {
    double pts[4][3];
    tet_points(v, pts);
    for (int d = 0; d < 9; ++d) out[d] = 0.0;
    for (int q = 0; q < 4; ++q) {
        double xi[3] = {(pts[q][0] - c[0]) / h, (pts[q][1] - c[1]) / h, (pts[q][2] - c[2]) / h};
        for (int d = 0; d < 9; ++d) out[d] += 0.25 * mono(DEXP[d], xi);
    }
}

/* Hexahedron: reference coordinates of node k on [0,1]^3 (nodes 0-3 at zeta = 0
 * going around, node k+4 above node k), and the six faces in cyclic node order. */
static const int HXI[8][3] = {{0,0,0},{1,0,0},{1,1,0},{0,1,0},{0,0,1},{1,0,1},{1,1,1},{0,1,1}};
static const int HEXF[6][4] = {{0,1,2,3},{0,1,5,4},{1,2,6,5},{2,3,7,6},{3,0,4,7},{4,5,6,7}};
/* hex sub-stencils (Sec. 2.3): the face neighbours of each, 0-based faces */
static const int HEXSUB[8][3] = {{0,1,2},{0,2,3},{0,3,4},{0,4,1},{5,1,2},{5,2,3},{5,3,4},{5,4,1}};
/* tet sub-stencils: S_1 = {i1,i2,i3} + N(i1), S_2 = {i1,i2,i4} + N(i2),
 * S_3 = {i2,i3,i4} + N(i3), S_4 = {i3,i1,i4} + N(i4) */
static const int TETSUB[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {2, 0, 3}};

/* Gauss-Legendre rules on [0, 1] */
static const double GL2X[2] = {0.21132486540518711775, 0.78867513459481288225};
static const double GL3X[3] = {0.11270166537925831148, 0.5, 0.88729833462074168852};
static const double GL3W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

/* Trilinear map of a hexahedron at reference point r: position x and det dx/dr. */
static double hex_map(const double v[8][3], const double r[3], double x[3]) {
    double J[3][3] = {{0}};
    for (int a = 0; a < 3; ++a) x[a] = 0.0;
    for (int k = 0; k < 8; ++k) {
        double f[3], df[3];
        for (int d = 0; d < 3; ++d) {
            f[d] = HXI[k][d] ? r[d] : 1.0 - r[d];
            df[d] = HXI[k][d] ? 1.0 : -1.0;
        }
        const double N = f[0] * f[1] * f[2];
        const double dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
        for (int a = 0; a < 3; ++a) {
            x[a] += N * v[k][a];
            for (int d = 0; d < 3; ++d) J[a][d] += dN[d] * v[k][a];
        }
    }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Quadrature of a cell: points and weights (weights sum to the volume).
 * Tet: the degree-2 four-point rule; hex: 3x3x3 Gauss-Legendre over the trilinear
 * map.  jmin/jmax (nullable) receive the extreme Jacobians (hex). */
static int cell_quadrature(int npc, const double v[8][3], double pts[MAXCQ][3], double wts[MAXCQ], double *jmin,
                           double *jmax) {
    if (npc == 4) {
        tet_points(v, pts);
        double e1[3], e2[3], e3[3], cr[3];
        sub3(v[1], v[0], e1);
        sub3(v[2], v[0], e2);
        sub3(v[3], v[0], e3);
        cross3(e2, e3, cr);
        const double vol = fabs(dot3(e1, cr)) / 6.0;
        for (int q = 0; q < 4; ++q) wts[q] = 0.25 * vol;
        if (jmin) *jmin = vol;
        if (jmax) *jmax = vol;
        return 4;
    }
    int n = 0;
    double lo = INFINITY, hi = -INFINITY;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                const double r[3] = {GL3X[a], GL3X[b], GL3X[c]};
                const double J = hex_map(v, r, pts[n]);
                lo = fmin(lo, J); hi = fmax(hi, J);
                wts[n] = GL3W[a] * GL3W[b] * GL3W[c] * fabs(J);
                ++n;
            }
    if (jmin) *jmin = lo;
    if (jmax) *jmax = hi;
    return n;
}

/* Mean of the 9 scaled monomials over a cell with vertices v (any frame). */
static void cell_monomial_means(int npc, const double v[8][3], const double *c, double h, double out[9]) {
    if (npc == 4) { tet_monomial_means(v, c, h, out); return; }
    double pts[MAXCQ][3], wts[MAXCQ];
    const int n = cell_quadrature(npc, v, pts, wts, NULL, NULL);
    double V = 0.0;
    for (int d = 0; d < 9; ++d) out[d] = 0.0;
    for (int q = 0; q < n; ++q) {
        double xi[3] = {(pts[q][0] - c[0]) / h, (pts[q][1] - c[1]) / h, (pts[q][2] - c[2]) / h};
        V += wts[q];
        for (int d = 0; d < 9; ++d) out[d] += wts[q] * mono(DEXP[d], xi);
    }
    for (int d = 0; d < 9; ++d) out[d] /= V;
}

/* Least squares min ||A x - B|| via the normal equations and Cholesky.
 * A: m x n row-major, B: m x r, X: n x r.  Returns 0 or -1 (not positive definite). */
static int lsq_normal(int m, int n, const double *A, int r, const double *B, double *X) {
    double N[9 * 9], R[9 * 5], Lc[9 * 9];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += A[k * n + a] * A[k * n + b];
            N[a * n + b] = s;
        }
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < r; ++c) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += A[k * n + a] * B[k * r + c];
            R[a * r + c] = s;
        }
    memset(Lc, 0, sizeof(Lc));
    for (int j = 0; j < n; ++j) {
        double s = N[j * n + j];
        for (int k = 0; k < j; ++k) s -= Lc[j * n + k] * Lc[j * n + k];
        if (!(s > 1e-14 * N[j * n + j]) || !(s > 0.0)) return -1;
        Lc[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = N[i * n + j];
            for (int k = 0; k < j; ++k) t -= Lc[i * n + k] * Lc[j * n + k];
            Lc[i * n + j] = t / Lc[j * n + j];
        }
    }
    for (int c = 0; c < r; ++c) {
        double y[9];
        for (int i = 0; i < n; ++i) {
            double t = R[i * r + c];
            for (int k = 0; k < i; ++k) t -= Lc[i * n + k] * y[k];
            y[i] = t / Lc[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < n; ++k) t -= Lc[k * n + i] * X[k * r + c];
            X[i * r + c] = t / Lc[i * n + i];
        }
    }
    return 0;
}

/* Dense n x n solve with partial pivoting (n <= 5). */
static int gauss_solve(int n, const double *Ain, const double *bin, double *x) {
    double A[25], b[5];
    memcpy(A, Ain, sizeof(double) * n * n);
    memcpy(b, bin, sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r) if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return -1;
        if (p != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[p * n + k]; A[p * n + k] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* mesh: connectivity (Sec. 3.1) and geometry                                */
/* ------------------------------------------------------------------------- */

typedef struct { int64_t key[4]; int64_t cell; int p; } face_rec;

static int cmp_key(const int64_t *x, const int64_t *y) {
    for (int k = 0; k < 4; ++k) {
        if (x[k] < y[k]) return -1;
        if (x[k] > y[k]) return 1;
    }
    return 0;
}

static int cmp_face(const void *a, const void *b) {
    const face_rec *x = (const face_rec *)a, *y = (const face_rec *)b;
    int c = cmp_key(x->key, y->key);
    if (c) return c;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->p - y->p;
}

/* sorted node ids of a face; a triangle's fourth key is -1 */
static void face_key(const int64_t *nodes, int nk, int64_t key[4]) {
    for (int k = 0; k < 4; ++k) key[k] = k < nk ? nodes[k] : -1;
    for (int a = 0; a < nk; ++a)
        for (int b = a + 1; b < nk; ++b)
            if (key[b] < key[a]) { int64_t t = key[a]; key[a] = key[b]; key[b] = t; }
}

/* local node q of face p (nk nodes, cyclic order) */
static int face_node(int npc, int p, int k) {
    if (npc == 8) return HEXF[p][k];
    return k + (k >= p ? 1 : 0);        /* the three nodes other than p */
}

void orc_mesh_free(orc_mesh *m);

static int same_member(int64_t c1, const xform *x1, int64_t c2, const xform *x2) {
    if (c1 != c2) return 0;
    for (int a = 0; a < 3; ++a)
        if (x1->s[a] != x2->s[a] || fabs(x1->o[a] - x2->o[a]) > 1e-9 * (1.0 + fabs(x1->o[a]))) return 0;
    return 1;
}

/* x -> A(B(x)) */
static xform compose(const xform *A, const xform *B) {
    xform r;
    for (int a = 0; a < 3; ++a) { r.s[a] = A->s[a] * B->s[a]; r.o[a] = A->s[a] * B->o[a] + A->o[a]; }
    return r;
}

/* Gauss points, their unit normals and weights of a face given its nodes in cyclic
 * order (left cell's frame).  Returns the number of points. */
static int face_points(int nk, const double fv[4][3], double gp[MAXGP][3], double gn[MAXGP][3], double gw[MAXGP]) {
    if (nk == 3) {
        double e1[3], e2[3], nrm[3];
        sub3(fv[1], fv[0], e1);
        sub3(fv[2], fv[0], e2);
        cross3(e1, e2, nrm);
        const double len = sqrt(dot3(nrm, nrm));
        /* 3-point degree-2 rule: barycentric permutations of (2/3, 1/6, 1/6) */
        for (int g = 0; g < 3; ++g) {
            for (int a = 0; a < 3; ++a) {
                double s_ = 0.0;
                for (int v = 0; v < 3; ++v) s_ += (v == g ? 2.0 / 3.0 : 1.0 / 6.0) * fv[v][a];
                gp[g][a] = s_;
                gn[g][a] = nrm[a] / len;
            }
            gw[g] = 0.5 * len / 3.0;
        }
        return 3;
    }
    /* bilinear patch x(s,t) = (1-s)(1-t) a + s(1-t) b + s t c + (1-s) t d */
    int g = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j, ++g) {
            const double s_ = GL2X[i], t = GL2X[j];
            double xs[3], xt[3], nrm[3];
            for (int a = 0; a < 3; ++a) {
                gp[g][a] = (1 - s_) * (1 - t) * fv[0][a] + s_ * (1 - t) * fv[1][a] + s_ * t * fv[2][a] + (1 - s_) * t * fv[3][a];
                xs[a] = (1 - t) * (fv[1][a] - fv[0][a]) + t * (fv[2][a] - fv[3][a]);
                xt[a] = (1 - s_) * (fv[3][a] - fv[0][a]) + s_ * (fv[2][a] - fv[1][a]);
            }
            cross3(xs, xt, nrm);
            const double len = sqrt(dot3(nrm, nrm));
            for (int a = 0; a < 3; ++a) gn[g][a] = nrm[a] / len;
            gw[g] = 0.25 * len;
        }
    return 4;
}

/*
 * Builds the oracle mesh.  npc = 4 (tetrahedra) or 8 (hexahedra).  nbf boundary
 * faces (bface_nodes [nbf][3 or 4], any order) with kinds ORC_BC_WALL / ORC_BC_FAR;
 * a mesh with listed boundary faces has no periodic axis, and every face that
 * belongs to one cell must then be listed.
 */
orc_mesh *orc_mesh_new2(int64_t nn, const double *xyz, int64_t nc, int npc, const int64_t *cell_nodes,
                        const double *period, int64_t nbf, const int64_t *bface_nodes, const int *bface_kind,
                        char *err, int errlen) {
    if (nn <= 0 || nc <= 0 || !xyz || !cell_nodes || (npc != 4 && npc != 8)) { set_err(err, errlen, "empty mesh or bad cell type"); return NULL; }
    const int nfc = npc == 4 ? 4 : 6, nk = npc == 4 ? 3 : 4;
    if (nbf > 0) {
        if (!bface_nodes || !bface_kind) { set_err(err, errlen, "boundary faces without nodes or kinds"); return NULL; }
        for (int a = 0; a < 3; ++a)
            if (period && period[a] > 0.0) { set_err(err, errlen, "listed boundary faces need a mesh without periodic axes"); return NULL; }
        for (int64_t k = 0; k < nbf; ++k)
            if (bface_kind[k] != ORC_BC_WALL && bface_kind[k] != ORC_BC_FAR) { set_err(err, errlen, "unknown boundary kind"); return NULL; }
    }
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->nc = nc; m->nn = nn;
    m->npc = npc; m->nfc = nfc; m->ngp = npc == 4 ? 3 : 4; m->msub = npc == 4 ? 4 : 8;
    for (int a = 0; a < 3; ++a) m->period[a] = period ? period[a] : 0.0;
    m->vert = calloc((size_t)nc, sizeof(*m->vert));
    m->vol = malloc(sizeof(double) * nc);
    m->cen = malloc(sizeof(*m->cen) * nc);
    m->h = malloc(sizeof(double) * nc);
    m->hdt = malloc(sizeof(double) * nc);
    m->cface = malloc(sizeof(*m->cface) * nc);
    m->nb = malloc(sizeof(*m->nb) * nc);
    m->nbx = malloc(sizeof(*m->nbx) * nc);
    for (int a = 0; a < 3; ++a) { m->lo[a] = INFINITY; m->hi[a] = -INFINITY; }
    for (int64_t k = 0; k < nn; ++k)
        for (int a = 0; a < 3; ++a) { m->lo[a] = fmin(m->lo[a], xyz[3 * k + a]); m->hi[a] = fmax(m->hi[a], xyz[3 * k + a]); }

    /* unwrap every cell around its first node; volume, centroid */
    for (int64_t c = 0; c < nc; ++c) {
        for (int q = 0; q < npc; ++q) {
            int64_t nid = cell_nodes[c * npc + q];
            if (nid < 0 || nid >= nn) { set_err(err, errlen, "node id out of range"); orc_mesh_free(m); return NULL; }
        }
        const double *x0 = xyz + 3 * cell_nodes[c * npc];
        for (int q = 0; q < npc; ++q) {
            const double *xq = xyz + 3 * cell_nodes[c * npc + q];
            for (int a = 0; a < 3; ++a) {
                double d = xq[a] - x0[a];
                if (m->period[a] > 0.0) d -= m->period[a] * nearbyint(d / m->period[a]);
                m->vert[c][q][a] = x0[a] + d;
            }
        }
        double ext = 0.0;
        for (int q = 1; q < npc; ++q)
            for (int a = 0; a < 3; ++a) ext = fmax(ext, fabs(m->vert[c][q][a] - m->vert[c][0][a]));
        if (npc == 4) {
            double e1[3], e2[3], e3[3], cr[3];
            sub3(m->vert[c][1], m->vert[c][0], e1);
            sub3(m->vert[c][2], m->vert[c][0], e2);
            sub3(m->vert[c][3], m->vert[c][0], e3);
            cross3(e2, e3, cr);
            double v = fabs(dot3(e1, cr)) / 6.0;
            ext = 0.0;
            for (int a = 0; a < 3; ++a) ext = fmax(ext, fabs(e1[a]) + fabs(e2[a]) + fabs(e3[a]));
            if (!(v > 1e-12 * ext * ext * ext)) { set_err(err, errlen, "degenerate tetrahedron"); orc_mesh_free(m); return NULL; }
            m->vol[c] = v;
            for (int a = 0; a < 3; ++a)
                m->cen[c][a] = 0.25 * (m->vert[c][0][a] + m->vert[c][1][a] + m->vert[c][2][a] + m->vert[c][3][a]);
        } else {
            double pts[MAXCQ][3], wts[MAXCQ], jlo, jhi;
            const int n = cell_quadrature(npc, m->vert[c], pts, wts, &jlo, &jhi);
            /* the trilinear map must not fold: one Jacobian sign at every point */
            if (!(jlo * jhi > 0.0) || !(fmin(fabs(jlo), fabs(jhi)) > 1e-12 * ext * ext * ext)) {
                set_err(err, errlen, "degenerate or folded hexahedron"); orc_mesh_free(m); return NULL;
            }
            double V = 0.0, cx[3] = {0, 0, 0};
            for (int q = 0; q < n; ++q) {
                V += wts[q];
                for (int a = 0; a < 3; ++a) cx[a] += wts[q] * pts[q][a];
            }
            m->vol[c] = V;
            for (int a = 0; a < 3; ++a) m->cen[c][a] = cx[a] / V;
        }
        m->h[c] = cbrt(m->vol[c]);
    }

    /* listed boundary faces, sorted by key for lookup */
    int64_t (*bkey)[4] = NULL;
    int *bkind = NULL;
    int64_t *border = NULL;
    if (nbf > 0) {
        bkey = malloc(sizeof(*bkey) * nbf);
        bkind = malloc(sizeof(int) * nbf);
        face_rec *br = malloc(sizeof(face_rec) * nbf);
        for (int64_t k = 0; k < nbf; ++k) {
            face_key(bface_nodes + k * nk, nk, br[k].key);
            br[k].cell = k; br[k].p = 0;
        }
        qsort(br, (size_t)nbf, sizeof(face_rec), cmp_face);
        border = malloc(sizeof(int64_t) * nbf);
        for (int64_t k = 0; k < nbf; ++k) { memcpy(bkey[k], br[k].key, sizeof(bkey[k])); bkind[k] = bface_kind[br[k].cell]; border[k] = br[k].cell; }
        free(br);
    }

    /* faces: match the node sets of all cell faces (CellFace / FaceCell) */
    face_rec *fr = malloc(sizeof(face_rec) * nc * nfc);
    for (int64_t c = 0; c < nc; ++c)
        for (int p = 0; p < nfc; ++p) {
            face_rec *r = &fr[c * nfc + p];
            int64_t nodes[4];
            for (int k = 0; k < nk; ++k) nodes[k] = cell_nodes[c * npc + face_node(npc, p, k)];
            face_key(nodes, nk, r->key);
            r->cell = c; r->p = p;
        }
    const int64_t nrec = nc * nfc;
    qsort(fr, (size_t)nrec, sizeof(face_rec), cmp_face);
    int64_t nf = 0;
    for (int64_t k = 0; k < nrec;) {
        int64_t j = k + 1;
        while (j < nrec && cmp_key(fr[j].key, fr[k].key) == 0) ++j;
        if (j - k > 2) { set_err(err, errlen, "non-conforming face"); free(fr); free(bkey); free(bkind); free(border); orc_mesh_free(m); return NULL; }
        ++nf; k = j;
    }
    m->nf = nf;
    m->fcell = malloc(sizeof(*m->fcell) * nf);
    m->fkind = calloc((size_t)nf, sizeof(int));
    m->fshift = malloc(sizeof(*m->fshift) * nf);
    m->fnrm = malloc(sizeof(*m->fnrm) * nf);
    m->farea = malloc(sizeof(double) * nf);
    m->fgp = calloc((size_t)nf, sizeof(*m->fgp));
    m->fpn = calloc((size_t)nf, sizeof(*m->fpn));
    m->fpw = calloc((size_t)nf, sizeof(*m->fpw));
    m->gcell = malloc(sizeof(int64_t) * (nbf > 0 ? nbf : 1));
    m->gface = malloc(sizeof(int64_t) * (nbf > 0 ? nbf : 1));
    m->gkind = malloc(sizeof(int) * (nbf > 0 ? nbf : 1));
    m->gpt = malloc(sizeof(*m->gpt) * (nbf > 0 ? nbf : 1));
    m->gnrm = malloc(sizeof(*m->gnrm) * (nbf > 0 ? nbf : 1));
    m->ng = 0;
    unsigned char *bused = nbf > 0 ? calloc((size_t)nbf, 1) : NULL;
    double *asum = calloc((size_t)nc, sizeof(double));
    int64_t f = 0;
    const char *fail = NULL;
    for (int64_t k = 0; k < nrec && !fail; ++f) {
        const int single = k + 1 >= nrec || cmp_key(fr[k + 1].key, fr[k].key) != 0;
        const face_rec *A = &fr[k], *B = single ? NULL : &fr[k + 1];     /* A->cell <= B->cell */
        k += single ? 1 : 2;
        int64_t l = A->cell;
        int pl = A->p;
        m->fcell[f][0] = l;
        m->cface[l][pl] = f;
        /* face vertices in the left frame, cyclic order */
        double fv[4][3];
        for (int q = 0; q < nk; ++q) memcpy(fv[q], m->vert[l][face_node(npc, pl, q)], sizeof(fv[q]));
        double gw[MAXGP];
        const int ng = face_points(nk, fv, m->fgp[f], m->fpn[f], gw);
        /* orient out of the left cell: the weighted normals give the vector area */
        double va[3] = {0, 0, 0}, fc[3] = {0, 0, 0}, area = 0.0;
        for (int g = 0; g < ng; ++g) {
            area += gw[g];
            for (int a = 0; a < 3; ++a) { va[a] += gw[g] * m->fpn[f][g][a]; fc[a] += m->fgp[f][g][a] / ng; }
        }
        double d[3];
        sub3(fc, m->cen[l], d);
        const double sg = dot3(va, d) < 0.0 ? -1.0 : 1.0;
        const double vlen = sqrt(dot3(va, va));
        for (int a = 0; a < 3; ++a) m->fnrm[f][a] = npc == 4 ? sg * m->fpn[f][0][a] : sg * va[a] / vlen;
        for (int g = 0; g < ng; ++g) {
            for (int a = 0; a < 3; ++a) m->fpn[f][g][a] *= sg;
            m->fpw[f][g] = gw[g];
        }
        m->farea[f] = area;
        if (npc == 4) {   /* the triangle's area, as 0.5 |e1 x e2| */
            double e1[3], e2[3], nrm[3];
            sub3(fv[1], fv[0], e1);
            sub3(fv[2], fv[0], e2);
            cross3(e1, e2, nrm);
            m->farea[f] = 0.5 * sqrt(dot3(nrm, nrm));
        }
        asum[l] += m->farea[f];
        if (single) {
            m->fcell[f][1] = -1;
            for (int a = 0; a < 3; ++a) m->fshift[f][a] = 0.0;
            if (nbf > 0) {
                /* a listed boundary face: a ghost of the given kind */
                int64_t lo_ = 0, hi_ = nbf - 1, at = -1;
                while (lo_ <= hi_) {
                    int64_t mid = (lo_ + hi_) / 2;
                    int c = cmp_key(bkey[mid], A->key);
                    if (c == 0) { at = mid; break; }
                    if (c < 0) lo_ = mid + 1; else hi_ = mid - 1;
                }
                if (at < 0) { fail = "a face of one cell is not in the boundary-face list"; break; }
                bused[at] = 1;
                const int64_t g = m->ng++;
                m->fkind[f] = bkind[at];
                m->gcell[g] = l; m->gface[g] = f; m->gkind[g] = bkind[at];
                memcpy(m->gnrm[g], m->fnrm[f], sizeof(m->gnrm[g]));
                for (int a = 0; a < 3; ++a) m->gpt[g][a] = fc[a];
                m->nb[l][pl] = nc + g;
                m->nbx[l][pl] = XID;
                continue;
            }
            /* a wall of a non-periodic axis: all nodes on the lowest or highest coordinate */
            int axis = -1;
            double w = 0.0;
            for (int a = 0; a < 3 && axis < 0; ++a) {
                if (m->period[a] > 0.0) continue;
                const double x0 = xyz[3 * A->key[0] + a];
                int on = x0 == m->lo[a] || x0 == m->hi[a];
                for (int q = 1; q < nk; ++q) on = on && xyz[3 * A->key[q] + a] == x0;
                if (on) { axis = a; w = x0; }
            }
            if (axis < 0) {
                fail = "boundary face off the walls (an unmatched face must lie on the lowest or highest "
                       "coordinate of a non-periodic axis)";
                break;
            }
            m->nb[l][pl] = l;
            m->nbx[l][pl] = XID;
            m->nbx[l][pl].s[axis] = -1.0;
            m->nbx[l][pl].o[axis] = 2.0 * w;
            continue;
        }
        int64_t r = B->cell;
        int pr = B->p;
        m->fcell[f][1] = r;
        m->cface[r][pr] = f;
        /* the right cell's image shift in the left frame, from a shared node */
        int64_t n0 = cell_nodes[l * npc + face_node(npc, pl, 0)];
        int ql = -1, qr = -1;
        for (int q = 0; q < npc; ++q) { if (cell_nodes[l * npc + q] == n0) ql = q; if (cell_nodes[r * npc + q] == n0) qr = q; }
        sub3(m->vert[l][ql], m->vert[r][qr], m->fshift[f]);
        asum[r] += m->farea[f];
        m->nb[l][pl] = r;
        m->nb[r][pr] = l;
        m->nbx[l][pl] = XID;
        m->nbx[r][pr] = XID;
        for (int a = 0; a < 3; ++a) { m->nbx[l][pl].o[a] = m->fshift[f][a]; m->nbx[r][pr].o[a] = -m->fshift[f][a]; }
    }
    if (!fail)
        for (int64_t k = 0; k < nbf; ++k)
            if (!bused[k]) { fail = "a listed boundary face is not a face of exactly one cell"; break; }
    free(fr); free(bkey); free(bkind); free(border); free(bused);
    if (fail) { set_err(err, errlen, fail); free(asum); orc_mesh_free(m); return NULL; }
    for (int64_t c = 0; c < nc; ++c) m->hdt[c] = 6.0 * m->vol[c] / asum[c];
    free(asum);

    /* two-layer stencil (Algorithm 1, self excluded) and the sub-stencils (Sec. 2.3).
     * A ghost of a listed boundary face is a member but has no neighbours. */
    m->nsten = malloc(sizeof(int) * nc);
    m->sten = malloc(sizeof(*m->sten) * nc);
    m->stx = malloc(sizeof(*m->stx) * nc);
    m->nsub = calloc((size_t)nc, sizeof(*m->nsub));
    m->sub = malloc(sizeof(*m->sub) * nc);
    m->subx = malloc(sizeof(*m->subx) * nc);
    for (int64_t i = 0; i < nc; ++i) {
        /* a neighbour's neighbours are placed by composing the two placements */
        int n = 0;
        for (int p = 0; p < nfc; ++p) {
            int dup = same_member(m->nb[i][p], &m->nbx[i][p], i, &XID);
            for (int k = 0; k < n; ++k) dup |= same_member(m->sten[i][k], &m->stx[i][k], m->nb[i][p], &m->nbx[i][p]);
            if (!dup) { m->sten[i][n] = m->nb[i][p]; m->stx[i][n] = m->nbx[i][p]; ++n; }
        }
        for (int p = 0; p < nfc; ++p) {
            int64_t j = m->nb[i][p];
            if (j >= nc) continue;                           /* a ghost: no neighbours */
            for (int q = 0; q < nfc; ++q) {
                int64_t c = m->nb[j][q];
                xform x = compose(&m->nbx[i][p], &m->nbx[j][q]);
                int dup = same_member(c, &x, i, &XID);
                for (int k = 0; k < n; ++k) dup |= same_member(m->sten[i][k], &m->stx[i][k], c, &x);
                if (!dup) {
                    if (n >= MAXSTEN) { set_err(err, errlen, "stencil too large"); orc_mesh_free(m); return NULL; }
                    m->sten[i][n] = c; m->stx[i][n] = x; ++n;
                }
            }
        }
        m->nsten[i] = n;
        for (int s_ = 0; s_ < m->msub; ++s_) {
            int k = 0;
            for (int t = 0; t < 3; ++t) {
                int p = npc == 4 ? TETSUB[s_][t] : HEXSUB[s_][t];
                int dup = 0;
                for (int u = 0; u < k; ++u) dup |= same_member(m->sub[i][s_][u], &m->subx[i][s_][u], m->nb[i][p], &m->nbx[i][p]);
                if (!dup) { m->sub[i][s_][k] = m->nb[i][p]; m->subx[i][s_][k] = m->nbx[i][p]; ++k; }
            }
            if (npc == 4 && m->nb[i][s_] < nc) {             /* tet: add N(i_m) */
                int64_t j = m->nb[i][s_];
                for (int q = 0; q < 4; ++q) {
                    int64_t c = m->nb[j][q];
                    xform x = compose(&m->nbx[i][s_], &m->nbx[j][q]);
                    int dup = same_member(c, &x, i, &XID);
                    for (int u = 0; u < k; ++u) dup |= same_member(m->sub[i][s_][u], &m->subx[i][s_][u], c, &x);
                    if (!dup) { m->sub[i][s_][k] = c; m->subx[i][s_][k] = x; ++k; }
                }
            }
            m->nsub[i][s_] = k;
        }
    }
    return m;
}

orc_mesh *orc_mesh_new(int64_t nn, const double *xyz, int64_t nc, const int64_t *cell_nodes,
                       const double *period, char *err, int errlen) {
    return orc_mesh_new2(nn, xyz, nc, 4, cell_nodes, period, 0, NULL, NULL, err, errlen);
}

void orc_mesh_free(orc_mesh *m) {
    if (!m) return;
    free(m->vert); free(m->vol); free(m->cen); free(m->h); free(m->hdt);
    free(m->fcell); free(m->fkind); free(m->fshift); free(m->fnrm); free(m->farea); free(m->fgp);
    free(m->fpn); free(m->fpw);
    free(m->cface); free(m->nb); free(m->nbx);
    free(m->gcell); free(m->gface); free(m->gkind); free(m->gpt); free(m->gnrm);
    free(m->nsten); free(m->sten); free(m->stx); free(m->nsub); free(m->sub); free(m->subx);
    free(m);
}

/* accessors for tests */
int64_t orc_mesh_nfaces(const orc_mesh *m) { return m->nf; }
/* info [6]: nodes per cell, faces per cell, Gauss points per face, sub-stencils, ghosts, max stencil size */
void orc_mesh_info(const orc_mesh *m, int64_t *info) {
    int64_t mx = 0;
    for (int64_t i = 0; i < m->nc; ++i) if (m->nsten[i] > mx) mx = m->nsten[i];
    info[0] = m->npc; info[1] = m->nfc; info[2] = m->ngp; info[3] = m->msub; info[4] = m->ng; info[5] = mx;
}
void orc_mesh_cells(const orc_mesh *m, double *vol, double *cen, double *hdt) {
    for (int64_t c = 0; c < m->nc; ++c) {
        if (vol) vol[c] = m->vol[c];
        if (cen) memcpy(cen + 3 * c, m->cen[c], sizeof(double) * 3);
        if (hdt) hdt[c] = m->hdt[c];
    }
}
/* gp [nf][ngp][3] */
void orc_mesh_faces(const orc_mesh *m, int64_t *lr, double *nrm, double *area, double *shift, double *gp) {
    for (int64_t f = 0; f < m->nf; ++f) {
        if (lr) { lr[2 * f] = m->fcell[f][0]; lr[2 * f + 1] = m->fcell[f][1]; }
        if (nrm) memcpy(nrm + 3 * f, m->fnrm[f], sizeof(double) * 3);
        if (area) area[f] = m->farea[f];
        if (shift) memcpy(shift + 3 * f, m->fshift[f], sizeof(double) * 3);
        if (gp) for (int g = 0; g < m->ngp; ++g) memcpy(gp + 3 * (m->ngp * f + g), m->fgp[f][g], sizeof(double) * 3);
    }
}
/* per Gauss point unit normals pn [nf][ngp][3] and weights pw [nf][ngp]; kind [nf] */
void orc_mesh_face_points(const orc_mesh *m, double *pn, double *pw, int *kind) {
    for (int64_t f = 0; f < m->nf; ++f) {
        for (int g = 0; g < m->ngp; ++g) {
            if (pn) memcpy(pn + 3 * (m->ngp * f + g), m->fpn[f][g], sizeof(double) * 3);
            if (pw) pw[m->ngp * f + g] = m->fpw[f][g];
        }
        if (kind) kind[f] = m->fkind[f];
    }
}
/* stencil of cell i: returns K; members[K] (ids >= nc are ghosts), shifts[K][3];
 * sub-stencil sizes[msub], members[msub][MAXSUB] */
int orc_mesh_stencil(const orc_mesh *m, int64_t i, int64_t *members, double *shifts, int *nsub, int64_t *sub) {
    int n = m->nsten[i];
    for (int k = 0; k < n; ++k) {
        if (members) members[k] = m->sten[i][k];
        if (shifts) memcpy(shifts + 3 * k, m->stx[i][k].o, sizeof(double) * 3);   /* offsets (s = 1 unless mirrored) */
    }
    for (int s = 0; s < m->msub; ++s) {
        if (nsub) nsub[s] = m->nsub[i][s];
        if (sub) for (int k = 0; k < MAXSUB; ++k) sub[s * MAXSUB + k] = k < m->nsub[i][s] ? m->sub[i][s][k] : -1;
    }
    return n;
}
/* nb [nc][nfc] */
void orc_mesh_neighbors(const orc_mesh *m, int64_t *nb) {
    for (int64_t c = 0; c < m->nc; ++c) for (int p = 0; p < m->nfc; ++p) nb[m->nfc * c + p] = m->nb[c][p];
}

/* ------------------------------------------------------------------------- */
/* ghosts of listed boundary faces (Sec. 5.2)                                */
/* ------------------------------------------------------------------------- */

typedef struct { double rho, U, V, W, lam, p; } prim;

static prim primitives(const double *q, double gamma) {
    prim s;
    s.rho = q[0];
    s.U = q[1] / q[0]; s.V = q[2] / q[0]; s.W = q[3] / q[0];
    s.p = (gamma - 1.0) * (q[4] - 0.5 * s.rho * (s.U * s.U + s.V * s.V + s.W * s.W));
    s.lam = s.rho / (2.0 * s.p);
    return s;
}

static void conservative(double rho, const double *U, double pr, double gamma, double *q) {
    q[0] = rho;
    for (int a = 0; a < 3; ++a) q[1 + a] = rho * U[a];
    q[4] = pr / (gamma - 1.0) + 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
}

/*
 * Far-field state by Riemann invariants (characteristic boundary): with the outward
 * normal n, interior state q and free stream (rho, U, p)_inf,
 *   R+ = U.n + 2c/(gamma-1) from the interior, R- = U_inf.n - 2c_inf/(gamma-1) from
 *   outside; the boundary normal velocity (R+ + R-)/2 and sound speed
 *   (gamma-1)(R+ - R-)/4; entropy p/rho^gamma and tangential velocity from the
 *   interior at an outflow, from the free stream at an inflow.  A supersonic outflow
 *   takes the interior state, a supersonic inflow the free stream.
 */
static void farfield_state(const orc_params *p, const double *q, const double *n, double *out) {
    const double g = p->gamma;
    const prim si = primitives(q, g);
    const double Ui[3] = {si.U, si.V, si.W};
    const double *Uf = p->farfield + 1;
    const double rf = p->farfield[0], pf = p->farfield[4];
    const double ci = sqrt(g * si.p / si.rho), cf = sqrt(g * pf / rf);
    const double vi = dot3(Ui, n), vf = dot3(Uf, n);
    if (vi >= ci) { memcpy(out, q, sizeof(double) * 5); return; }
    if (vi <= -ci) { conservative(rf, Uf, pf, g, out); return; }
    const double Rp = vi + 2.0 * ci / (g - 1.0), Rm = vf - 2.0 * cf / (g - 1.0);
    const double vb = 0.5 * (Rp + Rm), cb = 0.25 * (g - 1.0) * (Rp - Rm);
    const int outflow = vb > 0.0;
    const double ent = outflow ? si.p / pow(si.rho, g) : pf / pow(rf, g);
    const double *Ut = outflow ? Ui : Uf;
    const double vt = outflow ? vi : vf;
    const double rb = pow(cb * cb / (g * ent), 1.0 / (g - 1.0));
    const double pb = rb * cb * cb / g;
    double Ub[3];
    for (int a = 0; a < 3; ++a) Ub[a] = Ut[a] - vt * n[a] + vb * n[a];
    conservative(rb, Ub, pb, g, out);
}

/* the state a boundary-face ghost holds for the adjacent state q */
static void ghost_state(const orc_params *p, int kind, const double *q, const double *n, double *out) {
    if (kind == ORC_BC_WALL) {                       /* zero velocity on the face, same temperature */
        out[0] = q[0]; out[1] = -q[1]; out[2] = -q[2]; out[3] = -q[3]; out[4] = q[4];
    } else {
        farfield_state(p, q, n, out);
    }
}

/* state of a stencil member (a cell or a ghost) */
static void member_state(const orc_mesh *m, const orc_params *p, const double *Q, int64_t id, double *out) {
    if (id < m->nc) { memcpy(out, Q + 5 * id, sizeof(double) * 5); return; }
    const int64_t g = id - m->nc;
    ghost_state(p, m->gkind[g], Q + 5 * m->gcell[g], m->gnrm[g], out);
}

/* ------------------------------------------------------------------------- */
/* WENO reconstruction (Sec. 2.3)                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    double a[5][9];          /* P0 coefficients, per variable */
    double b[MAXM][5][3];    /* P_m coefficients (linear), per sub-stencil and variable */
    double beta[5][MAXM + 1];   /* [variable][m], m = 0..M */
    double wbar[5][MAXM + 1];   /* normalised non-linear weights [variable][m] */
    double mean_i[9];        /* mean over the cell of xi^d */
} orc_weno;

/* A member's vertices placed in the target cell's frame: a periodic image or axis
 * mirror of a cell, or a boundary ghost (the cell's mirror image in the face plane). */
static void member_vertices(const orc_mesh *m, int64_t k, const xform *x, double v[8][3]) {
    if (k >= m->nc) {
        const int64_t g = k - m->nc;
        const double *pt = m->gpt[g], *n = m->gnrm[g];
        for (int q = 0; q < m->npc; ++q) {
            const double *y = m->vert[m->gcell[g]][q];
            const double d = (y[0] - pt[0]) * n[0] + (y[1] - pt[1]) * n[1] + (y[2] - pt[2]) * n[2];
            for (int a = 0; a < 3; ++a) v[q][a] = y[a] - 2.0 * d * n[a];
        }
        return;
    }
    for (int q = 0; q < m->npc; ++q) for (int a = 0; a < 3; ++a) v[q][a] = x->s[a] * m->vert[k][q][a] + x->o[a];
}

static int weno_cell(const orc_mesh *m, const orc_params *p, const double *Q, int64_t i, orc_weno *w) {
    const double *ci = m->cen[i];
    const double hi = m->h[i];
    const int M = m->msub;
    cell_monomial_means(m->npc, m->vert[i], ci, hi, w->mean_i);
    /* quadratic P0 on the big stencil: constraints (1/|Omega_k|) int_{Omega_k} P0 = Q_k */
    int K = m->nsten[i];
    double A[MAXSTEN * 9], B[MAXSTEN * 5];
    for (int k = 0; k < K; ++k) {
        double v[8][3], mk[9], qk[5];
        member_vertices(m, m->sten[i][k], &m->stx[i][k], v);
        cell_monomial_means(m->npc, v, ci, hi, mk);
        member_state(m, p, Q, m->sten[i][k], qk);
        for (int d = 0; d < 9; ++d) A[k * 9 + d] = mk[d] - w->mean_i[d];
        for (int q = 0; q < 5; ++q) B[k * 5 + q] = qk[q] - Q[5 * i + q];
    }
    double X[9 * 5];
    if (lsq_normal(K, 9, A, 5, B, X)) return ORC_E_MESH;
    for (int d = 0; d < 9; ++d) for (int q = 0; q < 5; ++q) w->a[q][d] = X[d * 5 + q];
    /* linear P_m on the sub-stencils */
    for (int s = 0; s < M; ++s) {
        int n = m->nsub[i][s];
        double As[MAXSUB * 3], Bs[MAXSUB * 5], Xs[3 * 5];
        for (int k = 0; k < n; ++k) {
            double v[8][3], mk[9], qk[5];
            member_vertices(m, m->sub[i][s][k], &m->subx[i][s][k], v);
            cell_monomial_means(m->npc, v, ci, hi, mk);
            member_state(m, p, Q, m->sub[i][s][k], qk);
            for (int d = 0; d < 3; ++d) As[k * 3 + d] = mk[d] - w->mean_i[d];
            for (int q = 0; q < 5; ++q) Bs[k * 5 + q] = qk[q] - Q[5 * i + q];
        }
        if (lsq_normal(n, 3, As, 5, Bs, Xs)) return ORC_E_MESH;
        for (int d = 0; d < 3; ++d) for (int q = 0; q < 5; ++q) w->b[s][q][d] = Xs[d * 5 + q];
    }
    /* smoothness indicators: beta_m = sum_{1<=|l|<=r_m} |Omega|^(2|l|/3-1) int (d^l P_m)^2 dV,
     * evaluated in physical coordinates with the cell rule (exact for these integrands) */
    double pts[MAXCQ][3], wts[MAXCQ];
    const int nq = cell_quadrature(m->npc, m->vert[i], pts, wts, NULL, NULL);
    const double V = m->vol[i];
    const double w1 = pow(V, 2.0 / 3.0 - 1.0), w2 = pow(V, 4.0 / 3.0 - 1.0);
    static const int L2IDX[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int q = 0; q < 5; ++q) {
        for (int s = 0; s <= M; ++s) {
            int nd = s == 0 ? 9 : 3;
            const double *c = s == 0 ? w->a[q] : w->b[s - 1][q];
            double beta = 0.0;
            for (int j = 0; j < 3; ++j) {               /* |l| = 1 */
                double integral = 0.0;
                for (int g = 0; g < nq; ++g) {
                    double xi[3] = {(pts[g][0] - ci[0]) / hi, (pts[g][1] - ci[1]) / hi, (pts[g][2] - ci[2]) / hi};
                    double dp = 0.0;
                    for (int d = 0; d < nd; ++d) dp += c[d] * dmono(DEXP[d], j, xi) / hi;
                    integral += (m->npc == 4 ? 0.25 * V : wts[g]) * dp * dp;
                }
                beta += w1 * integral;
            }
            if (s == 0) {                                 /* |l| = 2, each multi-index once */
                for (int t = 0; t < 6; ++t) {
                    double xi0[3] = {0, 0, 0};
                    double d2 = 0.0;
                    for (int d = 0; d < 9; ++d) d2 += c[d] * d2mono(DEXP[d], L2IDX[t][0], L2IDX[t][1], xi0) / (hi * hi);
                    beta += w2 * V * d2 * d2;
                }
            }
            w->beta[q][s] = beta;
        }
        /* WENO-Z non-linear weights, gamma_0 = 1 - M gamma */
        double g[MAXM + 1];
        g[0] = 1.0 - (double)M * p->gamma_lin;
        for (int s = 1; s <= M; ++s) g[s] = p->gamma_lin;
        double tauZ = 0.0;
        for (int s = 1; s <= M; ++s) tauZ += fabs(w->beta[q][0] - w->beta[q][s]) / (double)M;
        double om[MAXM + 1], sum = 0.0;
        for (int s = 0; s <= M; ++s) { om[s] = g[s] * (1.0 + tauZ / (w->beta[q][s] + p->weno_eps)); sum += om[s]; }
        for (int s = 0; s <= M; ++s) w->wbar[q][s] = om[s] / sum;
    }
    return ORC_OK;
}

/* Point value and gradient of the WENO combination (Eq. weno) at x (cell i's frame). */
static void weno_eval(const orc_mesh *m, const orc_params *p, const double *Q, int64_t i, const orc_weno *w,
                      const double *x, double *val, double grad[5][3]) {
    const double hi = m->h[i];
    const int M = m->msub;
    double xi[3] = {(x[0] - m->cen[i][0]) / hi, (x[1] - m->cen[i][1]) / hi, (x[2] - m->cen[i][2]) / hi};
    const double g0 = 1.0 - (double)M * p->gamma_lin, gm = p->gamma_lin;
    for (int q = 0; q < 5; ++q) {
        double P[MAXM + 1], dP[MAXM + 1][3];
        for (int s = 0; s <= M; ++s) {
            int nd = s == 0 ? 9 : 3;
            const double *c = s == 0 ? w->a[q] : w->b[s - 1][q];
            double v = Q[5 * i + q];
            for (int d = 0; d < nd; ++d) v += c[d] * (mono(DEXP[d], xi) - w->mean_i[d]);
            P[s] = v;
            for (int j = 0; j < 3; ++j) {
                double t = 0.0;
                for (int d = 0; d < nd; ++d) t += c[d] * dmono(DEXP[d], j, xi) / hi;
                dP[s][j] = t;
            }
        }
        double v = w->wbar[q][0] * P[0] / g0;
        for (int s = 1; s <= M; ++s) v += -w->wbar[q][0] * gm / g0 * P[s] + w->wbar[q][s] * P[s];
        val[q] = v;
        for (int j = 0; j < 3; ++j) {
            double t = w->wbar[q][0] * dP[0][j] / g0;
            for (int s = 1; s <= M; ++s) t += -w->wbar[q][0] * gm / g0 * dP[s][j] + w->wbar[q][s] * dP[s][j];
            grad[q][j] = t;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Maxwellian moments (Sec. 2.1)                                             */
/* ------------------------------------------------------------------------- */

/* A polynomial in (u, v, w, xi^2): sum of c * u^a v^b w^c (xi^2)^d. */
typedef struct { double c; int e[4]; } term;
typedef struct { int n; term t[16]; } poly;

static poly PSI[5];            /* collision invariants psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2) */
static poly P_PP[5][5];        /* psi_a psi_b */
static poly P_UPP[3][5][5];    /* u_j psi_a psi_b */
static poly P_UUPP[3][5][5];   /* u u_j psi_a psi_b */
static poly P_UP[5];           /* u psi_a */
static int tables_ready = 0;

static poly pmul(const poly *x, const poly *y) {
    poly r; r.n = 0;
    for (int i = 0; i < x->n; ++i)
        for (int j = 0; j < y->n; ++j) {
            term t;
            t.c = x->t[i].c * y->t[j].c;
            for (int k = 0; k < 4; ++k) t.e[k] = x->t[i].e[k] + y->t[j].e[k];
            r.t[r.n++] = t;
        }
    return r;
}

static poly pvar(int k) { poly r; r.n = 1; r.t[0].c = 1.0; memset(r.t[0].e, 0, sizeof(r.t[0].e)); if (k >= 0) r.t[0].e[k] = 1; return r; }

static void build_tables(void) {
    if (tables_ready) return;
    PSI[0] = pvar(-1);
    PSI[1] = pvar(0);
    PSI[2] = pvar(1);
    PSI[3] = pvar(2);
    PSI[4].n = 4;
    for (int k = 0; k < 4; ++k) {
        PSI[4].t[k].c = 0.5;
        memset(PSI[4].t[k].e, 0, sizeof(PSI[4].t[k].e));
        if (k < 3) PSI[4].t[k].e[k] = 2; else PSI[4].t[k].e[3] = 1;
    }
    poly U = pvar(0);
    for (int a = 0; a < 5; ++a) {
        P_UP[a] = pmul(&U, &PSI[a]);
        for (int b = 0; b < 5; ++b) {
            P_PP[a][b] = pmul(&PSI[a], &PSI[b]);
            for (int j = 0; j < 3; ++j) {
                poly uj = pvar(j);
                P_UPP[j][a][b] = pmul(&uj, &P_PP[a][b]);
                poly uuj = pmul(&U, &uj);
                P_UUPP[j][a][b] = pmul(&uuj, &P_PP[a][b]);
            }
        }
    }
    tables_ready = 1;
}

/* Normalised moments <u^n>, <v^n>, <w^n>, <xi^(2n)> of one Maxwellian;
 * half = +1 / -1 selects the half space u > 0 / u < 0 for the u-moments. */
typedef struct { double mu[7], mv[7], mw[7], mxi[3]; } moments;

static void full_moments_1d(double U, double lam, double *m) {
    m[0] = 1.0;
    m[1] = U;
    for (int n = 2; n < 7; ++n) m[n] = U * m[n - 1] + (double)(n - 1) / (2.0 * lam) * m[n - 2];
}

static void half_moments_1d(double U, double lam, int half, double *m) {
    double s = sqrt(lam) * U;
    double g = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    if (half > 0) { m[0] = 0.5 * erfc(-s); m[1] = U * m[0] + g; }
    else          { m[0] = 0.5 * erfc(s);  m[1] = U * m[0] - g; }
    for (int n = 2; n < 7; ++n) m[n] = U * m[n - 1] + (double)(n - 1) / (2.0 * lam) * m[n - 2];
}

static void make_moments(double U, double V, double W, double lam, double K, int half, moments *M) {
    if (half == 0) full_moments_1d(U, lam, M->mu); else half_moments_1d(U, lam, half, M->mu);
    full_moments_1d(V, lam, M->mv);
    full_moments_1d(W, lam, M->mw);
    M->mxi[0] = 1.0;
    M->mxi[1] = K / (2.0 * lam);
    M->mxi[2] = K * (K + 2.0) / (4.0 * lam * lam);
}

static double expect(const moments *M, const poly *P) {
    double s = 0.0;
    for (int i = 0; i < P->n; ++i) {
        const term *t = &P->t[i];
        s += t->c * M->mu[t->e[0]] * M->mv[t->e[1]] * M->mw[t->e[2]] * M->mxi[t->e[3]];
    }
    return s;
}

/* The 5x5 moment matrix <psi psi^T> of one state. */
static void moment_matrix(const moments *M, double *A) {
    for (int r = 0; r < 5; ++r) for (int c = 0; c < 5; ++c) A[r * 5 + c] = expect(M, &P_PP[r][c]);
}

/* Solve <(a.psi) psi> = b for the micro-slope a (5x5 moment system, dense elimination). */
static int slope_solve(const moments *M, const double *b, double *a) {
    double A[25];
    moment_matrix(M, A);
    return gauss_solve(5, A, b, a);
}

/* ------------------------------------------------------------------------- */
/* Gas-kinetic flux at one Gauss point (Sec. 2.1, Eq. flux; Sec. 2.2)        */
/* ------------------------------------------------------------------------- */

static void local_frame(const double *n, double *t1, double *t2) {
    int k = 0;
    for (int a = 1; a < 3; ++a) if (fabs(n[a]) < fabs(n[k])) k = a;
    double e[3] = {0, 0, 0};
    e[k] = 1.0;
    cross3(n, e, t1);
    double l = sqrt(dot3(t1, t1));
    for (int a = 0; a < 3; ++a) t1[a] /= l;
    cross3(n, t1, t2);
}

/* rotate the momentum components of a 5-vector into (n, t1, t2) */
static void to_local(const double *q, const double *n, const double *t1, const double *t2, double *out) {
    out[0] = q[0];
    out[1] = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    out[2] = q[1] * t1[0] + q[2] * t1[1] + q[3] * t1[2];
    out[3] = q[1] * t2[0] + q[2] * t2[1] + q[3] * t2[2];
    out[4] = q[4];
}

/*
 * F(t) fitted linearly over [0, dt] (Eq. expansion-1).  Inputs are the
 * reconstructed left/right states at the Gauss point and their gradients in
 * the global frame; outputs are F^n and dF^n/dt per unit area, global frame.
 */
int orc_gks_flux(const orc_params *p, const double *ql, const double *gl /*[5][3]*/,
                 const double *qr, const double *gr, const double *n, double dt,
                 double *F, double *dF) {
    build_tables();
    const double K = (5.0 - 3.0 * p->gamma) / (p->gamma - 1.0);
    double t1[3], t2[3];
    local_frame(n, t1, t2);
    const double *e[3] = {n, t1, t2};
    double Ql[5], Qr[5], dQl[3][5], dQr[3][5];
    to_local(ql, n, t1, t2, Ql);
    to_local(qr, n, t1, t2, Qr);
    for (int j = 0; j < 3; ++j) {               /* derivative along local axis j, then rotate */
        double dl[5], dr[5];
        for (int q = 0; q < 5; ++q) {
            dl[q] = gl[q * 3 + 0] * e[j][0] + gl[q * 3 + 1] * e[j][1] + gl[q * 3 + 2] * e[j][2];
            dr[q] = gr[q * 3 + 0] * e[j][0] + gr[q * 3 + 1] * e[j][1] + gr[q * 3 + 2] * e[j][2];
        }
        to_local(dl, n, t1, t2, dQl[j]);
        to_local(dr, n, t1, t2, dQr[j]);
    }
    prim sl = primitives(Ql, p->gamma), sr = primitives(Qr, p->gamma);
    if (!(sl.rho > 0 && sr.rho > 0 && sl.p > 0 && sr.p > 0)) return ORC_E_NONPHYS;
    moments Ml, Mr, Mlp, Mrn;
    make_moments(sl.U, sl.V, sl.W, sl.lam, K, 0, &Ml);
    make_moments(sr.U, sr.V, sr.W, sr.lam, K, 0, &Mr);
    make_moments(sl.U, sl.V, sl.W, sl.lam, K, +1, &Mlp);
    make_moments(sr.U, sr.V, sr.W, sr.lam, K, -1, &Mrn);
    /* compatibility: Q0 = int_{u>0} psi g_l + int_{u<0} psi g_r */
    double Q0[5];
    for (int a = 0; a < 5; ++a) Q0[a] = sl.rho * expect(&Mlp, &PSI[a]) + sr.rho * expect(&Mrn, &PSI[a]);
    prim s0;
    s0.rho = Q0[0]; s0.U = Q0[1] / Q0[0]; s0.V = Q0[2] / Q0[0]; s0.W = Q0[3] / Q0[0];
    s0.lam = (K + 3.0) * s0.rho / (4.0 * (Q0[4] - 0.5 * s0.rho * (s0.U * s0.U + s0.V * s0.V + s0.W * s0.W)));
    if (!(s0.rho > 0 && s0.lam > 0)) return ORC_E_NONPHYS;
    moments M0;
    make_moments(s0.U, s0.V, s0.W, s0.lam, K, 0, &M0);
    /* spatial micro-slopes: <a^k_j> = dQ_k/dn_j ; <abar_j> = dQ0/dn_j with dQ0 = (dQ_l + dQ_r)/2 */
    double Gl[25], Gr[25], G0[25];
    moment_matrix(&Ml, Gl);
    moment_matrix(&Mr, Gr);
    moment_matrix(&M0, G0);
    double al[3][5], ar[3][5], a0[3][5];
    for (int j = 0; j < 3; ++j) {
        double bl[5], br[5], b0[5];
        for (int q = 0; q < 5; ++q) {
            bl[q] = dQl[j][q] / sl.rho;
            br[q] = dQr[j][q] / sr.rho;
            b0[q] = 0.5 * (dQl[j][q] + dQr[j][q]) / s0.rho;
        }
        if (gauss_solve(5, Gl, bl, al[j]) || gauss_solve(5, Gr, br, ar[j]) || gauss_solve(5, G0, b0, a0[j])) return ORC_E_NONPHYS;
    }
    /* temporal slopes: <a_1 u + a_2 v + a_3 w + A> = 0 (full-space moments of each state) */
    double Al[5], Ar[5], A0[5];
    {
        double bl[5], br[5], b0[5];
        for (int a = 0; a < 5; ++a) {
            double sl_ = 0, sr_ = 0, s0_ = 0;
            for (int j = 0; j < 3; ++j)
                for (int b = 0; b < 5; ++b) {
                    sl_ += al[j][b] * expect(&Ml, &P_UPP[j][b][a]);
                    sr_ += ar[j][b] * expect(&Mr, &P_UPP[j][b][a]);
                    s0_ += a0[j][b] * expect(&M0, &P_UPP[j][b][a]);
                }
            bl[a] = -sl_; br[a] = -sr_; b0[a] = -s0_;
        }
        if (gauss_solve(5, Gl, bl, Al) || gauss_solve(5, Gr, br, Ar) || gauss_solve(5, G0, b0, A0)) return ORC_E_NONPHYS;
    }
    /* collision time */
    double tau = 0.0;
    if (p->tau_mode == 1) tau = p->tau_eps * dt + p->tau_C * fabs(sl.p - sr.p) / (sl.p + sr.p) * dt;
    const double p0 = s0.rho / (2.0 * s0.lam);
    if (p->tau_mode == 2) {
        /* viscous: mu = mu_ref (T0/T_ref)^mu_exp with T = p/rho, tau = mu/p0 + the jump term */
        const double mu = p->mu_ref * pow((p0 / s0.rho) / p->T_ref, p->mu_exp);
        tau = mu / p0 + p->tau_C * fabs(sl.p - sr.p) / (sl.p + sr.p) * dt;
    }
    /* moments of the three pieces of f (Eq. flux) that the time integrals weight:
     * the equilibrium part, and the left/right initial parts on their half spaces */
    double e0[3][5], el[3][5], er[3][5];       /* [0]: <u psi>, [1]: sum_j <u u_j (a_j.psi) psi>, [2]: <u (A.psi) psi> */
    for (int a = 0; a < 5; ++a) {
        e0[0][a] = expect(&M0, &P_UP[a]); el[0][a] = expect(&Mlp, &P_UP[a]); er[0][a] = expect(&Mrn, &P_UP[a]);
        e0[1][a] = el[1][a] = er[1][a] = 0.0;
        e0[2][a] = el[2][a] = er[2][a] = 0.0;
        for (int b = 0; b < 5; ++b) {
            for (int j = 0; j < 3; ++j) {
                e0[1][a] += a0[j][b] * expect(&M0, &P_UUPP[j][b][a]);
                el[1][a] += al[j][b] * expect(&Mlp, &P_UUPP[j][b][a]);
                er[1][a] += ar[j][b] * expect(&Mrn, &P_UUPP[j][b][a]);
            }
            e0[2][a] += A0[b] * expect(&M0, &P_UPP[0][b][a]);
            el[2][a] += Al[b] * expect(&Mlp, &P_UPP[0][b][a]);
            er[2][a] += Ar[b] * expect(&Mrn, &P_UPP[0][b][a]);
        }
    }
    /* for the Prandtl correction: the same three pieces without the factor u, i.e.
     * the conserved moments W = <psi f> of the interface distribution */
    const int prandtl = p->tau_mode == 2 && p->prandtl != 1.0;
    double w0[3][5], wl[3][5], wr[3][5];
    if (prandtl)
        for (int a = 0; a < 5; ++a) {
            w0[0][a] = expect(&M0, &PSI[a]); wl[0][a] = expect(&Mlp, &PSI[a]); wr[0][a] = expect(&Mrn, &PSI[a]);
            w0[1][a] = wl[1][a] = wr[1][a] = 0.0;
            w0[2][a] = wl[2][a] = wr[2][a] = 0.0;
            for (int b = 0; b < 5; ++b) {
                for (int j = 0; j < 3; ++j) {
                    w0[1][a] += a0[j][b] * expect(&M0, &P_UPP[j][b][a]);
                    wl[1][a] += al[j][b] * expect(&Mlp, &P_UPP[j][b][a]);
                    wr[1][a] += ar[j][b] * expect(&Mrn, &P_UPP[j][b][a]);
                }
                w0[2][a] += A0[b] * expect(&M0, &P_PP[b][a]);
                wl[2][a] += Al[b] * expect(&Mlp, &P_PP[b][a]);
                wr[2][a] += Ar[b] * expect(&Mrn, &P_PP[b][a]);
            }
        }
    /* time-integrated flux I(delta) = int_0^delta F(t) dt, for delta = dt and dt/2
     * (and IW, the same integral of W) */
    double I[2][5], IW[2][5];
    for (int h = 0; h < 2; ++h) {
        double d = h == 0 ? dt : 0.5 * dt;
        double q0, q1, q2, q3, q4, q5;
        if (tau == 0.0) { q0 = d; q1 = 0.0; q2 = 0.5 * d * d; q3 = q4 = q5 = 0.0; }
        else {
            double E = exp(-d / tau);
            q0 = d - tau * (1.0 - E);
            q1 = 2.0 * tau * tau - tau * d - tau * (d + 2.0 * tau) * E;
            q2 = 0.5 * d * d - tau * d + tau * tau * (1.0 - E);
            q3 = tau * (1.0 - E);
            q4 = -2.0 * tau * tau + tau * (d + 2.0 * tau) * E;
            q5 = -tau * tau * (1.0 - E);
        }
        for (int a = 0; a < 5; ++a) {
            I[h][a] = s0.rho * (q0 * e0[0][a] + q1 * e0[1][a] + q2 * e0[2][a])
                    + sl.rho * (q3 * el[0][a] + q4 * el[1][a] + q5 * el[2][a])
                    + sr.rho * (q3 * er[0][a] + q4 * er[1][a] + q5 * er[2][a]);
            IW[h][a] = !prandtl ? 0.0
                     : s0.rho * (q0 * w0[0][a] + q1 * w0[1][a] + q2 * w0[2][a])
                     + sl.rho * (q3 * wl[0][a] + q4 * wl[1][a] + q5 * wl[2][a])
                     + sr.rho * (q3 * wr[0][a] + q4 * wr[1][a] + q5 * wr[2][a]);
        }
    }
    /* solve  F dt + dF dt^2/2 = I(dt),  F dt/2 + dF dt^2/8 = I(dt/2)  (Cramer) */
    const double m11 = dt, m12 = 0.5 * dt * dt, m21 = 0.5 * dt, m22 = dt * dt / 8.0;
    const double det = m11 * m22 - m12 * m21;
    double Fl[5], dFl[5];
    for (int a = 0; a < 5; ++a) {
        Fl[a] = (I[0][a] * m22 - m12 * I[1][a]) / det;
        dFl[a] = (m11 * I[1][a] - I[0][a] * m21) / det;
    }
    if (prandtl) {
        /* heat flux of f in the frame of U0: q = 1/2 <(u - U0)_n ((u - U0)^2 + xi^2) f>
         *   = F_E - U0.F_m + |U0|^2/2 F_rho - U0_n (W_E - U0.W_m + |U0|^2/2 W_rho),
         * fitted in time like F; the energy flux takes (1/Pr - 1) q */
        const double U0[3] = {s0.U, s0.V, s0.W};
        const double u2 = 0.5 * dot3(U0, U0);
        double Wf[5], dWf[5];
        for (int a = 0; a < 5; ++a) {
            Wf[a] = (IW[0][a] * m22 - m12 * IW[1][a]) / det;
            dWf[a] = (m11 * IW[1][a] - IW[0][a] * m21) / det;
        }
        const double qh = Fl[4] - (U0[0] * Fl[1] + U0[1] * Fl[2] + U0[2] * Fl[3]) + u2 * Fl[0]
                        - U0[0] * (Wf[4] - (U0[0] * Wf[1] + U0[1] * Wf[2] + U0[2] * Wf[3]) + u2 * Wf[0]);
        const double dqh = dFl[4] - (U0[0] * dFl[1] + U0[1] * dFl[2] + U0[2] * dFl[3]) + u2 * dFl[0]
                         - U0[0] * (dWf[4] - (U0[0] * dWf[1] + U0[1] * dWf[2] + U0[2] * dWf[3]) + u2 * dWf[0]);
        Fl[4] += (1.0 / p->prandtl - 1.0) * qh;
        dFl[4] += (1.0 / p->prandtl - 1.0) * dqh;
    }
    /* rotate back to the global frame */
    F[0] = Fl[0]; dF[0] = dFl[0];
    for (int a = 0; a < 3; ++a) {
        F[1 + a] = Fl[1] * n[a] + Fl[2] * t1[a] + Fl[3] * t2[a];
        dF[1 + a] = dFl[1] * n[a] + dFl[2] * t1[a] + dFl[3] * t2[a];
    }
    F[4] = Fl[4]; dF[4] = dFl[4];
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* L(Q), dL/dt (Eq. finite) and the S2O4 step (Sec. 2.2)                     */
/* ------------------------------------------------------------------------- */

/*
 * L_i = -(1/|Omega_i|) sum_faces F S (outward), and the same for dL/dt.
 * Independent loops (cells, then faces, then cells) may run on several OpenMP
 * threads: each iteration writes only its own slot, and the per-cell sum over a
 * cell's four faces runs in local face order, so the result does not depend on
 * the thread count.
 */
/*
 * Positivity fallback (not in the paper, which has no limiter): at a Gauss point
 * where the reconstructed state of either side has rho <= 0 or p <= 0, the point
 * takes the first-order gas-kinetic flux, the flux of piecewise-constant data:
 * no slopes on either side, and each non-physical side's value replaced by its
 * cell average (a physical side keeps its point value).  Both slopes go because
 * in Eq. (flux) they do not act separately: the equilibrium slope is formed from
 * both sides, dQ0 = (dQ_l + dQ_r)/2, and the time slopes follow from the spatial
 * ones through the compatibility condition, so once one side's gradient is
 * unusable the equilibrium part has no consistent slope left; dropping only that
 * side would leave the equilibrium half of the other side's slope, which belongs
 * to no reconstruction.  It never acts in smooth flow; at a strong discontinuity
 * (the shock tube) the quadratic reconstruction would otherwise hand the flux a
 * state with negative pressure on the first step.
 */
static int physical_point(const orc_params *p, const double *v) {
    const double rho = v[0];
    const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho;
    return rho > 0.0 && (p->gamma - 1.0) * (v[4] - ke) > 0.0;
}

static void gauss_point_fallback(const orc_params *p, const double *ql_cell, const double *qr_cell, double *vl,
                                 double gl[5][3], double *vr, double gr[5][3]) {
    const int okl = physical_point(p, vl), okr = physical_point(p, vr);
    if (okl && okr) return;
    for (int q = 0; q < 5; ++q) {
        if (!okl) vl[q] = ql_cell[q];
        if (!okr) vr[q] = qr_cell[q];
        gl[q][0] = gl[q][1] = gl[q][2] = 0.0;
        gr[q][0] = gr[q][1] = gr[q][2] = 0.0;
    }
}

/* Right side of Gauss point g of face f: the right cell's reconstruction, or at a
 * boundary face the ghost's.  At a transmissive wall the ghost is the wall cell's
 * reconstruction mirrored (the same value at the in-wall point, the gradient
 * reflected in the wall); at a no-slip wall the same with the momentum negated; at
 * the far field the Riemann-invariant state of the left point value, no gradient.
 * qr_cell receives the right cell's (or ghost's) cell average. */
static void right_point(const orc_mesh *m, const orc_params *p, const double *Q, const orc_weno *W, int64_t f,
                        int g, const double *vl, double gl[5][3], double *vr, double gr[5][3], double *qr_cell) {
    const int64_t l = m->fcell[f][0], r = m->fcell[f][1];
    if (r >= 0) {
        double xr[3];
        for (int a = 0; a < 3; ++a) xr[a] = m->fgp[f][g][a] - m->fshift[f][a];
        weno_eval(m, p, Q, r, &W[r], xr, vr, gr);
        memcpy(qr_cell, Q + 5 * r, sizeof(double) * 5);
        return;
    }
    const double *n = m->fnrm[f];
    const int kind = m->fkind[f];
    if (kind == ORC_BC_FAR) {
        farfield_state(p, vl, m->fpn[f][g], vr);
        for (int q = 0; q < 5; ++q) gr[q][0] = gr[q][1] = gr[q][2] = 0.0;
        farfield_state(p, Q + 5 * l, n, qr_cell);
        return;
    }
    const double sg = kind == ORC_BC_WALL ? -1.0 : 1.0;      /* momentum sign of the ghost */
    for (int q = 0; q < 5; ++q) {
        const double s_ = (q >= 1 && q <= 3) ? sg : 1.0;
        const double gn = gl[q][0] * n[0] + gl[q][1] * n[1] + gl[q][2] * n[2];
        vr[q] = s_ * vl[q];
        for (int a = 0; a < 3; ++a) gr[q][a] = s_ * (gl[q][a] - 2.0 * gn * n[a]);
        qr_cell[q] = s_ * Q[5 * l + q];
    }
}

/* S * sum_G w_G (F, dF) of face f; with tets the three points share the face
 * normal and weigh 1/3 each. */
static int face_flux(const orc_mesh *m, const orc_params *p, const double *Q, const orc_weno *W, int64_t f,
                     double dt, double out[10]) {
    const int64_t l = m->fcell[f][0];
    double Ff[5] = {0}, dFf[5] = {0};
    int rc = ORC_OK;
    for (int g = 0; g < m->ngp; ++g) {
        double vl[5], vr[5], gl[5][3], gr[5][3], F[5], dF[5], qr_cell[5];
        weno_eval(m, p, Q, l, &W[l], m->fgp[f][g], vl, gl);
        right_point(m, p, Q, W, f, g, vl, gl, vr, gr, qr_cell);
        gauss_point_fallback(p, Q + 5 * l, qr_cell, vl, gl, vr, gr);
        int r_ = orc_gks_flux(p, vl, &gl[0][0], vr, &gr[0][0], m->ngp == 3 ? m->fnrm[f] : m->fpn[f][g], dt, F, dF);
        if (r_ > rc) rc = r_;
        for (int q = 0; q < 5; ++q) {
            if (m->ngp == 3) { Ff[q] += F[q] / 3.0; dFf[q] += dF[q] / 3.0; }
            else { Ff[q] += m->fpw[f][g] * F[q]; dFf[q] += m->fpw[f][g] * dF[q]; }
        }
    }
    const double S = m->ngp == 3 ? m->farea[f] : 1.0;
    for (int q = 0; q < 5; ++q) { out[q] = Ff[q] * S; out[5 + q] = dFf[q] * S; }
    return rc;
}

int orc_rhs(const orc_mesh *m, const orc_params *p, const double *Q, double dt, double *L, double *dL) {
    orc_weno *W = malloc(sizeof(orc_weno) * m->nc);
    double (*FF)[10] = malloc(sizeof(double[10]) * m->nf);   /* S * sum_G w_G (F, dF) per face */
    int rc = ORC_OK;
#pragma omp parallel for schedule(static) reduction(max: rc)
    for (int64_t i = 0; i < m->nc; ++i) {
        int r_ = weno_cell(m, p, Q, i, &W[i]);
        if (r_ > rc) rc = r_;
    }
    if (rc == ORC_OK) {
#pragma omp parallel for schedule(static) reduction(max: rc)
        for (int64_t f = 0; f < m->nf; ++f) {
            int r_ = face_flux(m, p, Q, W, f, dt, FF[f]);
            if (r_ > rc) rc = r_;
        }
    }
    if (rc == ORC_OK) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m->nc; ++i) {
            double s[10] = {0};
            for (int p_ = 0; p_ < m->nfc; ++p_) {
                int64_t f = m->cface[i][p_];
                double sign = m->fcell[f][0] == i ? -1.0 : 1.0;    /* the normal points out of the left cell */
                for (int q = 0; q < 10; ++q) s[q] += sign * FF[f][q];
            }
            for (int q = 0; q < 5; ++q) { L[5 * i + q] = s[q] / m->vol[i]; dL[5 * i + q] = s[5 + q] / m->vol[i]; }
        }
    }
    free(W);
    free(FF);
    return rc;
}

double orc_cfl_dt(const orc_mesh *m, const orc_params *p, const double *Q) {
    double best = INFINITY;
    for (int64_t i = 0; i < m->nc; ++i) {
        prim s = primitives(Q + 5 * i, p->gamma);
        double c = sqrt(p->gamma * s.p / s.rho);
        double v = sqrt(s.U * s.U + s.V * s.V + s.W * s.W);
        double d = m->hdt[i] / (v + c);
        if (d < best) best = d;
    }
    return p->cfl * best;
}

void orc_s2o4_stage1(int64_t n, const double *q, const double *L, const double *dL, double dt, double *qs) {
    for (int64_t k = 0; k < n; ++k) qs[k] = q[k] + 0.5 * dt * L[k] + dt * dt / 8.0 * dL[k];
}

void orc_s2o4_stage2(int64_t n, const double *q, const double *L, const double *dL, const double *dLs,
                     double dt, double *qn) {
    for (int64_t k = 0; k < n; ++k) qn[k] = q[k] + dt * L[k] + dt * dt / 6.0 * (dL[k] + 2.0 * dLs[k]);
}

static int physical(const double *Q, int64_t nc, double gamma) {
    for (int64_t i = 0; i < nc; ++i) {
        for (int q = 0; q < 5; ++q) if (!isfinite(Q[5 * i + q])) return 0;
        prim s = primitives(Q + 5 * i, gamma);
        if (!(s.rho > 0.0 && s.p > 0.0)) return 0;
    }
    return 1;
}

/* nsteps S2O4 steps in place; dt from the CFL rule unless dt_fixed > 0. */
int orc_step(const orc_mesh *m, const orc_params *p, double *Q, int nsteps, double dt_fixed, double *dt_last) {
    const int64_t n = 5 * m->nc;
    double *L = malloc(sizeof(double) * n), *dL = malloc(sizeof(double) * n);
    double *Ls = malloc(sizeof(double) * n), *dLs = malloc(sizeof(double) * n);
    double *Qs = malloc(sizeof(double) * n), *Qn = malloc(sizeof(double) * n);
    int rc = ORC_OK;
    for (int s = 0; s < nsteps && rc == ORC_OK; ++s) {
        double dt = dt_fixed > 0.0 ? dt_fixed : orc_cfl_dt(m, p, Q);
        if (dt_last) *dt_last = dt;
        rc = orc_rhs(m, p, Q, dt, L, dL);
        if (rc) break;
        orc_s2o4_stage1(n, Q, L, dL, dt, Qs);
        if (!physical(Qs, m->nc, p->gamma)) { rc = ORC_E_NONPHYS; break; }
        rc = orc_rhs(m, p, Qs, dt, Ls, dLs);
        if (rc) break;
        orc_s2o4_stage2(n, Q, L, dL, dLs, dt, Qn);
        if (!physical(Qn, m->nc, p->gamma)) { rc = ORC_E_NONPHYS; break; }
        memcpy(Q, Qn, sizeof(double) * n);
    }
    free(L); free(dL); free(Ls); free(dLs); free(Qs); free(Qn);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* test hooks: pieces of the method exposed for pinning                      */
/* ------------------------------------------------------------------------- */

void orc_moments_1d(double U, double lam, double *full, double *pos, double *neg) {
    if (full) full_moments_1d(U, lam, full);
    if (pos) half_moments_1d(U, lam, +1, pos);
    if (neg) half_moments_1d(U, lam, -1, neg);
}

int orc_slope(double U, double V, double W, double lam, double K, const double *b, double *a) {
    build_tables();
    moments M;
    make_moments(U, V, W, lam, K, 0, &M);
    return slope_solve(&M, b, a);
}

/* Q0 of the collision of two states (conservative, already in the local frame). */
void orc_collision(const orc_params *p, const double *ql, const double *qr, double *q0) {
    build_tables();
    const double K = (5.0 - 3.0 * p->gamma) / (p->gamma - 1.0);
    prim sl = primitives(ql, p->gamma), sr = primitives(qr, p->gamma);
    moments Mlp, Mrn;
    make_moments(sl.U, sl.V, sl.W, sl.lam, K, +1, &Mlp);
    make_moments(sr.U, sr.V, sr.W, sr.lam, K, -1, &Mrn);
    for (int a = 0; a < 5; ++a) q0[a] = sl.rho * expect(&Mlp, &PSI[a]) + sr.rho * expect(&Mrn, &PSI[a]);
}

/* WENO of one cell: P0 coefficients a[5][9], P_m coefficients b[M][5][3], beta[5][M+1],
 * wbar[5][M+1] (M = 4 for tets, 8 for hexes). */
int orc_weno_cell(const orc_mesh *m, const orc_params *p, const double *Q, int64_t i,
                  double *a, double *b, double *beta, double *wbar) {
    orc_weno w;
    int rc = weno_cell(m, p, Q, i, &w);
    if (rc) return rc;
    const int M = m->msub;
    if (a) memcpy(a, w.a, sizeof(w.a));
    if (b) memcpy(b, w.b, sizeof(double) * 15 * M);
    for (int q = 0; q < 5; ++q)
        for (int s = 0; s <= M; ++s) {
            if (beta) beta[q * (M + 1) + s] = w.beta[q][s];
            if (wbar) wbar[q * (M + 1) + s] = w.wbar[q][s];
        }
    return ORC_OK;
}

/* The state a boundary ghost of the given kind holds next to state q (outward normal n). */
void orc_ghost_state(const orc_params *p, int kind, const double *q, const double *n, double *out) {
    ghost_state(p, kind, q, n, out);
}

/* Reconstructed value and gradient of cell i at point x (cell i's frame). */
int orc_reconstruct(const orc_mesh *m, const orc_params *p, const double *Q, int64_t i, const double *x,
                    double *val, double *grad) {
    orc_weno w;
    int rc = weno_cell(m, p, Q, i, &w);
    if (rc) return rc;
    double g[5][3];
    weno_eval(m, p, Q, i, &w, x, val, g);
    memcpy(grad, g, sizeof(g));
    return ORC_OK;
}

/* S * sum_G w_G (F, dF) of face f for the state Q (WENO of both cells formed here). */
int orc_face_flux(const orc_mesh *m, const orc_params *p, const double *Q, int64_t f, double dt, double *out) {
    if (f < 0 || f >= m->nf) return ORC_E_ARG;
    orc_weno *W = malloc(sizeof(orc_weno) * m->nc);
    const int64_t l = m->fcell[f][0], r = m->fcell[f][1];
    int rc = weno_cell(m, p, Q, l, &W[l]);
    if (!rc && r >= 0) rc = weno_cell(m, p, Q, r, &W[r]);
    if (!rc) rc = face_flux(m, p, Q, W, f, dt, out);
    free(W);
    return rc;
}

/*
 * Census of the positivity fallback for the state Q: out[0] Gauss points where it
 * acts, out[1] of those the points with exactly one non-physical side, out[2] of
 * those the points where the physical side's reconstructed gradient is nonzero
 * (some component above 1e-6 of that side's value scale).
 */
int orc_fallback_census(const orc_mesh *m, const orc_params *p, const double *Q, int64_t *out) {
    orc_weno *W = malloc(sizeof(orc_weno) * m->nc);
    int rc = ORC_OK;
    for (int64_t i = 0; i < m->nc && !rc; ++i) rc = weno_cell(m, p, Q, i, &W[i]);
    int64_t all = 0, one = 0, one_grad = 0;
    for (int64_t f = 0; f < m->nf && !rc; ++f) {
        const int64_t l = m->fcell[f][0];
        for (int g = 0; g < m->ngp; ++g) {
            double vl[5], vr[5], gl[5][3], gr[5][3], qr_cell[5];
            weno_eval(m, p, Q, l, &W[l], m->fgp[f][g], vl, gl);
            right_point(m, p, Q, W, f, g, vl, gl, vr, gr, qr_cell);
            const int okl = physical_point(p, vl), okr = physical_point(p, vr);
            if (okl && okr) continue;
            ++all;
            if (okl == okr) continue;
            ++one;
            const double *v = okl ? vl : vr;
            double (*gg)[3] = okl ? gl : gr;
            double vs = 0.0, gs = 0.0;
            for (int q = 0; q < 5; ++q) {
                if (fabs(v[q]) > vs) vs = fabs(v[q]);
                for (int a = 0; a < 3; ++a) if (fabs(gg[q][a]) > gs) gs = fabs(gg[q][a]);
            }
            if (gs > 1e-6 * vs) ++one_grad;
        }
    }
    free(W);
    out[0] = all; out[1] = one; out[2] = one_grad;
    return rc;
}

/* mean over cell i of the scaled monomials, as used by the least-squares rows */
void orc_cell_monomial_means(const orc_mesh *m, int64_t i, const double *target_c, double target_h, double *out) {
    cell_monomial_means(m->npc, m->vert[i], target_c, target_h, out);
}

/* ------------------------------------------------------------------------- */
/* One S2O4 step for a sample of cells only                                   */
/* ------------------------------------------------------------------------- */

/* mark every cell of the two-layer stencil of each marked cell, and the cell */
static void mark_stencils(const orc_mesh *m, const unsigned char *in, unsigned char *out) {
    for (int64_t i = 0; i < m->nc; ++i) {
        if (!in[i]) continue;
        out[i] = 1;
        for (int k = 0; k < m->nsten[i]; ++k) {
            const int64_t id = m->sten[i][k];
            out[id < m->nc ? id : m->gcell[id - m->nc]] = 1;     /* a ghost reads its cell */
        }
    }
}

/* faces touching a marked cell, and the cells on their other side */
static void mark_faces(const orc_mesh *m, const unsigned char *cells, unsigned char *faces, unsigned char *both) {
    for (int64_t f = 0; f < m->nf; ++f) {
        int64_t l = m->fcell[f][0], r = m->fcell[f][1];
        if (r < 0) r = l;                              /* wall face: the ghost images l */
        if (cells[l] || cells[r]) { faces[f] = 1; both[l] = both[r] = 1; }
    }
}

/* L and dL/dt of the cells in `need`, evaluating WENO and fluxes only where needed. */
static int rhs_subset(const orc_mesh *m, const orc_params *p, const double *Q, double dt,
                      const unsigned char *need, double *L, double *dL) {
    unsigned char *faces = calloc((size_t)m->nf, 1), *wcells = calloc((size_t)m->nc, 1);
    mark_faces(m, need, faces, wcells);
    orc_weno *W = malloc(sizeof(orc_weno) * m->nc);
    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64) reduction(max: rc)
    for (int64_t i = 0; i < m->nc; ++i) {
        if (!wcells[i]) continue;
        int r_ = weno_cell(m, p, Q, i, &W[i]);
        if (r_ > rc) rc = r_;
    }
    double (*FF)[10] = calloc((size_t)m->nf, sizeof(double[10]));
    if (rc == ORC_OK) {
#pragma omp parallel for schedule(dynamic, 64) reduction(max: rc)
        for (int64_t f = 0; f < m->nf; ++f) {
            if (!faces[f]) continue;
            int r_ = face_flux(m, p, Q, W, f, dt, FF[f]);
            if (r_ > rc) rc = r_;
        }
    }
    if (rc == ORC_OK)
        for (int64_t i = 0; i < m->nc; ++i) {
            if (!need[i]) continue;
            double s[10] = {0};
            for (int p_ = 0; p_ < m->nfc; ++p_) {
                int64_t f = m->cface[i][p_];
                double sign = m->fcell[f][0] == i ? -1.0 : 1.0;
                for (int q = 0; q < 10; ++q) s[q] += sign * FF[f][q];
            }
            for (int q = 0; q < 5; ++q) { L[5 * i + q] = s[q] / m->vol[i]; dL[5 * i + q] = s[5 + q] / m->vol[i]; }
        }
    free(faces); free(wcells); free(W); free(FF);
    return rc;
}

/*
 * Q^{n+1} of the listed cells after one S2O4 step of size dt from Q (the whole
 * state): the same arithmetic as orc_step, evaluated only on the dependency
 * region of the sample (the cells whose stage values the sample's fluxes read).
 */
int orc_step_sample(const orc_mesh *m, const orc_params *p, const double *Q, double dt,
                    int64_t ns, const int64_t *cells, double *out /*[ns][5]*/) {
    const int64_t nc = m->nc;
    unsigned char *s2 = calloc((size_t)nc, 1), *w2 = calloc((size_t)nc, 1), *qs_need = calloc((size_t)nc, 1);
    unsigned char *f2 = calloc((size_t)m->nf, 1);
    for (int64_t k = 0; k < ns; ++k) s2[cells[k]] = 1;
    mark_faces(m, s2, f2, w2);                 /* cells whose WENO at Q* the sample needs */
    mark_stencils(m, w2, qs_need);             /* cells whose Q* those reconstructions read */
    double *L = calloc((size_t)(5 * nc), sizeof(double)), *dL = calloc((size_t)(5 * nc), sizeof(double));
    double *Qs = malloc(sizeof(double) * 5 * nc);
    memcpy(Qs, Q, sizeof(double) * 5 * nc);
    int rc = rhs_subset(m, p, Q, dt, qs_need, L, dL);
    if (rc == ORC_OK) {
        for (int64_t i = 0; i < nc; ++i)
            if (qs_need[i])
                for (int q = 0; q < 5; ++q) Qs[5 * i + q] = Q[5 * i + q] + 0.5 * dt * L[5 * i + q] + dt * dt / 8.0 * dL[5 * i + q];
        double *Ls = calloc((size_t)(5 * nc), sizeof(double)), *dLs = calloc((size_t)(5 * nc), sizeof(double));
        rc = rhs_subset(m, p, Qs, dt, s2, Ls, dLs);
        for (int64_t k = 0; k < ns && rc == ORC_OK; ++k) {
            int64_t i = cells[k];
            for (int q = 0; q < 5; ++q)
                out[5 * k + q] = Q[5 * i + q] + dt * L[5 * i + q] + dt * dt / 6.0 * (dL[5 * i + q] + 2.0 * dLs[5 * i + q]);
        }
        free(Ls); free(dLs);
    }
    free(s2); free(w2); free(qs_need); free(f2); free(L); free(dL); free(Qs);
    return rc;
}

/* number of threads the parallel loops use */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
