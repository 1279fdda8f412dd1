"""Seeded synthetic inputs for the HGKS step: meshes, initial states, request streams.

This module only *generates inputs*; it holds none of the scheme's arithmetic.
Both the GPU path (tests, bench, serving) and the CPU oracle's tests draw their
inputs from here.

* Meshes: the periodic accuracy-test box of Sec. 5.1, "every cube divided into six
  tetrahedra" (below), the same box of jittered hexahedra, and the cubed-sphere
  O-grid of hexahedra around a sphere (Sec. 5.2: six patches of N x N cells by the
  radial layers).  The split is the Kuhn split along the main diagonal: for cube
  (i, j, k) and each permutation sigma of the axes (lexicographic order), the
  tetrahedron is the lattice path v0 -> v0+e_s1 -> v0+e_s1+e_s2 -> v0+(1,1,1).
  Cell id = 6*((i*N + j)*N + k) + sigma.  Interior vertices are jittered by
  i.i.d. U(-j*h, j*h) per component; vertices on the box boundary (index 0 mod N
  on any axis) are not moved.
* Random numbers: SplitMix64 in counter form (Steele, Lea & Flood, 2014): the
  k-th draw of a stream with seed s is mix(s + (k+1) * 0x9E3779B97F4A7C15), and a
  uniform double in [0,1) is (x >> 11) * 2^-53.
* Cell averages: collapsed-coordinate (Duffy) Gauss-Jacobi product rule on each
  tetrahedron, exact for polynomials of total degree 2n-1.
* Initial data: the advection test of Sec. 5.1, rho = 1 + A sin(pi k.(x - U t) + phi),
  uniform velocity U and pressure p, given as exact cell averages of the
  conservative variables (point values at centroids would add an O(h^2) error).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as _sp

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Lexicographic permutations of the three axes; tet sigma walks e_s[0], e_s[1], e_s[2].
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))

SEED_ADVECTION = 0x2407006561


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws start..start+count-1 of the counter-form SplitMix64 stream `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    return (splitmix64(seed, count, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class TetMesh:
    """A mesh in the form the library and the oracle both take (tetrahedra or
    hexahedra; the name is historical).

    nodes       [n_nodes, 3] float64 coordinates
    cell_nodes  [n_cells, 4] (tetrahedra) or [n_cells, 8] (hexahedra: nodes 0-3
                around one face, node k+4 above node k) int64 node ids (0-based)
    period      [3] float64; period[a] > 0 identifies x_a and x_a + period[a]
    cell_vertices [n_cells, 4 or 8, 3] unwrapped vertex coordinates (generator-side
                only, used to integrate initial data)
    bfaces, bkinds  listed boundary faces ([nb, 4] node ids) and their kinds
                (BC_WALL, BC_FAR), or None
    """
    nodes: np.ndarray
    cell_nodes: np.ndarray
    period: np.ndarray
    cell_vertices: np.ndarray
    n: int = 0
    box: float = 2.0
    meta: dict = field(default_factory=dict)
    bfaces: np.ndarray | None = None
    bkinds: np.ndarray | None = None

    @property
    def n_cells(self) -> int:
        return int(self.cell_nodes.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])


def kuhn_box(n, box=2.0, jitter: float = 0.1, seed: int = SEED_ADVECTION,
             periodic=(True, True, True)) -> TetMesh:
    """6 nx ny nz Kuhn tetrahedra in [0, Lx] x [0, Ly] x [0, Lz], jittered from `seed`.

    `n` is the number of cubes per axis (an int for a cubic lattice, or a triple) and
    `box` the box length (a float, or a triple).  Interior nodes move by
    U(-jitter h_a, jitter h_a) per component a; nodes on the box faces do not move.
    """
    nv = np.array([n, n, n] if np.isscalar(n) else list(n), dtype=np.int64)
    bv = np.array([box, box, box] if np.isscalar(box) else list(box), dtype=np.float64)
    if np.any(nv < 4):
        raise ValueError("kuhn_box needs n >= 4 per axis (two-layer stencils must not wrap onto themselves)")
    periodic = tuple(bool(p) for p in periodic)
    h = bv / nv
    dims = np.array([nv[a] if periodic[a] else nv[a] + 1 for a in range(3)], dtype=np.int64)
    ix, iy, iz = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]), np.arange(dims[2]), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)          # node id order
    nodes = idx.astype(np.float64) * h[None, :]
    interior = np.all((idx % nv[None, :]) != 0, axis=1)
    if jitter > 0.0:
        u = uniform01(seed, 3 * idx.shape[0]).reshape(-1, 3)
        nodes = nodes + np.where(interior[:, None], (2.0 * u - 1.0) * jitter * h[None, :], 0.0)

    def node_id(a, b, c):
        return (a * dims[1] + b) * dims[2] + c

    ci, cj, ck = np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)          # cube order (i, j, k)
    n_cubes = base.shape[0]
    cell_nodes = np.empty((n_cubes, 6, 4), dtype=np.int64)
    cell_vertices = np.empty((n_cubes, 6, 4, 3), dtype=np.float64)
    period = np.array([bv[a] if periodic[a] else 0.0 for a in range(3)])
    for s, perm in enumerate(KUHN_PERMS):
        off = np.zeros(3, dtype=np.int64)
        for v in range(4):
            if v > 0:
                off = off.copy()
                off[perm[v - 1]] += 1
            lat = base + off                                               # unwrapped lattice index
            wrap = np.zeros_like(lat)
            for a in range(3):
                if periodic[a]:
                    wrap[:, a] = lat[:, a] // nv[a]
            li = lat - wrap * nv[None, :]
            nid = node_id(li[:, 0], li[:, 1], li[:, 2])
            cell_nodes[:, s, v] = nid
            cell_vertices[:, s, v, :] = nodes[nid] + wrap * period
    cubic = bool(np.all(nv == nv[0]) and np.all(bv == bv[0]))
    return TetMesh(nodes=nodes, cell_nodes=cell_nodes.reshape(-1, 4),
                   period=period, cell_vertices=cell_vertices.reshape(-1, 4, 3),
                   n=int(nv[0]) if cubic else 0, box=float(bv[0]) if cubic else 0.0,
                   meta={"seed": seed, "jitter": jitter, "periodic": periodic, "n": tuple(int(x) for x in nv),
                         "box": tuple(float(x) for x in bv)})


# boundary kinds of listed boundary faces
BC_WALL = 1     # no-slip adiabatic wall
BC_FAR = 2      # far field (Riemann invariants)

# reference coordinates of the hexahedron's nodes on [0, 1]^3
HEX_REF = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.float64)


def hex_box(n, box=2.0, jitter: float = 0.1, seed: int = SEED_ADVECTION + 0x4E58,
            periodic=(True, True, True)) -> TetMesh:
    """nx ny nz hexahedra (the cubes themselves) in [0, Lx] x [0, Ly] x [0, Lz],
    interior nodes jittered by U(-jitter h_a, jitter h_a) per component (so the
    faces are bilinear, not planar).  Cell id = (i*ny + j)*nz + k."""
    nv = np.array([n, n, n] if np.isscalar(n) else list(n), dtype=np.int64)
    bv = np.array([box, box, box] if np.isscalar(box) else list(box), dtype=np.float64)
    if np.any(nv < 5):
        raise ValueError("hex_box needs n >= 5 per axis (two-layer stencils must not wrap onto themselves)")
    periodic = tuple(bool(p) for p in periodic)
    h = bv / nv
    dims = np.array([nv[a] if periodic[a] else nv[a] + 1 for a in range(3)], dtype=np.int64)
    ix, iy, iz = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]), np.arange(dims[2]), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    nodes = idx.astype(np.float64) * h[None, :]
    interior = np.all((idx % nv[None, :]) != 0, axis=1)
    if jitter > 0.0:
        u = uniform01(seed, 3 * idx.shape[0]).reshape(-1, 3)
        nodes = nodes + np.where(interior[:, None], (2.0 * u - 1.0) * jitter * h[None, :], 0.0)
    ci, cj, ck = np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    period = np.array([bv[a] if periodic[a] else 0.0 for a in range(3)])
    cell_nodes = np.empty((base.shape[0], 8), dtype=np.int64)
    cell_vertices = np.empty((base.shape[0], 8, 3))
    for v in range(8):
        lat = base + HEX_REF[v].astype(np.int64)[None, :]
        wrap = np.zeros_like(lat)
        for a in range(3):
            if periodic[a]:
                wrap[:, a] = lat[:, a] // nv[a]
        li = lat - wrap * nv[None, :]
        nid = (li[:, 0] * dims[1] + li[:, 1]) * dims[2] + li[:, 2]
        cell_nodes[:, v] = nid
        cell_vertices[:, v, :] = nodes[nid] + wrap * period
    cubic = bool(np.all(nv == nv[0]) and np.all(bv == bv[0]))
    return TetMesh(nodes=nodes, cell_nodes=cell_nodes, period=period, cell_vertices=cell_vertices,
                   n=int(nv[0]) if cubic else 0, box=float(bv[0]) if cubic else 0.0,
                   meta={"seed": seed, "jitter": jitter, "periodic": periodic, "n": tuple(int(x) for x in nv),
                         "box": tuple(float(x) for x in bv), "cell": "hex"})


def cubed_sphere(n: int, layers: int, r0: float = 0.5, r1: float = 20.0) -> TetMesh:
    """The O-grid of hexahedra around a sphere (Sec. 5.2): six patches, each the
    equiangular gnomonic projection of an n x n grid on a cube face, extruded over
    `layers` radial layers whose radii grow geometrically from r0 (the sphere) to r1
    (the far field).  Nodes 0-3 of a cell lie on its inner sphere, 4-7 on its outer,
    so faces 1 and 6 (0-based 0 and 5) are the radial pair.  The inner faces of the
    first layer are no-slip walls and the outer faces of the last layer far-field
    faces (bfaces / bkinds).  Cell id = ((patch*n + i)*n + j)*layers + k."""
    if n < 2 or layers < 4:
        raise ValueError("cubed_sphere needs n >= 2 and layers >= 4")
    t = np.tan(np.linspace(-math.pi / 4, math.pi / 4, n + 1))
    radii = r0 * (r1 / r0) ** (np.arange(layers + 1) / layers)
    # patch p: axis p // 2, side +1 / -1; (a, b) run over the two other axes in a
    # right-handed order so that every patch's cells have the same orientation
    dirs = []
    for p in range(6):
        ax, sg = p // 2, (1.0 if p % 2 == 0 else -1.0)
        o1, o2 = (ax + 1) % 3, (ax + 2) % 3
        A, B = np.meshgrid(t, t, indexing="ij")
        d = np.empty((n + 1, n + 1, 3))
        d[..., ax] = sg
        d[..., o1] = A if sg > 0 else B
        d[..., o2] = B if sg > 0 else A
        dirs.append(d / np.linalg.norm(d, axis=-1, keepdims=True))
    dirs = np.stack(dirs)                                              # [6, n+1, n+1, 3]
    # shared patch edges give the same direction: merge them by rounded key
    key = np.round(dirs.reshape(-1, 3) * 2 ** 30).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(6, n + 1, n + 1)
    udir = dirs.reshape(-1, 3)[first]
    nd = udir.shape[0]
    nodes = (radii[None, :, None] * udir[:, None, :]).reshape(-1, 3)   # node id = dir * (layers+1) + k
    P, I, J, K = np.meshgrid(np.arange(6), np.arange(n), np.arange(n), np.arange(layers), indexing="ij")
    P, I, J, K = P.ravel(), I.ravel(), J.ravel(), K.ravel()
    corner = [(0, 0), (1, 0), (1, 1), (0, 1)]
    cell_nodes = np.empty((P.shape[0], 8), dtype=np.int64)
    for v, (di, dj) in enumerate(corner):
        dn = inv[P, I + di, J + dj]
        cell_nodes[:, v] = dn * (layers + 1) + K
        cell_nodes[:, v + 4] = dn * (layers + 1) + K + 1
    cell_vertices = nodes[cell_nodes]
    inner = cell_nodes[K == 0][:, :4]
    outer = cell_nodes[K == layers - 1][:, 4:]
    bfaces = np.concatenate([inner, outer])
    bkinds = np.concatenate([np.full(inner.shape[0], BC_WALL), np.full(outer.shape[0], BC_FAR)]).astype(np.int32)
    return TetMesh(nodes=nodes, cell_nodes=cell_nodes, period=np.zeros(3), cell_vertices=cell_vertices,
                   n=n, box=0.0, bfaces=bfaces, bkinds=bkinds,
                   meta={"cell": "hex", "patches": 6, "n": n, "layers": layers, "r0": r0, "r1": r1,
                         "unique_directions": int(nd)})


def hex_cell_average(cell_vertices: np.ndarray, fun, npts: int, chunk: int = 32768) -> np.ndarray:
    """Cell averages of fun(x, y, z) over trilinear hexahedra: the npts^3
    Gauss-Legendre product rule over the map, weighted by |det J|."""
    g, w = np.polynomial.legendre.leggauss(npts)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    R = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)     # [P, 3]
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    # shape functions and their derivatives at the points
    f = np.where(HEX_REF[None, :, :] > 0, R[:, None, :], 1.0 - R[:, None, :])       # [P, 8, 3]
    df = np.where(HEX_REF[None, :, :] > 0, 1.0, -1.0) * np.ones_like(f)
    N = f.prod(axis=2)                                                             # [P, 8]
    dN = np.stack([df[..., 0] * f[..., 1] * f[..., 2], f[..., 0] * df[..., 1] * f[..., 2],
                   f[..., 0] * f[..., 1] * df[..., 2]], axis=2)                     # [P, 8, 3]
    out = np.empty(cell_vertices.shape[0])
    for s in range(0, cell_vertices.shape[0], chunk):
        v = cell_vertices[s:s + chunk]                                             # [c, 8, 3]
        x = np.einsum("pk,cka->cpa", N, v)
        J = np.einsum("pkd,cka->cpad", dN, v)
        det = np.abs(np.linalg.det(J))
        wd = det * W[None, :]
        out[s:s + chunk] = np.sum(fun(x[..., 0], x[..., 1], x[..., 2]) * wd, axis=1) / np.sum(wd, axis=1)
    return out


def hex_volumes(cell_vertices: np.ndarray) -> np.ndarray:
    """Volumes of trilinear hexahedra (2x2x2 Gauss-Legendre, exact for the Jacobian's degree)."""
    g, w = np.polynomial.legendre.leggauss(2)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    R = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    f = np.where(HEX_REF[None, :, :] > 0, R[:, None, :], 1.0 - R[:, None, :])
    df = np.where(HEX_REF[None, :, :] > 0, 1.0, -1.0) * np.ones_like(f)
    dN = np.stack([df[..., 0] * f[..., 1] * f[..., 2], f[..., 0] * df[..., 1] * f[..., 2],
                   f[..., 0] * f[..., 1] * df[..., 2]], axis=2)
    J = np.einsum("pkd,cka->cpad", dN, cell_vertices)
    return np.abs(np.linalg.det(J)) @ W


def cell_volumes(mesh: TetMesh) -> np.ndarray:
    return hex_volumes(mesh.cell_vertices) if mesh.cell_nodes.shape[1] == 8 else tet_volumes(mesh.cell_vertices)


@dataclass
class SphereCase:
    """Viscous flow past the unit-diameter sphere (Sec. 5.2): free stream
    (rho, U, V, W, p) = (1, Ma, 0, 0, 1/gamma), mu = mu_inf (T/T_inf)^0.7 with
    mu_inf = rho U D / Re, T = p/rho.  The initial state is the free stream."""
    mach: float = 0.2535
    reynolds: float = 118.0
    prandtl: float = 0.72
    gamma: float = 1.4

    def freestream(self):
        return (1.0, self.mach, 0.0, 0.0, 1.0 / self.gamma)

    def mu_inf(self) -> float:
        return 1.0 * self.mach * 1.0 / self.reynolds

    def t_inf(self) -> float:
        return (1.0 / self.gamma) / 1.0

    def conservative(self, mesh: TetMesh) -> np.ndarray:
        rho, u, v, w, p = self.freestream()
        return uniform_state(mesh.n_cells, rho=rho, vel=(u, v, w), p=p, gamma=self.gamma)


def tet_rule(npts: int):
    """Collapsed Gauss-Jacobi product rule on the reference tetrahedron.

    Returns (xyz [P,3] reference coordinates, w [P]) with sum(w) = 1/6; exact for
    polynomials of total degree <= 2*npts - 1.
    """
    ta, wa = _sp.roots_jacobi(npts, 2.0, 0.0)
    tb, wb = _sp.roots_jacobi(npts, 1.0, 0.0)
    tc, wc = _sp.roots_jacobi(npts, 0.0, 0.0)
    a, b, c = (ta + 1) / 2, (tb + 1) / 2, (tc + 1) / 2
    wa, wb, wc = wa / 8, wb / 4, wc / 2
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :]
    x = A
    y = (1 - A) * B
    z = (1 - A) * (1 - B) * C
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), W.ravel()


def default_npts(cell_vertices: np.ndarray, ksum: float) -> int:
    """Points per direction so that the rule error for sin(k.x) stays near 1e-15.

    ksum = sum_a |k_a| bounds the phase change per unit of per-axis extent; the
    Gauss error for an entire function of half-range r behaves like
    (r/2)^(2n) / (2n)!.
    """
    ext = float(np.max(np.ptp(cell_vertices[: min(len(cell_vertices), 4096)], axis=1)))
    r = 0.5 * ksum * ext
    for npts in range(2, 12):
        d = 2 * npts
        if (0.5 * r) ** d / math.factorial(d) < 1e-15:
            return npts
    return 12


def cell_average(cell_vertices: np.ndarray, fun, npts: int, chunk: int = 65536) -> np.ndarray:
    """Exact-to-rule cell averages of fun(x, y, z) -> [..] over every tetrahedron."""
    ref, w = tet_rule(npts)
    w6 = 6.0 * w
    nc = cell_vertices.shape[0]
    out = np.empty(nc, dtype=np.float64)
    refT = np.ascontiguousarray(ref.T)                                        # [3, P]
    for s in range(0, nc, chunk):
        v = cell_vertices[s:s + chunk]
        v0 = v[:, 0, :]
        e = v[:, 1:, :] - v0[:, None, :]                                      # [c, 3 edges, 3]
        x, y, z = (v0[:, d:d + 1] + e[:, :, d] @ refT for d in range(3))
        out[s:s + chunk] = fun(x, y, z) @ w6
    return out


@dataclass
class AdvectionCase:
    """rho = 1 + amp*sin(pi*(k.(x - U t)) + phase), velocity U, pressure p."""
    amp: float = 0.2
    k: tuple = (1.0, 1.0, 1.0)
    phase: float = 0.0
    vel: tuple = (1.0, 1.0, 1.0)
    p: float = 1.0
    gamma: float = 1.4

    def density_fn(self, t: float):
        kx, ky, kz = self.k
        ux, uy, uz = self.vel

        def f(x, y, z):
            return 1.0 + self.amp * np.sin(math.pi * (kx * (x - ux * t) + ky * (y - uy * t)
                                                      + kz * (z - uz * t)) + self.phase)
        return f

    def density_average(self, mesh: TetMesh, t: float = 0.0, npts: int | None = None) -> np.ndarray:
        if npts is None:
            npts = default_npts(mesh.cell_vertices, math.pi * sum(abs(v) for v in self.k))
        if mesh.cell_nodes.shape[1] == 8:
            # the trilinear Jacobian adds degree 2 per direction to the integrand
            return hex_cell_average(mesh.cell_vertices, self.density_fn(t), npts + 2)
        return cell_average(mesh.cell_vertices, self.density_fn(t), npts)

    def conservative(self, mesh: TetMesh, t: float = 0.0, npts: int | None = None) -> np.ndarray:
        """[n_cells, 5] cell averages of (rho, rho U, rho V, rho W, rho E)."""
        rho = self.density_average(mesh, t, npts)
        u = np.asarray(self.vel, dtype=np.float64)
        q = np.empty((rho.shape[0], 5))
        q[:, 0] = rho
        q[:, 1:4] = rho[:, None] * u[None, :]
        q[:, 4] = self.p / (self.gamma - 1.0) + 0.5 * rho * float(u @ u)
        return q


def uniform_state(n_cells: int, rho=1.0, vel=(0.3, -0.2, 0.5), p=1.0, gamma=1.4) -> np.ndarray:
    u = np.asarray(vel, dtype=np.float64)
    q = np.empty((n_cells, 5))
    q[:, 0] = rho
    q[:, 1:4] = rho * u
    q[:, 4] = p / (gamma - 1.0) + 0.5 * rho * float(u @ u)
    return q


@dataclass
class SodCase:
    """Sod's shock tube along x ((rho, p) = (1, 1) | (0.125, 0.1), zero velocity,
    gamma 1.4; the shock-tube workload of this build, not a case of the paper), laid
    out periodically: the high state fills
    [x0, x0 + half) of the period [0, 2 half) and the low state the rest, so the
    slab [x0 + half/2, x0 + 3 half/2) holds one standard tube with its diaphragm at
    x0 + half and the other half its mirror image.  Until the waves of the two
    diaphragms meet (t < half / (2 * shock speed), 0.286 for half = 1) the
    solution on each half equals the tube with transmissive ends.  Each cell takes
    the state on its centroid's side (no cut-cell averaging)."""
    rho_l: float = 1.0
    p_l: float = 1.0
    rho_r: float = 0.125
    p_r: float = 0.1
    x0: float = 0.5
    half: float = 1.0
    gamma: float = 1.4

    def high(self, x: np.ndarray) -> np.ndarray:
        xm = np.mod(x - self.x0, 2.0 * self.half)
        return xm < self.half

    def star(self):
        """Pressure and velocity between the waves: Newton's method on the pressure
        function of the exact Riemann solution (Toro, ch. 4)."""
        g = self.gamma
        rl, pl, rr, pr = self.rho_l, self.p_l, self.rho_r, self.p_r
        cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

        def fk(p, rk, pk, ck):
            if p > pk:                       # shock
                a = 2.0 / ((g + 1.0) * rk)
                b = (g - 1.0) / (g + 1.0) * pk
                return (p - pk) * math.sqrt(a / (p + b)), math.sqrt(a / (b + p)) * (1.0 - (p - pk) / (2.0 * (b + p)))
            e = (g - 1.0) / (2.0 * g)            # rarefaction
            return 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rk * ck)

        p = 0.5 * (pl + pr)
        for _ in range(100):
            f1, d1 = fk(p, rl, pl, cl)
            f2, d2 = fk(p, rr, pr, cr)
            dp = (f1 + f2) / (d1 + d2)
            p = max(1e-14, p - dp)
            if abs(dp) < 1e-15 * p:
                break
        f1, _ = fk(p, rl, pl, cl)
        f2, _ = fk(p, rr, pr, cr)
        return p, 0.5 * (f2 - f1)

    def exact(self, x: np.ndarray, t: float) -> np.ndarray:
        """(rho, u_x, p) of the exact solution at positions x (any half of the period):
        left rarefaction, contact, right shock, for this data at rest."""
        g = self.gamma
        rl, pl, rr, pr = self.rho_l, self.p_l, self.rho_r, self.p_r
        cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
        ps, us = self.star()
        xm = np.mod(np.asarray(x, dtype=np.float64) - self.x0, 2.0 * self.half)
        # distance from the nearest diaphragm, oriented from the high to the low state
        d = np.where(xm >= 0.5 * self.half * 3.0, xm - 2.0 * self.half,
                     np.where(xm < 0.5 * self.half, xm, xm - self.half))
        sign = np.where((xm >= 0.5 * self.half) & (xm < 1.5 * self.half), 1.0, -1.0)
        xi = sign * d / t
        head, tail = -cl, us - cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        shock = cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        rho_sl = rl * (ps / pl) ** (1.0 / g)
        rho_sr = rr * ((ps / pr + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * ps / pr + 1.0))
        c = 2.0 / (g + 1.0) * (cl - 0.5 * (g - 1.0) * xi)
        out = np.empty((xi.shape[0], 3))
        out[:, 0] = np.select([xi < head, xi < tail, xi < us, xi < shock],
                              [rl, rl * (np.abs(c) / cl) ** (2.0 / (g - 1.0)), rho_sl, rho_sr], rr)
        out[:, 1] = sign * np.select([xi < head, xi < tail, xi < shock], [0.0, 2.0 / (g + 1.0) * (cl + xi), us], 0.0)
        out[:, 2] = np.select([xi < head, xi < tail, xi < shock],
                              [pl, pl * (np.abs(c) / cl) ** (2.0 * g / (g - 1.0)), ps], pr)
        return out

    def conservative(self, mesh: TetMesh) -> np.ndarray:
        cx = mesh.cell_vertices[:, :, 0].mean(axis=1)
        hi = self.high(cx)
        rho = np.where(hi, self.rho_l, self.rho_r)
        p = np.where(hi, self.p_l, self.p_r)
        q = np.zeros((cx.shape[0], 5))
        q[:, 0] = rho
        q[:, 4] = p / (self.gamma - 1.0)
        return q


def sod_box(nx: int, ny: int, nz: int, jitter: float = 0.1, seed: int = SEED_ADVECTION + 7, walls: bool = False):
    """Sod's tube on jittered Kuhn tetrahedra.

    walls=False: the periodic doubled tube, [0, 2] x [0, ny h] x [0, nz h] with cubes of
    edge h = 2/nx, every axis periodic (each half is one tube until t = 0.286).
    walls=True: the tube itself, [0, 1] x [0, ny h] x [0, nz h] with h = 1/nx, the
    diaphragm at x = 0.5, transmissive walls at x = 0 and x = 1, y and z periodic."""
    if walls:
        h = 1.0 / nx
        mesh = kuhn_box((nx, ny, nz), (1.0, ny * h, nz * h), jitter, seed, periodic=(False, True, True))
        return mesh, SodCase(x0=-0.5)
    h = 2.0 / nx
    mesh = kuhn_box((nx, ny, nz), (2.0, ny * h, nz * h), jitter, seed)
    return mesh, SodCase()


def error_norms(mesh_volumes: np.ndarray, num: np.ndarray, exact: np.ndarray) -> dict:
    """Volume-weighted L1 / L2 / Linf of cell-average errors (not divided by |D|)."""
    e = num - exact
    return {"L1": float(np.sum(np.abs(e) * mesh_volumes)),
            "L2": float(np.sqrt(np.sum(e * e * mesh_volumes))),
            "Linf": float(np.max(np.abs(e)))}


def tet_volumes(cell_vertices: np.ndarray) -> np.ndarray:
    e = cell_vertices[:, 1:, :] - cell_vertices[:, :1, :]
    return np.abs(np.linalg.det(e)) / 6.0


def advection_config(n: int, seed_offset: int | None = None, jitter: float = 0.1):
    """The periodic accuracy-test box at resolution n (seed SEED+n unless given)."""
    seed = SEED_ADVECTION + (n if seed_offset is None else seed_offset)
    if n == 8 and seed_offset is None:
        seed = SEED_ADVECTION
    mesh = kuhn_box(n, 2.0, jitter, seed)
    case = AdvectionCase()
    return mesh, case


@dataclass
class Request:
    rid: int
    n: int
    seed: int
    case: AdvectionCase
    precision: int          # 0 = FP64, 1 = FP32-mixed
    steps: int
    arrival: float = 0.0


def serve_requests(count: int = 256, seed: int = 2407, n_range=(8, 48), steps: int = 200,
                   rate: float = 1.0) -> list:
    """Seeded request stream: Kuhn boxes of 6 N^3 cells with random smooth data.

    N ~ U{n_range}, amplitude ~ U[0.05, 0.2], k in {1,2}^3, phase ~ U[0, 2pi),
    Mach ~ U[0.1, 2.0] along a direction uniform on the sphere, p = 1,
    precision ~ Bernoulli(1/2), Poisson arrivals at `rate` per second.
    """
    u = uniform01(seed, 16 * count).reshape(count, 16)
    reqs = []
    t = 0.0
    for r in range(count):
        row = u[r]
        n = n_range[0] + int(row[0] * (n_range[1] - n_range[0] + 1))
        amp = 0.05 + 0.15 * row[1]
        k = tuple(1.0 + float(row[2 + a] >= 0.5) for a in range(3))
        phase = 2 * math.pi * row[5]
        mach = 0.1 + 1.9 * row[6]
        cz = 2 * row[7] - 1
        ph = 2 * math.pi * row[8]
        sz = math.sqrt(max(0.0, 1 - cz * cz))
        d = (sz * math.cos(ph), sz * math.sin(ph), cz)
        c = math.sqrt(1.4)            # sound speed at rho = 1, p = 1
        vel = tuple(mach * c * x for x in d)
        prec = int(row[9] >= 0.5)
        t += -math.log(max(1e-300, 1.0 - row[10])) / rate
        reqs.append(Request(rid=r, n=n, seed=seed * 1000003 + r, precision=prec, steps=steps,
                            case=AdvectionCase(amp=amp, k=k, phase=phase, vel=vel), arrival=t))
    return reqs
