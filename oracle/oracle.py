"""ctypes wrapper of the FP64 CPU oracle (hgks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hgks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_ip = C.POINTER(C.c_int)


def build() -> str:
    """Compile the oracle with gcc: -O2, no contraction into FMA, no fast-math.

    OpenMP is enabled; the thread count (OMP_NUM_THREADS) changes only the speed,
    never the result (every parallel loop writes disjoint slots in a fixed order).
    """
    out = LIB
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", SRC,
           "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("tau_mode", C.c_int),
                ("tau_eps", C.c_double), ("tau_C", C.c_double), ("weno_eps", C.c_double),
                ("gamma_lin", C.c_double), ("mu_ref", C.c_double), ("T_ref", C.c_double),
                ("mu_exp", C.c_double), ("prandtl", C.c_double), ("farfield", C.c_double * 5)]


# boundary kinds of listed boundary faces
BC_WALL = 1     # no-slip adiabatic wall
BC_FAR = 2      # far field (Riemann invariants)


def default_params(**kw) -> Params:
    p = Params(gamma=1.4, cfl=0.3, tau_mode=0, tau_eps=0.05, tau_C=1.0, weno_eps=1e-8, gamma_lin=0.025,
               mu_ref=0.0, T_ref=1.0, mu_exp=0.7, prandtl=1.0)
    p.farfield[:] = (1.0, 0.0, 0.0, 0.0, 1.0)
    for k, v in kw.items():
        if k == "farfield":
            p.farfield[:] = tuple(float(x) for x in v)
        else:
            setattr(p, k, v)
    return p


_lib = None


def _configure(L):
    """Declares the argument and return types of the oracle's C entry points."""
    L.orc_mesh_new.restype = C.c_void_p
    L.orc_mesh_new.argtypes = [C.c_int64, _dp, C.c_int64, _i64p, _dp, C.c_char_p, C.c_int]
    L.orc_mesh_new2.restype = C.c_void_p
    L.orc_mesh_new2.argtypes = [C.c_int64, _dp, C.c_int64, C.c_int, _i64p, _dp, C.c_int64, _i64p, _ip,
                                C.c_char_p, C.c_int]
    L.orc_mesh_info.argtypes = [C.c_void_p, _i64p]
    L.orc_mesh_face_points.argtypes = [C.c_void_p, _dp, _dp, _ip]
    L.orc_ghost_state.argtypes = [C.POINTER(Params), C.c_int, _dp, _dp, _dp]
    L.orc_mesh_free.argtypes = [C.c_void_p]
    L.orc_mesh_nfaces.restype = C.c_int64
    L.orc_mesh_nfaces.argtypes = [C.c_void_p]
    L.orc_mesh_cells.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_mesh_faces.argtypes = [C.c_void_p, _i64p, _dp, _dp, _dp, _dp]
    L.orc_mesh_stencil.restype = C.c_int
    L.orc_mesh_stencil.argtypes = [C.c_void_p, C.c_int64, _i64p, _dp, _ip, _i64p]
    L.orc_mesh_neighbors.argtypes = [C.c_void_p, _i64p]
    L.orc_gks_flux.restype = C.c_int
    L.orc_gks_flux.argtypes = [C.POINTER(Params), _dp, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp]
    L.orc_rhs.restype = C.c_int
    L.orc_rhs.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_double, _dp, _dp]
    L.orc_cfl_dt.restype = C.c_double
    L.orc_cfl_dt.argtypes = [C.c_void_p, C.POINTER(Params), _dp]
    L.orc_s2o4_stage1.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, _dp]
    L.orc_s2o4_stage2.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, _dp]
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_int, C.c_double, _dp]
    L.orc_moments_1d.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp]
    L.orc_slope.restype = C.c_int
    L.orc_slope.argtypes = [C.c_double] * 5 + [_dp, _dp]
    L.orc_collision.argtypes = [C.POINTER(Params), _dp, _dp, _dp]
    L.orc_weno_cell.restype = C.c_int
    L.orc_weno_cell.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_int64, _dp, _dp, _dp, _dp]
    L.orc_reconstruct.restype = C.c_int
    L.orc_reconstruct.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_int64, _dp, _dp, _dp]
    L.orc_cell_monomial_means.argtypes = [C.c_void_p, C.c_int64, _dp, C.c_double, _dp]
    L.orc_face_flux.restype = C.c_int
    L.orc_face_flux.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_int64, C.c_double, _dp]
    L.orc_fallback_census.restype = C.c_int
    L.orc_fallback_census.argtypes = [C.c_void_p, C.POINTER(Params), _dp, _i64p]
    L.orc_threads.restype = C.c_int
    L.orc_step_sample.restype = C.c_int
    L.orc_step_sample.argtypes = [C.c_void_p, C.POINTER(Params), _dp, C.c_double, C.c_int64, _i64p, _dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _configure(C.CDLL(LIB))
    return _lib


def build_variant(src: str, out: str):
    """Compiles a variant of the oracle source (the tests plant mistakes in copies
    to show that the pins catch them) with the oracle's own flags and loads it."""
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return _configure(C.CDLL(out))


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    pass


class Mesh:
    """Oracle-side mesh: connectivity, geometry and stencils built from nodes + cells."""

    def __init__(self, nodes, cell_nodes, period=(0.0, 0.0, 0.0), bfaces=None, bkinds=None):
        """cell_nodes [nc][4] (tetrahedra) or [nc][8] (hexahedra); bfaces [nb][3 or 4]
        node ids of listed boundary faces with bkinds [nb] (BC_WALL / BC_FAR)."""
        L = lib()
        self.nodes = _f64(nodes)
        self.cell_nodes = np.ascontiguousarray(cell_nodes, dtype=np.int64)
        self.period = _f64(period)
        npc = self.cell_nodes.shape[1]
        err = C.create_string_buffer(256)
        if bfaces is None:
            bf = np.zeros((0, 4), dtype=np.int64)
            bk = np.zeros(0, dtype=np.int32)
        else:
            bf = np.ascontiguousarray(bfaces, dtype=np.int64)
            bk = np.ascontiguousarray(bkinds, dtype=np.int32)
        self._bf, self._bk = bf, bk
        self._h = L.orc_mesh_new2(self.nodes.shape[0], _d(self.nodes), self.cell_nodes.shape[0], npc,
                                  self.cell_nodes.ctypes.data_as(_i64p), _d(self.period), bf.shape[0],
                                  bf.ctypes.data_as(_i64p), bk.ctypes.data_as(_ip), err, 256)
        if not self._h:
            raise OracleError(err.value.decode())
        self.nc = self.cell_nodes.shape[0]
        self.nf = int(L.orc_mesh_nfaces(self._h))
        info = np.zeros(6, dtype=np.int64)
        L.orc_mesh_info(self._h, info.ctypes.data_as(_i64p))
        self.npc, self.nfc, self.ngp, self.msub, self.n_ghosts, self.max_stencil = (int(x) for x in info)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_mesh_free(h)
            self._h = None

    @classmethod
    def from_workload(cls, mesh):
        return cls(mesh.nodes, mesh.cell_nodes, mesh.period, getattr(mesh, "bfaces", None),
                   getattr(mesh, "bkinds", None))

    def cells(self):
        vol, cen, hdt = np.empty(self.nc), np.empty((self.nc, 3)), np.empty(self.nc)
        lib().orc_mesh_cells(self._h, _d(vol), _d(cen), _d(hdt))
        return vol, cen, hdt

    def faces(self):
        lr = np.empty((self.nf, 2), dtype=np.int64)
        nrm, area = np.empty((self.nf, 3)), np.empty(self.nf)
        shift, gp = np.empty((self.nf, 3)), np.empty((self.nf, self.ngp, 3))
        lib().orc_mesh_faces(self._h, lr.ctypes.data_as(_i64p), _d(nrm), _d(area), _d(shift), _d(gp))
        pn, pw = np.empty((self.nf, self.ngp, 3)), np.empty((self.nf, self.ngp))
        kind = np.empty(self.nf, dtype=np.int32)
        lib().orc_mesh_face_points(self._h, _d(pn), _d(pw), kind.ctypes.data_as(_ip))
        return {"lr": lr, "normal": nrm, "area": area, "shift": shift, "gauss": gp,
                "point_normal": pn, "point_weight": pw, "kind": kind}

    def neighbors(self):
        nb = np.empty((self.nc, self.nfc), dtype=np.int64)
        lib().orc_mesh_neighbors(self._h, nb.ctypes.data_as(_i64p))
        return nb

    def stencil(self, i):
        """(members, offsets, sub-stencils); member ids >= nc are boundary ghosts."""
        mem = np.empty(40, dtype=np.int64)
        sh = np.empty((40, 3))
        ns = np.empty(8, dtype=np.int32)
        sub = np.empty((8, 8), dtype=np.int64)
        k = lib().orc_mesh_stencil(self._h, int(i), mem.ctypes.data_as(_i64p), _d(sh),
                                   ns.ctypes.data_as(_ip), sub.ctypes.data_as(_i64p))
        return mem[:k].copy(), sh[:k].copy(), [sub[s, :ns[s]].copy() for s in range(self.msub)]

    def monomial_means(self, i, center, h):
        out = np.empty(9)
        c = _f64(center)
        lib().orc_cell_monomial_means(self._h, int(i), _d(c), float(h), _d(out))
        return out

    # --- the method -------------------------------------------------------
    def rhs(self, q, dt, params=None):
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        L, dL = np.empty_like(q), np.empty_like(q)
        rc = lib().orc_rhs(self._h, C.byref(p), _d(q), float(dt), _d(L), _d(dL))
        if rc:
            raise OracleError(f"orc_rhs failed ({rc})")
        return L, dL

    def cfl_dt(self, q, params=None):
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        return float(lib().orc_cfl_dt(self._h, C.byref(p), _d(q)))

    def step(self, q, nsteps=1, dt_fixed=0.0, params=None):
        """Returns (q_new, dt_last)."""
        p = params or default_params()
        q = _f64(q, (self.nc, 5)).copy()
        dt = C.c_double(0.0)
        rc = lib().orc_step(self._h, C.byref(p), _d(q), int(nsteps), float(dt_fixed), C.byref(dt))
        if rc:
            raise OracleError(f"orc_step failed ({rc})")
        return q, dt.value

    def step_sample(self, q, dt, cells, params=None):
        """Q^{n+1} of the listed cells after one step of size dt (same arithmetic as step)."""
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((cells.shape[0], 5))
        rc = lib().orc_step_sample(self._h, C.byref(p), _d(q), float(dt), cells.shape[0],
                                   cells.ctypes.data_as(_i64p), _d(out))
        if rc:
            raise OracleError(f"orc_step_sample failed ({rc})")
        return out

    def face_flux(self, q, f, dt, params=None):
        """S * sum_G w_G (F, dF/dt) of face f, 10 values (global frame)."""
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        out = np.empty(10)
        rc = lib().orc_face_flux(self._h, C.byref(p), _d(q), int(f), float(dt), _d(out))
        if rc:
            raise OracleError(f"orc_face_flux failed ({rc})")
        return out

    def fallback_census(self, q, params=None):
        """Gauss points where the positivity fallback acts: (all, one-sided, one-sided
        with a nonzero gradient on the physical side)."""
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        out = np.zeros(3, dtype=np.int64)
        rc = lib().orc_fallback_census(self._h, C.byref(p), _d(q), out.ctypes.data_as(_i64p))
        if rc:
            raise OracleError(f"orc_fallback_census failed ({rc})")
        return tuple(int(x) for x in out)

    def weno_cell(self, q, i, params=None):
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        M = self.msub
        a, b = np.empty((5, 9)), np.empty((M, 5, 3))
        beta, wbar = np.empty((5, M + 1)), np.empty((5, M + 1))
        rc = lib().orc_weno_cell(self._h, C.byref(p), _d(q), int(i), _d(a), _d(b), _d(beta), _d(wbar))
        if rc:
            raise OracleError(f"orc_weno_cell failed ({rc})")
        return {"a": a, "b": b, "beta": beta, "wbar": wbar}

    def reconstruct(self, q, i, x, params=None):
        p = params or default_params()
        q = _f64(q, (self.nc, 5))
        x = _f64(x)
        val, grad = np.empty(5), np.empty((5, 3))
        rc = lib().orc_reconstruct(self._h, C.byref(p), _d(q), int(i), _d(x), _d(val), _d(grad))
        if rc:
            raise OracleError(f"orc_reconstruct failed ({rc})")
        return val, grad


def threads() -> int:
    return int(lib().orc_threads())


def gks_flux(ql, gl, qr, gr, n, dt, params=None):
    p = params or default_params()
    ql, gl, qr, gr, n = (_f64(x) for x in (ql, gl, qr, gr, n))
    F, dF = np.empty(5), np.empty(5)
    rc = lib().orc_gks_flux(C.byref(p), _d(ql), _d(gl), _d(qr), _d(gr), _d(n), float(dt), _d(F), _d(dF))
    if rc:
        raise OracleError(f"orc_gks_flux failed ({rc})")
    return F, dF


def moments_1d(U, lam):
    full, pos, neg = np.empty(7), np.empty(7), np.empty(7)
    lib().orc_moments_1d(float(U), float(lam), _d(full), _d(pos), _d(neg))
    return full, pos, neg


def slope(U, V, W, lam, K, b):
    b = _f64(b)
    a = np.empty(5)
    rc = lib().orc_slope(float(U), float(V), float(W), float(lam), float(K), _d(b), _d(a))
    if rc:
        raise OracleError("singular moment matrix")
    return a


def ghost_state(kind, q, n, params=None):
    """The state a boundary ghost of `kind` holds next to state q (outward normal n)."""
    p = params or default_params()
    q, n = _f64(q), _f64(n)
    out = np.empty(5)
    lib().orc_ghost_state(C.byref(p), int(kind), _d(q), _d(n), _d(out))
    return out


def collision(ql, qr, params=None):
    p = params or default_params()
    ql, qr = _f64(ql), _f64(qr)
    q0 = np.empty(5)
    lib().orc_collision(C.byref(p), _d(ql), _d(qr), _d(q0))
    return q0


def s2o4_stage1(q, L, dL, dt):
    q, L, dL = (_f64(x) for x in (q, L, dL))
    out = np.empty_like(q)
    lib().orc_s2o4_stage1(q.size, _d(q), _d(L), _d(dL), float(dt), _d(out))
    return out


def s2o4_stage2(q, L, dL, dLs, dt):
    q, L, dL, dLs = (_f64(x) for x in (q, L, dL, dLs))
    out = np.empty_like(q)
    lib().orc_s2o4_stage2(q.size, _d(q), _d(L), _d(dL), _d(dLs), float(dt), _d(out))
    return out
