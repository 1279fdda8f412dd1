"""Thin Python binding of libhgks.so (the C ABI declared in include/hgks.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels (and its host-side mesh precompute).  Raises if the library is not
built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhgks.so")

OK, E_INVALID_ARG, E_BAD_MESH, E_STATE, E_OOM, E_DEVICE, E_NONPHYSICAL = range(7)
FP64, FP32_MIXED, FP32 = 0, 1, 2
ACC_GATHER, ACC_COLOURED = 0, 1
BC_WALL, BC_FAR = 1, 2
KERNEL_IDS = {"dt": 0, "weno": 1, "flux": 2, "update": 3}

_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "BAD_MESH", 3: "STATE", 4: "OOM", 5: "DEVICE", 6: "NONPHYSICAL"}


class HGKSError(RuntimeError):
    def __init__(self, status, message=""):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("tau_mode", C.c_int),
                ("tau_eps", C.c_double), ("tau_C", C.c_double), ("weno_eps", C.c_double),
                ("gamma_lin", C.c_double), ("precision", C.c_int), ("accumulation", C.c_int),
                ("reorder", C.c_int), ("mu_ref", C.c_double), ("T_ref", C.c_double), ("mu_exp", C.c_double),
                ("prandtl", C.c_double), ("farfield", C.c_double * 5)]


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_lib = None


def lib():
    """Loads libhgks.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        L.hgks_default_params.argtypes = [C.POINTER(Params)]
        L.hgks_create.argtypes = [C.POINTER(Params), C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
        L.hgks_mesh_upload.argtypes = [C.c_void_p, C.c_int64, _dp, C.c_int64, C.c_int, _i64p, _dp, C.c_int64,
                                       _i64p, _i32p]
        L.hgks_init_state.argtypes = [C.c_void_p, _dp, C.c_double]
        L.hgks_step_s2o4.argtypes = [C.c_void_p, C.c_int32, C.c_double, _dp]
        L.hgks_get_state.argtypes = [C.c_void_p, _dp, _dp]
        L.hgks_sync.argtypes = [C.c_void_p]
        L.hgks_mesh_info.argtypes = [C.c_void_p, _i64p, _i64p, _i32p, _i32p]
        L.hgks_footprint.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.hgks_profile_enable.argtypes = [C.c_void_p, C.c_int]
        L.hgks_profile_read.argtypes = [C.c_void_p, C.c_int, _dp, _i64p]
        L.hgks_profile_reset.argtypes = [C.c_void_p]
        L.hgks_last_error.restype = C.c_char_p
        L.hgks_last_error.argtypes = [C.c_void_p]
        L.hgks_destroy.argtypes = [C.c_void_p]
        L.hgks_inspect_mesh.argtypes = [C.POINTER(Params), C.c_int64, _dp, C.c_int64, C.c_int, _i64p, _dp, _dp,
                                        _i64p, _i32p]
        L.hgks_pool_create.argtypes = [C.c_int, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]
        L.hgks_pool_footprint.argtypes = [C.POINTER(Params), C.c_int64, C.c_int, C.POINTER(C.c_size_t)]
        L.hgks_pool_add.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]
        L.hgks_pool_step.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.c_int32]
        L.hgks_pool_step_static.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.c_int32]
        L.hgks_pool_remove.argtypes = [C.c_void_p, C.c_int]
        L.hgks_pool_used.argtypes = [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int)]
        L.hgks_pool_destroy.argtypes = [C.c_void_p]
        for name in ("hgks_create", "hgks_mesh_upload", "hgks_init_state", "hgks_step_s2o4", "hgks_get_state",
                     "hgks_sync", "hgks_mesh_info", "hgks_footprint", "hgks_profile_enable", "hgks_profile_read",
                     "hgks_profile_reset", "hgks_inspect_mesh", "hgks_pool_create", "hgks_pool_footprint",
                     "hgks_pool_add", "hgks_pool_step", "hgks_pool_step_static", "hgks_pool_remove", "hgks_pool_used"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def params(**kw) -> Params:
    p = Params()
    lib().hgks_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        if k == "farfield":
            p.farfield[:] = tuple(float(x) for x in v)
        else:
            setattr(p, k, v)
    return p


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


OWN_STREAM = "own"


def _stream_handle(stream):
    """None: the device's null stream; "own": a stream the context (pool) creates and
    destroys (HGKS_OWN_STREAM); an int: a hipStream_t handle."""
    if stream is None:
        return None
    if stream == OWN_STREAM:
        return 1
    if isinstance(stream, int):
        return stream
    raise TypeError(f"stream must be None, 'own' or a hipStream_t handle, got {stream!r}")


class Solver:
    """One HGKS problem on one GPU (hgks_ctx)."""

    def __init__(self, prm: Params | None = None, device: int = 0, stream=None):
        L = lib()
        self.params = prm if prm is not None else params()
        h = C.c_void_p()
        st = L.hgks_create(C.byref(self.params), int(device), _stream_handle(stream), None, C.byref(h))
        if st != OK:
            raise HGKSError(st, "hgks_create failed")
        self._h = h
        self.device = device
        self.n_cells = 0

    def _check(self, st):
        if st != OK:
            raise HGKSError(st, lib().hgks_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().hgks_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def mesh_upload(self, nodes, cell_nodes, period=(0.0, 0.0, 0.0), bfaces=None, bkinds=None):
        """cell_nodes [n, 4] (tetrahedra) or [n, 8] (hexahedra); bfaces [nb, 4] node ids
        of listed boundary faces with bkinds [nb] (BC_WALL / BC_FAR), hexahedra only."""
        nodes = _f64(nodes)
        cells = np.ascontiguousarray(cell_nodes, dtype=np.int64)
        per = _f64(period)
        if bfaces is None:
            nb, bf, bk = 0, None, None
        else:
            bf_a = np.ascontiguousarray(bfaces, dtype=np.int64)
            bk_a = np.ascontiguousarray(bkinds, dtype=np.int32)
            if bk_a.shape[0] != bf_a.shape[0]:
                raise ValueError("one kind per boundary face")
            nb, bf, bk = bf_a.shape[0], bf_a.ctypes.data_as(_i64p), bk_a.ctypes.data_as(_i32p)
        self._check(lib().hgks_mesh_upload(self._h, nodes.shape[0], nodes.ctypes.data_as(_dp), cells.shape[0],
                                           cells.shape[1], cells.ctypes.data_as(_i64p), per.ctypes.data_as(_dp),
                                           nb, bf, bk))
        self.n_cells = cells.shape[0]

    def upload(self, mesh):
        """mesh_upload of a workload mesh (nodes, cell_nodes, period, listed boundary faces)."""
        self.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period, getattr(mesh, "bfaces", None),
                         getattr(mesh, "bkinds", None))

    def init_state(self, q, t0: float = 0.0):
        q = _f64(q)
        if self.n_cells and q.size != 5 * self.n_cells:
            raise ValueError(f"state must hold {self.n_cells} x 5 values, got shape {q.shape}")
        self._check(lib().hgks_init_state(self._h, q.ctypes.data_as(_dp), float(t0)))

    def step(self, nsteps: int = 1, dt_fixed: float = 0.0, want_dt: bool = False):
        dt = C.c_double(0.0)
        self._check(lib().hgks_step_s2o4(self._h, int(nsteps), float(dt_fixed), C.byref(dt) if want_dt else None))
        return dt.value if want_dt else None

    def get_state(self):
        q = np.empty((self.n_cells, 5))
        t = C.c_double(0.0)
        self._check(lib().hgks_get_state(self._h, q.ctypes.data_as(_dp), C.byref(t)))
        return q, t.value

    def get_time(self) -> float:
        """The simulated time (and the non-physical check) without reading the state back."""
        t = C.c_double(0.0)
        self._check(lib().hgks_get_state(self._h, None, C.byref(t)))
        return t.value

    def sync(self):
        self._check(lib().hgks_sync(self._h))

    def info(self):
        nc, nf = C.c_int64(), C.c_int64()
        sl, col = C.c_int32(), C.c_int32()
        self._check(lib().hgks_mesh_info(self._h, C.byref(nc), C.byref(nf), C.byref(sl), C.byref(col)))
        return {"n_cells": nc.value, "n_faces": nf.value, "slots": sl.value, "colours": col.value}

    def footprint(self) -> int:
        b = C.c_size_t()
        self._check(lib().hgks_footprint(self._h, C.byref(b)))
        return b.value

    def profile_enable(self, on=True):
        self._check(lib().hgks_profile_enable(self._h, int(on)))

    def profile_reset(self):
        self._check(lib().hgks_profile_reset(self._h))

    def profile_read(self, kernel: str):
        ms, n = C.c_double(), C.c_int64()
        self._check(lib().hgks_profile_read(self._h, KERNEL_IDS[kernel], C.byref(ms), C.byref(n)))
        return ms.value, n.value


def inspect_mesh(nodes, cell_nodes, period=(0.0, 0.0, 0.0), prm: Params | None = None):
    """Host-only view of the library's mesh precompute (no GPU needed)."""
    nodes = _f64(nodes)
    cells = np.ascontiguousarray(cell_nodes, dtype=np.int64)
    per = _f64(period)
    nc = cells.shape[0]
    stats = np.zeros(8)
    perm = np.empty(nc, dtype=np.int64)

    def call(sten):
        return lib().hgks_inspect_mesh(C.byref(prm) if prm is not None else None, nodes.shape[0],
                                       nodes.ctypes.data_as(_dp), nc, cells.shape[1], cells.ctypes.data_as(_i64p),
                                       per.ctypes.data_as(_dp), stats.ctypes.data_as(_dp), perm.ctypes.data_as(_i64p),
                                       sten.ctypes.data_as(_i32p) if sten is not None else None)
    if cells.shape[1] == 8:
        st = call(None)                    # the slot count first
        sten = np.empty((int(stats[1]) if st == OK else 0, nc), dtype=np.int32)
        if st == OK:
            st = call(sten)
    else:
        sten = np.empty((16, nc), dtype=np.int32)
        st = call(sten)
    if st != OK:
        raise HGKSError(st, "hgks_inspect_mesh failed")
    keys = ["n_faces", "slots", "max_members", "min_members", "n_colours", "pinv_residual", "closure", "dup_slots"]
    return {"stats": dict(zip(keys, stats.tolist())), "perm": perm, "sten": sten}


def pool_footprint(prm: Params, n_cells: int) -> int:
    b = C.c_size_t()
    st = lib().hgks_pool_footprint(C.byref(prm), int(n_cells), 4, C.byref(b))
    if st != OK:
        raise HGKSError(st, "hgks_pool_footprint failed")
    return b.value


class Pool:
    """Continuous batching of many Solvers on one GPU (hgks_pool)."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        h = C.c_void_p()
        st = lib().hgks_pool_create(int(device), _stream_handle(stream), C.c_size_t(hbm_budget), C.byref(h))
        if st != OK:
            raise HGKSError(st, "hgks_pool_create failed")
        self._h = h

    def add(self, solver: Solver) -> int:
        s = C.c_int()
        st = lib().hgks_pool_add(self._h, solver._h, C.byref(s))
        if st != OK:
            raise HGKSError(st, "hgks_pool_add failed")
        return s.value

    def step(self, slots, nsteps: int = 1):
        arr = (C.c_int * len(slots))(*slots)
        st = lib().hgks_pool_step(self._h, arr, len(slots), int(nsteps))
        if st != OK:
            raise HGKSError(st, "hgks_pool_step failed")

    def step_static(self, slots, nsteps: int = 1):
        """hgks_pool_step_static: the same step with the launch tables in the library's
        static per-GPU array (no device allocation)."""
        arr = (C.c_int * len(slots))(*slots)
        st = lib().hgks_pool_step_static(self._h, arr, len(slots), int(nsteps))
        if st != OK:
            raise HGKSError(st, "hgks_pool_step_static failed")

    def remove(self, slot: int):
        st = lib().hgks_pool_remove(self._h, int(slot))
        if st != OK:
            raise HGKSError(st, "hgks_pool_remove failed")

    def used(self):
        b, n = C.c_size_t(), C.c_int()
        lib().hgks_pool_used(self._h, C.byref(b), C.byref(n))
        return b.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().hgks_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
