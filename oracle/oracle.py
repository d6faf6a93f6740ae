"""ctypes binding of the reference oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the oracle is the plain sequential FP64
transcription of the paper's time loop that the GPU library is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  Nothing here touches the GPU library.

The binding takes any object with the attributes of a workload problem
(dim, n, lo, hi, faces, x, v, mass, rho, eint, ids, shape, av_form, gamma,
c0, c1, cfl, inflow_*, recycle_mass, seed, t_end, gradv, cell_mask,
node_normal) and returns plain numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "mpm_oracle.c")]

F_X, F_V, F_M, F_RHO, F_E, F_P, F_Q, F_G, F_VOL, F_VBAR = range(10)
G_M, G_P, G_F, G_PUPD, G_P2, G_FBC = range(6)


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("shape", C.c_int32), ("av_form", C.c_int32),
        ("gamma", C.c_double), ("c0", C.c_double), ("c1", C.c_double), ("cfl", C.c_double),
        ("face", (C.c_int32 * 2) * 3),
        ("inflow_rho", C.c_double), ("inflow_p", C.c_double), ("inflow_u", C.c_double * 3),
        ("recycle_mass", C.c_double),
        ("seed", C.c_uint64),
        ("t_end", C.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2, no fast-math; OpenMP
    for the optional multi-threaded loops)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", LIB_PATH] + SOURCES + ["-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(_Problem), C.c_int64, C.POINTER(dp), C.POINTER(dp),
                                 dp, dp, dp, C.POINTER(dp), C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_uint8), C.POINTER(dp), C.POINTER(C.c_void_p)]
        L.orc_create.restype = C.c_int
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_set_dt.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_threads.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_fp32_state.argtypes = [C.c_void_p, C.c_int]
        L.orc_projected.argtypes = [C.c_void_p, dp, dp]
        L.orc_get_particles.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_get_grid.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_grid_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.orc_status.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(C.c_int64), dp,
                                 C.POINTER(C.c_int64)]
        L.orc_basis_1d.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int32), dp, dp]
        L.orc_artificial_viscosity.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                               C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_artificial_viscosity.restype = C.c_double
        L.orc_obstacle_project.argtypes = [C.c_int, dp, dp]
        L.orc_nodal_gradient.argtypes = [C.POINTER(_Problem), C.POINTER(dp), dp, dp]
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_problem(pb) -> _Problem:
    s = _Problem()
    s.dim = pb.dim
    for a in range(3):
        s.n[a] = int(pb.n[a])
        s.lo[a] = float(pb.lo[a])
        s.hi[a] = float(pb.hi[a])
        s.face[a][0] = int(pb.faces[a][0])
        s.face[a][1] = int(pb.faces[a][1])
        s.inflow_u[a] = float(pb.inflow_u[a])
    s.shape = pb.shape
    s.av_form = pb.av_form
    s.gamma, s.c0, s.c1, s.cfl = pb.gamma, pb.c0, pb.c1, pb.cfl
    s.inflow_rho, s.inflow_p = pb.inflow_rho, pb.inflow_p
    s.recycle_mass = pb.recycle_mass
    s.seed = int(pb.seed) & 0xFFFFFFFFFFFFFFFF
    s.t_end = pb.t_end
    return s


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


class Oracle:
    """One oracle simulation built from a workload problem.  `threads` > 1
    runs its loops on that many OpenMP threads (the P2G sums then differ from
    the single-thread order by FP64 rounding)."""

    def __init__(self, pb, threads: int = 1):
        L = lib()
        self.pb = pb
        self.dim = pb.dim
        self.np = int(pb.mass.shape[0])
        self._keep = []
        dp = C.POINTER(C.c_double)

        def arrs(mat, count):
            mat = np.ascontiguousarray(mat, dtype=np.float64)
            self._keep.append(mat)
            return (dp * count)(*[_dptr(mat[c]) for c in range(count)])

        x = arrs(pb.x, self.dim)
        v = arrs(pb.v, self.dim)
        gradv = None
        if pb.gradv is not None:
            gradv = arrs(pb.gradv, self.dim * self.dim)
        scal = []
        for a in (pb.mass, pb.rho, pb.eint):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self._keep.append(a)
            scal.append(_dptr(a))
        ids = np.ascontiguousarray(pb.ids, dtype=np.uint32)
        self._keep.append(ids)
        mask_p = None
        nrm = None
        if pb.cell_mask is not None:
            mask = np.ascontiguousarray(pb.cell_mask, dtype=np.uint8)
            self._keep.append(mask)
            mask_p = mask.ctypes.data_as(C.POINTER(C.c_uint8))
            nrm = arrs(pb.node_normal, self.dim)
        self._prob = make_problem(pb)
        h = C.c_void_p()
        rc = L.orc_create(C.byref(self._prob), self.np, x, v, scal[0], scal[1], scal[2],
                          gradv, ids.ctypes.data_as(C.POINTER(C.c_uint32)), mask_p, nrm,
                          C.byref(h))
        self._keep = []
        if rc != 0:
            raise OracleError(rc, "orc_create")
        self._h = h
        shp = (C.c_int32 * 3)()
        L.orc_grid_shape(self._h, shp)
        self.nodes = tuple(int(v) for v in shp)
        self.nnodes = int(np.prod(self.nodes))
        self.threads = 1
        if threads > 1:
            rc = L.orc_set_threads(self._h, int(threads))
            if rc:
                raise OracleError(rc, "orc_set_threads")
            self.threads = int(threads)

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int = 1) -> int:
        return lib().orc_step(self._h, int(n))

    def set_fp32_state(self, on: bool = True):
        """Round the particle state to FP32 now and after every step (the
        arithmetic stays FP64): the effect of FP32 storage alone."""
        rc = lib().orc_set_fp32_state(self._h, int(bool(on)))
        if rc:
            raise OracleError(rc, "orc_set_fp32_state")

    def set_dt(self, dt: float):
        rc = lib().orc_set_dt(self._h, float(dt))
        if rc:
            raise OracleError(rc, "orc_set_dt")

    _NCOMP = {F_X: "d", F_V: "d", F_VBAR: "d", F_G: "dd"}

    def particles(self, field: int) -> np.ndarray:
        nc = {"d": self.dim, "dd": self.dim * self.dim}.get(self._NCOMP.get(field), 1)
        out = np.empty((nc, self.np))
        rc = lib().orc_get_particles(self._h, field, _dptr(out))
        if rc:
            raise OracleError(rc, "orc_get_particles")
        return out if nc > 1 else out[0]

    def grid(self, which: int) -> np.ndarray:
        nc = 1 if which == G_M else self.dim
        out = np.empty((nc, self.nnodes))
        rc = lib().orc_get_grid(self._h, which, _dptr(out))
        if rc:
            raise OracleError(rc, "orc_get_grid")
        return out if nc > 1 else out[0]

    def projected(self):
        """P2G of the masses and of the volumes M / rho at the current
        positions: (mass, vol) over the nodes; density = mass / vol."""
        m = np.empty(self.nnodes)
        v = np.empty(self.nnodes)
        rc = lib().orc_projected(self._h, _dptr(m), _dptr(v))
        if rc:
            raise OracleError(rc, "orc_projected")
        return m, v

    def status(self) -> dict:
        t, dtn, dtl = C.c_double(), C.c_double(), C.c_double()
        step, esc = C.c_int64(), C.c_int64()
        cons = (C.c_double * 6)()
        rc = lib().orc_status(self._h, C.byref(t), C.byref(dtn), C.byref(dtl), C.byref(step),
                              cons, C.byref(esc))
        return dict(t=t.value, dt_next=dtn.value, dt_last=dtl.value, step=step.value,
                    conserved=np.array(list(cons)), wall_escapes=esc.value, rc=rc)


def basis_1d(shape: int, n: int, s: float):
    first = C.c_int32()
    w = (C.c_double * 3)()
    dw = (C.c_double * 3)()
    width = lib().orc_basis_1d(shape, n, s, C.byref(first), w, dw)
    return first.value, np.array(w[:width]), np.array(dw[:width])


def artificial_viscosity(av_form, c0, c1, gamma, h, rho, p, divv) -> float:
    return lib().orc_artificial_viscosity(av_form, c0, c1, gamma, h, rho, p, divv)


def obstacle_project(normal, u):
    n = np.ascontiguousarray(normal, dtype=np.float64)
    out = np.array(u, dtype=np.float64)
    lib().orc_obstacle_project(len(out), _dptr(n), _dptr(out))
    return out


def nodal_gradient(pb, u: np.ndarray, point) -> np.ndarray:
    """G[a, b] = sum_i u_a(i) d_b phi_i(point) for a nodal field u (dim, nodes)."""
    dim = pb.dim
    u = np.ascontiguousarray(u, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    ptrs = (dp * dim)(*[_dptr(u[a]) for a in range(dim)])
    pt = np.ascontiguousarray(point, dtype=np.float64)
    G = np.empty(dim * dim)
    prob = make_problem(pb)
    rc = lib().orc_nodal_gradient(C.byref(prob), ptrs, _dptr(pt), _dptr(G))
    if rc:
        raise OracleError(rc, "orc_nodal_gradient")
    return G.reshape(dim, dim)


def splitmix64(z: int) -> int:
    return int(lib().orc_splitmix64(z & 0xFFFFFFFFFFFFFFFF))
