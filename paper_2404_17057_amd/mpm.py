"""Thin ctypes binding of libmpm.so (include/mpm.h).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  PyTorch provides the device workspace (a uint8 tensor) and
the stream.  The binding raises if the library is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

OK, E_ARG, E_WORKSPACE, E_HIP, E_NONPHYSICAL, E_OVERFLOW, E_UNSUPPORTED, E_STATE, E_SCRATCH = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
Q1, B2 = 1, 2
FP64, FP32_ACC_F64, FP32_ACC_F32, FP32_FIX64, FP64_COLOR = 0, 1, 2, 3, 4
PRECISION_NAMES = {FP64: "fp64", FP32_ACC_F64: "fp32_acc_f64",
                   FP32_ACC_F32: "fp32_acc_f32", FP32_FIX64: "fp32_fix64", FP64_COLOR: "fp64_color"}
F_X, F_V, F_M, F_RHO, F_E, F_P, F_Q, F_G, F_VOL, F_ID = range(10)
G_M, G_P, G_F, G_PUPD, G_P2, G_FBC, G_FLAGS, G_MPROJ, G_VOLPROJ = range(9)

EXPORTS = ["mpm_footprint", "mpm_init", "mpm_step", "mpm_step_batch", "mpm_read_fields",
           "mpm_read_grid", "mpm_read_grid_noalloc", "mpm_status", "mpm_counters", "mpm_profile_step", "mpm_grid_shape",
           "mpm_destroy", "mpm_strerror"]
SWEEPS = ["p2g", "frame_reduce", "g2p_p2g", "tilescan", "cellscan", "update", "finalize"]


class Desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("shape", C.c_int32), ("precision", C.c_int32), ("av_form", C.c_int32),
        ("gamma", C.c_double), ("c0", C.c_double), ("c1", C.c_double), ("cfl", C.c_double),
        ("face", (C.c_int32 * 2) * 3),
        ("inflow_rho", C.c_double), ("inflow_p", C.c_double), ("inflow_u", C.c_double * 3),
        ("recycle_mass", C.c_double),
        ("n_particles", C.c_int64),
        ("seed", C.c_uint64),
        ("t_end", C.c_double),
        ("rho_ref", C.c_double), ("u_ref", C.c_double),
        ("t0", C.c_double), ("step0", C.c_int64), ("dt0", C.c_double),
    ]


_DP = C.POINTER(C.c_double)


class ParticlesHost(C.Structure):
    _fields_ = [("x", _DP * 3), ("v", _DP * 3), ("mass", _DP), ("rho", _DP), ("eint", _DP),
                ("gradv", _DP * 9), ("id", C.POINTER(C.c_uint32))]


class ObstacleHost(C.Structure):
    _fields_ = [("cell_mask", C.POINTER(C.c_uint8)), ("node_normal", _DP * 3)]


class MPMError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().mpm_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libmpm.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2404_17057_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mpm_footprint.argtypes = [C.POINTER(Desc), C.POINTER(C.c_size_t)]
        L.mpm_init.argtypes = [C.POINTER(Desc), C.POINTER(ParticlesHost), C.POINTER(ObstacleHost),
                               vp, C.c_size_t, vp, C.POINTER(vp)]
        L.mpm_step.argtypes = [vp, C.c_int64, vp]
        L.mpm_step_batch.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(C.c_int64), vp]
        L.mpm_read_fields.argtypes = [vp, C.c_uint32, C.POINTER(_DP), vp]
        L.mpm_read_grid.argtypes = [vp, C.c_int32, _DP, vp]
        L.mpm_read_grid_noalloc.argtypes = [vp, C.c_int32, _DP, vp]
        L.mpm_status.argtypes = [vp, _DP, _DP, _DP, C.POINTER(C.c_int64), _DP, vp]
        L.mpm_counters.argtypes = [vp, C.POINTER(C.c_uint64), vp]
        L.mpm_profile_step.argtypes = [vp, C.c_int64, _DP, vp]
        L.mpm_grid_shape.argtypes = [vp, C.POINTER(C.c_int32)]
        L.mpm_destroy.argtypes = [vp]
        L.mpm_strerror.argtypes = [C.c_int]
        L.mpm_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def make_desc(pb, precision: int) -> Desc:
    d = Desc()
    d.dim = pb.dim
    for a in range(3):
        d.n[a] = int(pb.n[a])
        d.lo[a] = float(pb.lo[a])
        d.hi[a] = float(pb.hi[a])
        d.face[a][0] = int(pb.faces[a][0])
        d.face[a][1] = int(pb.faces[a][1])
        d.inflow_u[a] = float(pb.inflow_u[a])
    d.shape = pb.shape
    d.precision = precision
    d.av_form = pb.av_form
    d.gamma, d.c0, d.c1, d.cfl = pb.gamma, pb.c0, pb.c1, pb.cfl
    d.inflow_rho, d.inflow_p = pb.inflow_rho, pb.inflow_p
    d.recycle_mass = pb.recycle_mass
    d.n_particles = pb.n_particles
    d.seed = int(pb.seed) & 0xFFFFFFFFFFFFFFFF
    d.t_end = pb.t_end
    d.rho_ref = float(pb.rho_ref)
    d.u_ref = float(pb.u_ref)
    d.t0 = float(pb.t0)
    d.step0 = int(pb.step0)
    d.dt0 = float(pb.dt0)
    return d


def footprint(pb, precision: int) -> int:
    d = make_desc(pb, precision)
    n = C.c_size_t()
    rc = lib().mpm_footprint(C.byref(d), C.byref(n))
    if rc:
        raise MPMError(rc, "mpm_footprint")
    return int(n.value)


def _stream_ptr(stream) -> C.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


class Simulation:
    """One MPM problem resident in a device workspace owned by this object."""

    def __init__(self, pb, precision: int = FP32_FIX64, device: str = "cuda:0", stream=None,
                 workspace=None):
        import torch
        self.pb = pb
        self.precision = precision
        self.dim = pb.dim
        self.np = pb.n_particles
        self.device = torch.device(device)
        self._desc = make_desc(pb, precision)
        nbytes = footprint(pb, precision)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        base = workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        avail = workspace.numel() - (aligned - base)
        self.stream = stream
        keep = []

        def arr(a, dtype=np.float64):
            a = np.ascontiguousarray(a, dtype=dtype)
            keep.append(a)
            return a

        ph = ParticlesHost()
        for a in range(self.dim):
            ph.x[a] = arr(pb.x[a]).ctypes.data_as(_DP)
            ph.v[a] = arr(pb.v[a]).ctypes.data_as(_DP)
        ph.mass = arr(pb.mass).ctypes.data_as(_DP)
        ph.rho = arr(pb.rho).ctypes.data_as(_DP)
        ph.eint = arr(pb.eint).ctypes.data_as(_DP)
        if pb.gradv is not None:
            for c in range(self.dim * self.dim):
                ph.gradv[c] = arr(pb.gradv[c]).ctypes.data_as(_DP)
        ph.id = arr(pb.ids, np.uint32).ctypes.data_as(C.POINTER(C.c_uint32))
        obs = None
        if pb.cell_mask is not None:
            obs = ObstacleHost()
            obs.cell_mask = arr(pb.cell_mask, np.uint8).ctypes.data_as(C.POINTER(C.c_uint8))
            for a in range(self.dim):
                obs.node_normal[a] = arr(pb.node_normal[a]).ctypes.data_as(_DP)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().mpm_init(C.byref(self._desc), C.byref(ph),
                                C.byref(obs) if obs is not None else None,
                                C.c_void_p(aligned), C.c_size_t(avail), self._sp(), C.byref(h))
        if rc:
            raise MPMError(rc, "mpm_init")
        self._h = h
        shp = (C.c_int32 * 3)()
        lib().mpm_grid_shape(self._h, shp)
        self.nodes = tuple(int(v) for v in shp)
        self.nnodes = int(np.prod(self.nodes))

    def _sp(self):
        return _stream_ptr(self.stream)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().mpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        rc = lib().mpm_step(self._h, int(n), self._sp())
        if rc:
            raise MPMError(rc, "mpm_step")

    _NCOMP = {F_X: "d", F_V: "d", F_G: "dd"}

    def read(self, fields: Sequence[int], check: bool = True) -> Dict[int, np.ndarray]:
        fields = sorted(set(fields))
        outs = []
        mask = 0
        for f in fields:
            nc = {"d": self.dim, "dd": self.dim * self.dim}.get(self._NCOMP.get(f), 1)
            outs.append(np.empty((nc, self.np)))
            mask |= 1 << f
        ptrs = (_DP * len(outs))(*[o.ctypes.data_as(_DP) for o in outs])
        rc = lib().mpm_read_fields(self._h, mask, ptrs, self._sp())
        if rc and (check or rc not in (E_NONPHYSICAL, E_OVERFLOW)):
            raise MPMError(rc, "mpm_read_fields")
        return {f: (o if o.shape[0] > 1 else o[0]) for f, o in zip(fields, outs)}

    def field(self, f: int) -> np.ndarray:
        return self.read([f])[f]

    def grid(self, which: int) -> np.ndarray:
        nc = 1 if which in (G_M, G_FLAGS, G_MPROJ, G_VOLPROJ) else self.dim
        out = np.empty((nc, self.nnodes))
        rc = lib().mpm_read_grid(self._h, which, out.ctypes.data_as(_DP), self._sp())
        if rc:
            raise MPMError(rc, "mpm_read_grid")
        return out if nc > 1 else out[0]

    def grid_noalloc(self, which: int) -> np.ndarray:
        """The grid snapshot of `grid`, through the entry point that allocates
        no device memory (fixed 32 MiB scratch per GPU)."""
        nc = 1 if which in (G_M, G_FLAGS, G_MPROJ, G_VOLPROJ) else self.dim
        out = np.empty((nc, self.nnodes))
        rc = lib().mpm_read_grid_noalloc(self._h, which, out.ctypes.data_as(_DP), self._sp())
        if rc:
            raise MPMError(rc, "mpm_read_grid_noalloc")
        return out if nc > 1 else out[0]

    def status(self) -> dict:
        t, dtn, dtl = C.c_double(), C.c_double(), C.c_double()
        step = C.c_int64()
        cons = (C.c_double * 6)()
        rc = lib().mpm_status(self._h, C.byref(t), C.byref(dtn), C.byref(dtl), C.byref(step),
                              cons, self._sp())
        return dict(t=t.value, dt_next=dtn.value, dt_last=dtl.value, step=step.value,
                    conserved=np.array(list(cons)), rc=rc)

    def profile(self, n: int) -> Dict[str, float]:
        """Average milliseconds per sweep over n real steps (HIP events)."""
        ms = (C.c_double * len(SWEEPS))()
        rc = lib().mpm_profile_step(self._h, int(n), ms, self._sp())
        if rc:
            raise MPMError(rc, "mpm_profile_step")
        return dict(zip(SWEEPS, list(ms)))

    def counters(self) -> np.ndarray:
        c = (C.c_uint64 * 4)()
        rc = lib().mpm_counters(self._h, c, self._sp())
        if rc:
            raise MPMError(rc, "mpm_counters")
        return np.array(list(c), dtype=np.uint64)


def step_batch(sims: Sequence[Simulation], n_steps: Sequence[int], stream=None) -> None:
    hs = (C.c_void_p * len(sims))(*[s.handle for s in sims])
    ns = (C.c_int64 * len(sims))(*[int(n) for n in n_steps])
    rc = lib().mpm_step_batch(hs, len(sims), ns, _stream_ptr(stream))
    if rc:
        raise MPMError(rc, "mpm_step_batch")
