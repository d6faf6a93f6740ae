"""The C-ABI library loads on the CPU and exports every declared entry point.

No compute call is made here (there is no GPU in the CPU suite)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2404_17057_amd import mpm as G
from paper_2404_17057_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(G.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mpm_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    L = ctypes.CDLL(G.LIB_PATH)
    for f in declared_functions():
        assert hasattr(L, f)


def test_footprint_and_descriptor_checks_on_host():
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    pb = W.cylinder(nx=64, ny=32)
    n64 = G.footprint(pb, G.FP64)
    n32 = G.footprint(pb, G.FP32_FIX64)
    assert n64 > n32 > pb.n_particles * 48
    with pytest.raises(G.MPMError) as ei:
        bad = W.Problem(**{**pb.__dict__})
        bad.hi = (1.0, 0.7, 0.0)                 # cells not square
        G.footprint(bad, G.FP64)
    assert ei.value.code == G.E_ARG
    assert G.lib().mpm_strerror(G.E_OVERFLOW).decode().startswith("fixed-point")


def test_particle_count_limit_on_host():
    """Particle arrays are addressed with 32-bit byte offsets: the largest
    count keeps one array below 4 GiB (2^30 - 4 in FP32, 2^29 - 2 in FP64)."""
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    pb = W.cylinder(nx=64, ny=32)
    n = ctypes.c_size_t()
    for prec, size in ((G.FP32_FIX64, 4), (G.FP64, 8)):
        d = G.make_desc(pb, prec)
        d.n_particles = 0xFFFFFFF0 // size
        assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == 0
        d.n_particles += 1
        assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == G.E_UNSUPPORTED


def test_grid_size_limit_on_host():
    """Cell keys are 32-bit and node indices int: a grid of more than 2^31
    padded cells or nodes is refused before any layout arithmetic, also for
    cell counts whose products overflow 64 bits."""
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    n = ctypes.c_size_t()
    pb = W.blast3d(n=8, steps=1)
    d = G.make_desc(pb, G.FP32_FIX64)
    assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == 0
    # 1288^3 cells: 1288 = 161 tiles of 8 in x and y, 322 tiles of 4 in z,
    # 2.14e9 cells; (1290)^3 nodes = 2.147e9 <= 2^31 - 1
    for a in range(3):
        d.n[a] = 1288
        d.hi[a] = d.lo[a] + 1288 * 0.001
    assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == 0
    d.n[0] = 1296
    d.hi[0] = d.lo[0] + 1296 * 0.001
    assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == G.E_UNSUPPORTED
    for a in range(3):
        d.n[a] = 2 ** 30
        d.hi[a] = d.lo[a] + 2 ** 30 * 0.001
    assert G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n)) == G.E_UNSUPPORTED


def test_inflow_state_validated_on_host():
    """An INFLOW or OUTFLOW face needs a physical inflow state, and an OUTFLOW
    face a positive recycling mass; wall-only problems ignore them."""
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    n = ctypes.c_size_t()
    pb = W.cylinder(nx=64, ny=32)
    fp = lambda d: G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n))
    assert fp(G.make_desc(pb, G.FP32_FIX64)) == 0
    for field, value in (("inflow_rho", 0.0), ("inflow_rho", float("inf")), ("inflow_p", -1.0),
                         ("inflow_p", float("nan")), ("recycle_mass", 0.0)):
        d = G.make_desc(pb, G.FP32_FIX64)
        setattr(d, field, value)
        assert fp(d) == G.E_ARG, (field, value)
    d = G.make_desc(pb, G.FP32_FIX64)
    d.inflow_u[1] = float("nan")
    assert fp(d) == G.E_ARG
    sod = G.make_desc(W.sod(), G.FP64)
    sod.inflow_rho = 0.0
    sod.recycle_mass = 0.0
    assert fp(sod) == 0


def test_restart_fields_validated_on_host():
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libmpm.so not built")
    n = ctypes.c_size_t()
    fp = lambda d: G.lib().mpm_footprint(ctypes.byref(d), ctypes.byref(n))
    pb = W.cylinder(nx=64, ny=32)
    d = G.make_desc(pb, G.FP32_FIX64)
    d.t0, d.step0, d.dt0 = 0.125, 37, 1e-4
    assert fp(d) == 0
    for field, value in (("t0", -1.0), ("t0", float("nan")), ("t0", float("inf")), ("step0", -1),
                         ("dt0", float("inf")), ("dt0", float("nan"))):
        d = G.make_desc(pb, G.FP32_FIX64)
        setattr(d, field, value)
        assert fp(d) == G.E_ARG, (field, value)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(G, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(G, "_lib", None)
    with pytest.raises(RuntimeError):
        G.lib()
