"""GPU library (through the C ABI) on the closed-form single steps the oracle
is pinned with, and on the device error paths.

* uniform linear flow v = A x on a regular lattice: for deep-interior
  particles Vbar = A X, G' = A, rho' = rho / (1 + dt tr A) and
  e' = e - dt (P + Q) tr A / rho with the lagged Q (Sec. 3 (viii));
  FP64 against the oracle to 1e-9 and the closed form to 1e-12, the
  FP32 fixed-point path to the closed form at FP32 rounding (1e-5);
* a particle pushed through a wall is clamped onto it and counted, not an
  error (Sec. 3 (ix));
* a fixed-point accumulator out of range raises MPM_E_OVERFLOW, after which
  the handle refuses to step (every kernel still exits normally: the flag
  is raised by the kernels and read by the host);
* negative pressure is allowed, the sound speed is clamped to 0 (reading
  C-14), and one FP64 step matches the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_17057_amd import mpm as G
from paper_2404_17057_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _deep_interior(pb):
    c = np.floor((pb.x[:2] - np.array(pb.lo[:2])[:, None]) / pb.h).astype(int)
    n = np.array(pb.n[:2])[:, None]
    return ((c >= 2) & (c <= n - 3)).all(axis=0)


CASES = {
    "compression": (np.array([[-0.8, 0.3], [0.5, -0.4]]), None),
    "expansion_after_compression": (np.array([[0.7, -0.2], [0.6, 0.5]]), [[-2.0, 0.1], [0.3, -1.0]]),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [G.FP64, G.FP32_FIX64])
def test_linear_flow_step_closed_form(case, prec):
    _gpu()
    A, gprev = CASES[case]
    dt = 1e-3
    pb = W.linear_flow_box(A, gprev)
    pb.dt0 = dt
    o = O.Oracle(pb)
    o.set_dt(dt)
    assert o.step(1) == 0
    print(f"linear flow {case} prec {prec}: {pb.n_particles} particles", flush=True)
    s = G.Simulation(pb, prec)
    s.step(1)
    st = s.status()
    assert st["rc"] == 0 and st["dt_last"] == dt
    got = s.read([G.F_X, G.F_V, G.F_RHO, G.F_E, G.F_G])
    sel = _deep_interior(pb)
    trA = np.trace(A)
    rho0, e0 = pb.rho[sel], pb.eint[sel]
    P0 = 0.4 * rho0 * e0
    dprev = 0.0 if gprev is None else float(np.trace(np.asarray(gprev)))
    Q = np.array([O.artificial_viscosity(W.AV_PAPER, 1.0, 1.0, 1.4, pb.h, r, p, dprev)
                  for r, p in zip(rho0, P0)])
    tol = 1e-12 if prec == G.FP64 else 1e-5
    x0 = pb.x[:, sel]
    assert np.abs(got[G.F_X][:, sel] - (x0 + dt * (A @ x0))).max() <= tol
    assert np.abs(got[G.F_G][:, sel] - A.reshape(4, 1)).max() <= 1e3 * tol
    assert np.allclose(got[G.F_RHO][sel], rho0 / (1.0 + dt * trA), rtol=tol, atol=0)
    assert np.allclose(got[G.F_E][sel], e0 - dt * (P0 + Q) * trA / rho0, rtol=tol, atol=0)
    if prec == G.FP64:
        for gf, of in [(G.F_X, O.F_X), (G.F_V, O.F_V), (G.F_RHO, O.F_RHO), (G.F_E, O.F_E), (G.F_G, O.F_G)]:
            ref = o.particles(of)
            assert np.abs(got[gf] - ref).max() <= 1e-9 * np.abs(ref).max(), gf


@pytest.mark.parametrize("prec", [G.FP64, G.FP32_FIX64])
def test_wall_escape_is_clamped_and_counted(prec):
    _gpu()
    pb = W.wall_escape(n=8, s=0.3)
    pb.dt0 = 0.65 * pb.h
    o = O.Oracle(pb)
    o.set_dt(pb.dt0)
    assert o.step(1) == 0
    assert o.status()["wall_escapes"] == 1
    print(f"wall escape prec {prec}", flush=True)
    s = G.Simulation(pb, prec)
    s.step(1)
    st = s.status()
    assert st["rc"] == 0
    assert int(s.counters()[1]) == 1
    x = s.field(G.F_X)
    assert x[0, 0] == 0.0
    assert abs(x[1, 0] - o.particles(O.F_X)[1, 0]) <= 1e-7
    rho = s.field(G.F_RHO)[0]
    assert rho == pytest.approx(o.particles(O.F_RHO)[0], rel=1e-12 if prec == G.FP64 else 1e-5)
    # the run goes on: the next step starts from the clamped particle
    s.step(1)
    assert s.status()["rc"] == 0


@pytest.mark.parametrize("name", ["sod_64x2", "blast3d_16"])
def test_fixed_point_overflow_is_reported(name):
    """Quanta far below the mass of a cell (a reference density 1e-9 of the
    real one) put the node sums beyond the int64 range the kernels accept:
    the step raises the sticky overflow error and the handle stops (2D: the
    halo-record flush; 3D: the frame atomics)."""
    _gpu()
    pb = {"sod_64x2": lambda: W.sod(nx=64, ny=2, t_end=0.0),
          "blast3d_16": lambda: W.blast3d(n=16, steps=2)}[name]()
    pb.rho_ref = 1e-9
    print(f"fixed-point overflow: {name}, rho_ref 1e-9", flush=True)
    s = G.Simulation(pb, G.FP32_FIX64)
    s.step(2)
    st = s.status()
    assert st["rc"] == G.E_OVERFLOW
    assert st["step"] <= 1
    with pytest.raises(G.MPMError) as ei:
        s.step(1)
    assert ei.value.code == G.E_STATE
    # the same problem with the derived reference runs cleanly
    pb.rho_ref = 0.0
    ok = G.Simulation(pb, G.FP32_FIX64)
    ok.step(2)
    assert ok.status()["rc"] == 0


@pytest.mark.parametrize("prec,tol", [(G.FP64, 1e-9), (G.FP32_FIX64, 1e-4)])
def test_negative_pressure_matches_oracle(prec, tol):
    """Gas whose right quarter has a negative internal energy (negative
    pressure, no sound speed): allowed, with c clamped to 0 (reading C-14).
    Three steps against the oracle."""
    _gpu()
    pb = W.sod(nx=64, ny=4, t_end=0.0)
    pb.eint = np.where(pb.x[0] > 0.75, -0.05 * pb.eint, pb.eint)
    o = O.Oracle(pb)
    assert o.step(3) == 0
    print(f"negative pressure prec {prec}", flush=True)
    s = G.Simulation(pb, prec)
    assert s.status()["dt_next"] == pytest.approx(O.Oracle(pb).status()["dt_next"], rel=1e-7)
    s.step(3)
    assert s.status()["rc"] == 0
    for gf, of in [(G.F_RHO, O.F_RHO), (G.F_E, O.F_E), (G.F_V, O.F_V)]:
        ref = o.particles(of)
        assert np.abs(s.field(gf) - ref).max() <= tol * np.abs(ref).max(), gf
    assert (s.field(G.F_P) < 0).sum() > 0


# FP32 positions carry a rounding of 2^-24 |x|, up to 2^-24 L/h of a cell
# (L/h = 256 here); a B2 weight moves by at most twice that per rounding
# (|N'| <= 2 per cell), and five steps chain five roundings of the position.
_PROJ_FP32_TOL = 5 * 2 * 2.0 ** -24 * 256


@pytest.mark.parametrize("prec,tol", [(G.FP64, 1e-9), (G.FP32_FIX64, _PROJ_FP32_TOL)])
def test_projected_density_matches_oracle(prec, tol):
    """The read-out of the grid-projected density (P2G of M and of M / rho
    at the current positions) against the oracle's, after 5 steps of the
    256x128 cylinder: per node, relative to the largest value."""
    _gpu()
    pb = W.cylinder(nx=256, ny=128, steps=5)
    o = O.Oracle(pb)
    assert o.step(5) == 0
    print(f"projected density prec {prec}", flush=True)
    s = G.Simulation(pb, prec)
    s.step(5)
    m_o, v_o = o.projected()
    m, v = s.grid(G.G_MPROJ), s.grid(G.G_VOLPROJ)
    assert np.abs(m - m_o).max() <= tol * m_o.max()
    assert np.abs(v - v_o).max() <= tol * v_o.max()
    assert np.array_equal(m > 0, m_o > 0)


@pytest.mark.parametrize("prec", [G.FP64, G.FP32_FIX64])
def test_recycling_through_a_y_outflow_face(prec):
    """The same step as the oracle pin: the top row leaves through the y_hi
    outflow face and re-enters at the inflow face; positions against the
    oracle, recycled count from the counters."""
    _gpu()
    pb = W.outflow_drift(n=8)
    pb.dt0 = 0.6 * pb.h
    o = O.Oracle(pb)
    o.set_dt(pb.dt0)
    assert o.step(1) == 0
    print(f"y outflow recycling prec {prec}", flush=True)
    s = G.Simulation(pb, prec)
    s.step(1)
    assert s.status()["rc"] == 0
    assert int(s.counters()[2]) == 16 and int(s.counters()[1]) == 0
    x = s.field(G.F_X)
    tol = 1e-12 if prec == G.FP64 else 2e-7
    assert np.abs(x - o.particles(O.F_X)).max() <= tol
    assert np.array_equal(s.field(G.F_M), o.particles(O.F_M).astype(np.float32).astype(np.float64)
                          if prec == G.FP32_FIX64 else o.particles(O.F_M))
