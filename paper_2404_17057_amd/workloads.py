"""Seeded synthetic inputs: problem descriptions, particle clouds and obstacle
geometry for the MPM workloads.

This module is the only code shared by the GPU library's callers and the test
oracle.  It builds *inputs* only -- domains, particle placement, initial
states, obstacle masks and normals (the pre-processing stage of Sec. 3, step
1 of the paper) -- and holds none of the time-stepping arithmetic.

Workloads (all 2D unless stated, ideal gas gamma = 1.4):

* ``sod``       -- quasi-1D shock tube (Sec. 4.1, Sod): left rho=1, p=1; right
                   rho=0.125, p=0.1; diaphragm at x=0.5; walls everywhere.
* ``cylinder``  -- supersonic flow past a circular cylinder (Sec. 4.1): inflow
                   at x_lo, outflow (recycling) at x_hi, slip walls in y; far
                   field rho=1.4, p=1 so that c=1 and Mach = |u|.
* ``blast3d``   -- 3D spherical blast in the unit cube: rho=1, p=1e-5, and an
                   inner sphere at p=1e3; walls everywhere.
* ``sphere3d``  -- the cylinder's 3D counterpart: supersonic flow past a sphere
                   in a channel, inflow at x_lo, outflow (recycling) at x_hi and
                   optionally at the side faces, else walls.
* ``quadrant``  -- 2x2-quadrant Riemann problem on the unit square, random
                   per-quadrant states; walls everywhere.
* ``aerofoil``  -- transonic flow (Mach 0.73) past a NACA 4-digit section
                   given as sampled surface points; its mask and normals come
                   from the sampled signed distance function (Sec. 3.2).

Particles sit on a regular s^d lattice in every fluid cell at offsets
(j + 1/2)/s of the cell, each coordinate jittered by U(-0.05, 0.05) cells;
the particle mass is rho(X) h^d / ppc.  Cells whose centre lies inside an
obstacle get no particles.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np

WALL, INFLOW, OUTFLOW = 0, 1, 2
Q1, B2 = 1, 2
AV_PAPER, AV_BOOK = 0, 1
FP64, FP32_ACC_F64, FP32_ACC_F32, FP32_FIX64, FP64_COLOR = 0, 1, 2, 3, 4

DEFAULT_SEED = 17057


@dataclasses.dataclass
class Problem:
    """One MPM problem: descriptor values, particle arrays and obstacle data."""

    name: str
    dim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    faces: Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, int]]
    x: np.ndarray            # (dim, N) float64
    v: np.ndarray            # (dim, N) float64
    mass: np.ndarray         # (N,)
    rho: np.ndarray          # (N,)
    eint: np.ndarray         # (N,) specific internal energy
    ids: np.ndarray          # (N,) uint32, a permutation of 0..N-1
    shape: int = B2
    av_form: int = AV_PAPER
    gamma: float = 1.4
    c0: float = 1.0
    c1: float = 1.0
    cfl: float = 0.3
    inflow_rho: float = 0.0
    inflow_p: float = 0.0
    inflow_u: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    recycle_mass: float = 0.0
    seed: int = DEFAULT_SEED
    t_end: float = 0.0
    steps: int = 0                       # nominal step count of the workload
    gradv: Optional[np.ndarray] = None   # (dim*dim, N) or None for zero
    cell_mask: Optional[np.ndarray] = None   # uint8 over cells, x fastest
    node_normal: Optional[np.ndarray] = None  # (dim, nodes) float64, x fastest
    rho_ref: float = 0.0                 # fixed-point references (0: from the state)
    u_ref: float = 0.0
    t0: float = 0.0                      # restart: time, steps taken, next time step
    step0: int = 0                       # (a fresh start: all 0)
    dt0: float = 0.0

    @property
    def n_particles(self) -> int:
        return int(self.mass.shape[0])

    @property
    def h(self) -> float:
        return (self.hi[0] - self.lo[0]) / self.n[0]

    def node_counts(self) -> Tuple[int, int, int]:
        return node_counts(self.n, self.dim, self.shape)

    def permuted(self, seed: int) -> "Problem":
        """The same particle cloud handed over in a random order."""
        perm = np.random.default_rng(seed).permutation(self.n_particles)
        kw = dataclasses.asdict(self)
        kw.update(x=self.x[:, perm].copy(), v=self.v[:, perm].copy(),
                  mass=self.mass[perm].copy(), rho=self.rho[perm].copy(),
                  eint=self.eint[perm].copy(), ids=self.ids[perm].copy(),
                  gradv=None if self.gradv is None else self.gradv[:, perm].copy())
        return Problem(**kw)


# ---------------------------------------------------------------- geometry --

def _lattice(n, lo, h, dim, per_axis, jitter, rng, cell_ok=None):
    """Particle positions on the jittered lattice; returns (dim, N) and the
    flat cell index of each particle."""
    s = per_axis
    off1 = (np.arange(s) + 0.5) / s
    grids = np.meshgrid(*([off1] * dim), indexing="ij")
    offs = np.stack([g.ravel() for g in reversed(grids)], axis=0)  # x fastest
    ncell = int(np.prod(n[:dim]))
    cells = np.arange(ncell, dtype=np.int64)
    if cell_ok is not None:
        cells = cells[cell_ok.ravel() != 0]
    ci = []
    rem = cells.copy()
    for a in range(dim):
        ci.append(rem % n[a])
        rem //= n[a]
    ci = np.stack(ci, axis=0)                                    # (dim, ncell')
    nper = offs.shape[1]
    pos = (ci[:, :, None] + offs[:, None, :]).reshape(dim, -1)   # cell units
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    x = np.empty_like(pos)
    for a in range(dim):
        x[a] = lo[a] + pos[a] * h
    cell_of = np.repeat(cells, nper)
    return x, cell_of


def node_counts(n, dim, shape):
    """Nodes per axis: Q1 has the n+1 cell vertices; B2 (quadratic B-splines on
    the clamped knot vector of the cell faces) has n+2 basis functions."""
    extra = 2 if shape == B2 else 1
    return tuple(n[a] + extra if a < dim else 1 for a in range(3))


def node_axis(n_a, shape):
    """Node coordinates along one axis in cell units: Q1 vertices 0..n; B2
    Greville points 0, 1/2, 3/2, ..., n-1/2, n."""
    if shape == B2:
        return np.concatenate([[0.0], np.arange(n_a) + 0.5, [float(n_a)]])
    return np.arange(n_a + 1, dtype=np.float64)


def _node_positions(n, lo, h, dim, shape):
    axes = [lo[a] + node_axis(n[a], shape) * h for a in range(dim)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return [m.ravel() for m in reversed(mesh)]


def circle_obstacle(n, lo, h, dim, shape, center, radius):
    """Cell mask (cell centre inside the circle/sphere) and outward unit
    normals (x_i - c)/|x_i - c| on every node (0 at the centre)."""
    ncell = [n[a] for a in range(dim)]
    cax = [lo[a] + (np.arange(ncell[a]) + 0.5) * h for a in range(dim)]
    mesh = np.meshgrid(*reversed(cax), indexing="ij")
    cc = [m.ravel() for m in reversed(mesh)]
    r2 = sum((cc[a] - center[a]) ** 2 for a in range(dim))
    mask = (r2 < radius * radius).astype(np.uint8)
    nodes = _node_positions(n, lo, h, dim, shape)
    d = np.stack([nodes[a] - center[a] for a in range(dim)], axis=0)
    r = np.sqrt((d * d).sum(axis=0))
    normal = np.where(r > 1e-12, d / np.where(r > 1e-12, r, 1.0), 0.0)
    return mask, normal


def naca4_profile(code="0012", chord=1.0, leading_edge=(0.0, 0.0), alpha_deg=0.0,
                  n_side=200):
    """Closed polygon (2, 2*n_side - 1) sampling a NACA 4-digit section: the
    stand-in for a profile read from a file of surface points (Sec. 4.1,
    transonic aerofoil).  `code` = "MPTT": maximum camber M % of the chord at
    P/10 of the chord, thickness TT %.  Points are cosine-spaced along the
    chord, upper surface from the trailing edge to the leading edge, then
    the lower surface back; the trailing edge is closed (thickness
    polynomial with -0.1036 x^4).  The section is scaled by `chord`, rotated
    by the angle of attack `alpha_deg` (positive raises the nose) about the
    quarter-chord point and translated so that the unrotated leading edge
    sits at `leading_edge`."""
    m = int(code[0]) / 100.0
    p = int(code[1]) / 10.0
    t = int(code[2:]) / 100.0
    beta = np.linspace(0.0, math.pi, n_side)
    xc = 0.5 * (1.0 - np.cos(beta))                       # 0 .. 1, clustered at both ends
    yt = 5.0 * t * (0.2969 * np.sqrt(xc) - 0.1260 * xc - 0.3516 * xc ** 2
                    + 0.2843 * xc ** 3 - 0.1036 * xc ** 4)
    if m > 0.0:
        front = xc < p
        yc = np.where(front, m / p ** 2 * (2 * p * xc - xc ** 2),
                      m / (1 - p) ** 2 * ((1 - 2 * p) + 2 * p * xc - xc ** 2))
        dyc = np.where(front, 2 * m / p ** 2 * (p - xc), 2 * m / (1 - p) ** 2 * (p - xc))
    else:
        yc = np.zeros_like(xc)
        dyc = np.zeros_like(xc)
    th = np.arctan(dyc)
    xu, yu = xc - yt * np.sin(th), yc + yt * np.cos(th)
    xl, yl = xc + yt * np.sin(th), yc - yt * np.cos(th)
    px = np.concatenate([xu[::-1], xl[1:]]) - 0.25
    py = np.concatenate([yu[::-1], yl[1:]])
    a = math.radians(alpha_deg)
    rx = px * math.cos(a) + py * math.sin(a)
    ry = -px * math.sin(a) + py * math.cos(a)
    return np.stack([leading_edge[0] + chord * (rx + 0.25), leading_edge[1] + chord * ry])


def polygon_sdf(poly, qx, qy, chunk=16384):
    """Signed Euclidean distance from the points (qx, qy) to the closed
    polygon `poly` (2, S): the minimum distance to its S edges, negative
    inside (even-odd rule).  This is `eq:sdf` with the profile taken as the
    polyline through the sampled surface points."""
    ax, ay = poly[0], poly[1]
    bx, by = np.roll(ax, -1), np.roll(ay, -1)
    ex, ey = bx - ax, by - ay
    ee = np.where(ex * ex + ey * ey > 0.0, ex * ex + ey * ey, 1.0)
    qx = np.asarray(qx, dtype=np.float64).ravel()
    qy = np.asarray(qy, dtype=np.float64).ravel()
    out = np.empty(qx.size)
    for s in range(0, qx.size, chunk):
        x = qx[s:s + chunk, None]
        y = qy[s:s + chunk, None]
        u = np.clip(((x - ax) * ex + (y - ay) * ey) / ee, 0.0, 1.0)
        dx, dy = x - (ax + u * ex), y - (ay + u * ey)
        dist = np.sqrt((dx * dx + dy * dy).min(axis=1))
        straddle = (ay > y) != (by > y)
        xcross = ax + (y - ay) * ex / np.where(ey != 0.0, ey, 1.0)
        inside = (straddle & (x < xcross)).sum(axis=1) % 2 == 1
        out[s:s + chunk] = np.where(inside, -dist, dist)
    return out


def sdf_obstacle(n, lo, h, shape, poly, margin=4):
    """Cell mask and node normals of a 2D obstacle given as a sampled surface
    (Sec. 3.2, `eq:sdf`): the signed distance is sampled on the node lattice
    and at the cell centres; a cell is masked when its centre has negative
    distance, and each node's normal is the gradient of the node-sampled
    distance (second-order differences on the node coordinates), scaled to
    unit length (0 where it vanishes).  The distance is sampled on the
    window of nodes and cells within `margin` cells of the profile's
    bounding box; cells outside it lie outside the profile, and nodes
    outside it get a zero normal (only nodes of masked cells use one)."""
    ax = [lo[a] + node_axis(n[a], shape) * h for a in range(2)]
    cx = [lo[a] + (np.arange(n[a]) + 0.5) * h for a in range(2)]
    win_n, win_c = [], []
    for a in range(2):
        lo_a = poly[a].min() - margin * h
        hi_a = poly[a].max() + margin * h
        win_n.append(np.nonzero((ax[a] >= lo_a) & (ax[a] <= hi_a))[0])
        win_c.append(np.nonzero((cx[a] >= lo_a) & (cx[a] <= hi_a))[0])
    nn = [len(ax[0]), len(ax[1])]
    normal = np.zeros((2, nn[1], nn[0]))
    mask = np.zeros((n[1], n[0]), dtype=np.uint8)
    wx, wy = ax[0][win_n[0]], ax[1][win_n[1]]
    if len(wx) >= 3 and len(wy) >= 3:
        mx, my = np.meshgrid(wx, wy, indexing="xy")
        sd = polygon_sdf(poly, mx, my).reshape(mx.shape)
        gy, gx = np.gradient(sd, wy, wx)
        g = np.sqrt(gx * gx + gy * gy)
        safe = np.where(g > 1e-12, g, 1.0)
        sl = np.ix_(win_n[1], win_n[0])
        normal[0][sl] = np.where(g > 1e-12, gx / safe, 0.0)
        normal[1][sl] = np.where(g > 1e-12, gy / safe, 0.0)
    if len(win_c[0]) and len(win_c[1]):
        ccx, ccy = np.meshgrid(cx[0][win_c[0]], cx[1][win_c[1]], indexing="xy")
        inside = polygon_sdf(poly, ccx, ccy).reshape(ccx.shape) < 0.0
        mask[np.ix_(win_c[1], win_c[0])] = inside.astype(np.uint8)
    return mask.ravel(), normal.reshape(2, -1)


def _pad3(t, fill):
    t = tuple(t)
    return t + (fill,) * (3 - len(t))


# ---------------------------------------------------------------- workloads --

def sod(nx=256, ny=8, per_axis=2, jitter=0.05, seed=DEFAULT_SEED, shape=B2,
        av_form=AV_PAPER, c0=1.0, c1=1.0, t_end=0.2, cfl=0.3) -> Problem:
    """Quasi-1D Sod tube on [0,1] x [0, ny/nx] (square cells), walls."""
    h = 1.0 / nx
    n = (nx, ny, 1)
    lo = (0.0, 0.0, 0.0)
    hi = (1.0, ny * h, 0.0)
    rng = np.random.default_rng(seed)
    x, _ = _lattice(n, lo, h, 2, per_axis, jitter, rng)
    left = x[0] < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    gamma = 1.4
    N = x.shape[1]
    ppc = per_axis ** 2
    return Problem(
        name=f"sod_{nx}x{ny}", dim=2, n=n, lo=lo, hi=hi,
        faces=((WALL, WALL), (WALL, WALL), (WALL, WALL)),
        x=x, v=np.zeros((2, N)), mass=rho * h * h / ppc, rho=rho,
        eint=p / ((gamma - 1.0) * rho), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, c0=c0, c1=c1, cfl=cfl,
        seed=seed, t_end=t_end, steps=0)


def cylinder(nx=1024, ny=512, per_axis=2, mach=3.0, jitter=0.05, seed=DEFAULT_SEED,
             shape=B2, av_form=AV_PAPER, lx=1.0, center=(0.3, 0.25), radius=0.05,
             steps=2000, cfl=0.3) -> Problem:
    """Mach `mach` flow past a cylinder on [0,lx] x [0, lx*ny/nx]."""
    h = lx / nx
    n = (nx, ny, 1)
    lo = (0.0, 0.0, 0.0)
    hi = (lx, ny * h, 0.0)
    rho0, p0, gamma = 1.4, 1.0, 1.4
    mask, normal = circle_obstacle(n, lo, h, 2, shape, center, radius)
    rng = np.random.default_rng(seed)
    ok = (1 - mask).reshape(ny, nx)
    x, _ = _lattice(n, lo, h, 2, per_axis, jitter, rng, cell_ok=ok)
    N = x.shape[1]
    ppc = per_axis ** 2
    m0 = rho0 * h * h / ppc
    v = np.zeros((2, N))
    v[0] = mach
    return Problem(
        name=f"cylinder_{nx}x{ny}_ppc{ppc}", dim=2, n=n, lo=lo, hi=hi,
        faces=((INFLOW, OUTFLOW), (WALL, WALL), (WALL, WALL)),
        x=x, v=v, mass=np.full(N, m0), rho=np.full(N, rho0),
        eint=np.full(N, p0 / ((gamma - 1.0) * rho0)), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, cfl=cfl,
        inflow_rho=rho0, inflow_p=p0, inflow_u=(mach, 0.0, 0.0), recycle_mass=m0,
        seed=seed, t_end=0.0, steps=steps, cell_mask=mask, node_normal=normal)


def sphere3d(nx=64, per_axis=2, mach=3.0, jitter=0.05, seed=DEFAULT_SEED, shape=B2,
             av_form=AV_PAPER, center=(0.3, 0.25, 0.25), radius=0.1, outflow_sides=False,
             steps=100, cfl=0.3) -> Problem:
    """The cylinder's 3D counterpart: Mach `mach` flow past a sphere in the
    channel [0,1] x [0,0.5] x [0,0.5] (nx x nx/2 x nx/2 cells), the same gas
    (rho = 1.4, p = 1, c = 1) and inflow at x_lo; outflow (recycling) at
    x_hi, and at the four side faces too with `outflow_sides`, else walls
    there.  It exercises the 3D inflow, outflow, recycling and obstacle
    conditions that the all-wall blast does not reach."""
    assert nx % 2 == 0
    h = 1.0 / nx
    n = (nx, nx // 2, nx // 2)
    lo = (0.0, 0.0, 0.0)
    hi = (1.0, n[1] * h, n[2] * h)
    rho0, p0, gamma = 1.4, 1.0, 1.4
    mask, normal = circle_obstacle(n, lo, h, 3, shape, center, radius)
    rng = np.random.default_rng(seed)
    x, _ = _lattice(n, lo, h, 3, per_axis, jitter, rng, cell_ok=1 - mask)
    N = x.shape[1]
    ppc = per_axis ** 3
    m0 = rho0 * h ** 3 / ppc
    v = np.zeros((3, N))
    v[0] = mach
    side = (OUTFLOW, OUTFLOW) if outflow_sides else (WALL, WALL)
    return Problem(
        name=f"sphere3d_{nx}_ppc{ppc}", dim=3, n=n, lo=lo, hi=hi,
        faces=((INFLOW, OUTFLOW), side, side),
        x=x, v=v, mass=np.full(N, m0), rho=np.full(N, rho0),
        eint=np.full(N, p0 / ((gamma - 1.0) * rho0)), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, cfl=cfl,
        inflow_rho=rho0, inflow_p=p0, inflow_u=(mach, 0.0, 0.0), recycle_mass=m0,
        seed=seed, t_end=0.0, steps=steps, cell_mask=mask, node_normal=normal)


def aerofoil(nx=640, per_axis=2, mach=0.73, code="2412", alpha_deg=-3.5, chord=0.12,
             leading_edge=(0.1, 0.135), jitter=0.05, seed=DEFAULT_SEED, shape=B2,
             av_form=AV_PAPER, steps=2000, cfl=0.3, n_side=200) -> Problem:
    """Transonic flow past an aerofoil on [0,0.4] x [0,0.27] (Sec. 4.1): the
    obstacle is given by sampled surface points and its mask and normals
    come from the sampled signed distance (`sdf_obstacle`).  A NACA
    4-digit section stands in for the OAT15a profile, whose coordinates are
    not available.  Inflow at x_lo with u = (mach, 0) in gas with rho = 1.4,
    p = 1 (so c = 1), outflow (recycling) at the other three faces, as in
    Sec. 4.1."""
    h = 0.4 / nx
    ny = int(round(0.27 / h))
    n = (nx, ny, 1)
    lo = (0.0, 0.0, 0.0)
    hi = (0.4, ny * h, 0.0)
    rho0, p0, gamma = 1.4, 1.0, 1.4
    poly = naca4_profile(code, chord, leading_edge, alpha_deg, n_side)
    mask, normal = sdf_obstacle(n, lo, h, shape, poly)
    rng = np.random.default_rng(seed)
    x, _ = _lattice(n, lo, h, 2, per_axis, jitter, rng, cell_ok=(1 - mask).reshape(ny, nx))
    N = x.shape[1]
    ppc = per_axis ** 2
    m0 = rho0 * h * h / ppc
    v = np.zeros((2, N))
    v[0] = mach
    return Problem(
        name=f"aerofoil_naca{code}_{nx}x{ny}_ppc{ppc}", dim=2, n=n, lo=lo, hi=hi,
        faces=((INFLOW, OUTFLOW), (OUTFLOW, OUTFLOW), (WALL, WALL)),
        x=x, v=v, mass=np.full(N, m0), rho=np.full(N, rho0),
        eint=np.full(N, p0 / ((gamma - 1.0) * rho0)), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, cfl=cfl,
        inflow_rho=rho0, inflow_p=p0, inflow_u=(mach, 0.0, 0.0), recycle_mass=m0,
        seed=seed, t_end=0.0, steps=steps, cell_mask=mask, node_normal=normal)


def blast3d(n=256, per_axis=2, jitter=0.05, seed=DEFAULT_SEED, shape=B2,
            av_form=AV_PAPER, radius=0.05, p_in=1e3, p_out=1e-5, steps=100,
            cfl=0.3) -> Problem:
    """Spherical blast in the unit cube, walls on all six faces."""
    h = 1.0 / n
    nn = (n, n, n)
    lo = (0.0, 0.0, 0.0)
    hi = (1.0, 1.0, 1.0)
    gamma = 1.4
    rng = np.random.default_rng(seed)
    x, _ = _lattice(nn, lo, h, 3, per_axis, jitter, rng)
    r2 = ((x - 0.5) ** 2).sum(axis=0)
    p = np.where(r2 < radius * radius, p_in, p_out)
    N = x.shape[1]
    ppc = per_axis ** 3
    rho = np.ones(N)
    return Problem(
        name=f"blast3d_{n}", dim=3, n=nn, lo=lo, hi=hi,
        faces=((WALL, WALL), (WALL, WALL), (WALL, WALL)),
        x=x, v=np.zeros((3, N)), mass=rho * h ** 3 / ppc, rho=rho,
        eint=p / ((gamma - 1.0) * rho), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, cfl=cfl,
        seed=seed, t_end=0.0, steps=steps)


def quadrant(n=256, per_axis=2, jitter=0.05, seed=DEFAULT_SEED, shape=B2,
             av_form=AV_PAPER, steps=200, cfl=0.3) -> Problem:
    """2x2-quadrant Riemann problem on the unit square; per-quadrant rho, p in
    U[0.1, 2] and velocity components in U(-0.7, 0.7) (|u| < 1)."""
    h = 1.0 / n
    nn = (n, n, 1)
    lo = (0.0, 0.0, 0.0)
    hi = (1.0, 1.0, 0.0)
    gamma = 1.4
    rng = np.random.default_rng(seed)
    q_rho = rng.uniform(0.1, 2.0, 4)
    q_p = rng.uniform(0.1, 2.0, 4)
    q_u = rng.uniform(-0.7, 0.7, (4, 2))
    x, _ = _lattice(nn, lo, h, 2, per_axis, jitter, rng)
    q = (x[0] >= 0.5).astype(int) + 2 * (x[1] >= 0.5).astype(int)
    N = x.shape[1]
    ppc = per_axis ** 2
    rho = q_rho[q]
    return Problem(
        name=f"quadrant_{n}", dim=2, n=nn, lo=lo, hi=hi,
        faces=((WALL, WALL), (WALL, WALL), (WALL, WALL)),
        x=x, v=q_u[q].T.copy(), mass=rho * h * h / ppc, rho=rho,
        eint=q_p[q] / ((gamma - 1.0) * rho), ids=np.arange(N, dtype=np.uint32),
        shape=shape, av_form=av_form, gamma=gamma, cfl=cfl,
        seed=seed, t_end=0.0, steps=steps)


def uniform_box(dim=2, n=16, per_axis=2, rho=1.0, p=1.0, u=(0.0, 0.0, 0.0),
                jitter=0.05, seed=DEFAULT_SEED, shape=B2, faces=None, steps=1,
                cfl=0.3) -> Problem:
    """A uniform state in a box; used by invariance checks."""
    h = 1.0 / n
    nn = _pad3((n,) * dim, 1)
    lo = (0.0, 0.0, 0.0)
    hi = _pad3((1.0,) * dim, 0.0)
    gamma = 1.4
    rng = np.random.default_rng(seed)
    x, _ = _lattice(nn, lo, h, dim, per_axis, jitter, rng)
    N = x.shape[1]
    ppc = per_axis ** dim
    v = np.zeros((dim, N))
    for a in range(dim):
        v[a] = u[a]
    if faces is None:
        faces = ((WALL, WALL),) * 3
    return Problem(
        name=f"uniform{dim}d_{n}", dim=dim, n=nn, lo=lo, hi=hi, faces=faces,
        x=x, v=v, mass=np.full(N, rho * h ** dim / ppc), rho=np.full(N, rho),
        eint=np.full(N, p / ((gamma - 1.0) * rho)), ids=np.arange(N, dtype=np.uint32),
        shape=shape, gamma=gamma, cfl=cfl, seed=seed, steps=steps)


def random_blob(dim=2, n=12, count=300, seed=DEFAULT_SEED, shape=B2, margin=3,
                faces=None) -> Problem:
    """Particles with random positions, masses and states kept `margin` cells
    away from every face; used by conservation checks."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = _pad3((n,) * dim, 1)
    hi = _pad3((1.0,) * dim, 0.0)
    x = rng.uniform(margin * h, 1.0 - margin * h, size=(dim, count))
    rho = rng.uniform(0.5, 2.0, count)
    p = rng.uniform(0.5, 2.0, count)
    gamma = 1.4
    if faces is None:
        faces = ((WALL, WALL),) * 3
    return Problem(
        name=f"blob{dim}d", dim=dim, n=nn, lo=(0.0, 0.0, 0.0), hi=hi, faces=faces,
        x=x, v=rng.uniform(-0.3, 0.3, size=(dim, count)),
        mass=rng.uniform(0.5, 1.5, count) * h ** dim / 4, rho=rho,
        eint=p / ((gamma - 1.0) * rho), ids=np.arange(count, dtype=np.uint32),
        shape=shape, gamma=gamma, seed=seed, steps=1,
        gradv=rng.uniform(-0.5, 0.5, size=(dim * dim, count)))


def linear_flow_box(A, gprev=None, n=12, rho=1.0, p=1.0) -> Problem:
    """Uniform gas on a regular 2x2 lattice (offsets 1/4, 3/4 of each cell,
    no jitter) moving with the linear velocity field v = A x; `gprev` (2x2)
    is the stored velocity gradient of every particle (None: zero).  Walls on
    all faces.  Used by closed-form checks of one step."""
    pb = uniform_box(dim=2, n=n, jitter=0.0, rho=rho, p=p)
    A = np.asarray(A, dtype=np.float64)
    pb.v = A @ pb.x
    if gprev is not None:
        pb.gradv = np.repeat(np.asarray(gprev, np.float64).reshape(4, 1), pb.n_particles, axis=1)
    pb.name = f"linear_flow_{n}"
    return pb


def outflow_drift(n=8, u=(0.1, 0.5)) -> Problem:
    """Pressureless gas on a regular 2x2 lattice moving uniformly with u;
    inflow (with the same u) at x_lo, outflow at the other three faces.  A
    time step that carries the top row through the y_hi face recycles it."""
    pb = uniform_box(dim=2, n=n, jitter=0.0, rho=1.0, p=0.0, u=(u[0], u[1], 0.0),
                     faces=((INFLOW, OUTFLOW), (OUTFLOW, OUTFLOW), (WALL, WALL)))
    pb.inflow_rho, pb.inflow_p, pb.inflow_u = 1.0, 0.0, (u[0], u[1], 0.0)
    pb.recycle_mass = float(pb.mass[0])
    pb.name = f"outflow_drift_{n}"
    return pb


def wall_escape(n=8, s=0.3, speed=1.0) -> Problem:
    """One pressureless particle at s cells from the x_lo wall, half-way up,
    moving at -speed along x; walls on all faces.  A time step beyond the
    CFL bound carries it through the wall."""
    h = 1.0 / n
    return Problem(
        name=f"wall_escape_{n}", dim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
        faces=((WALL, WALL),) * 3, x=np.array([[s * h], [0.5 + 0.5 * h]]),
        v=np.array([[-speed], [0.0]]), mass=np.array([h * h / 4]), rho=np.array([1.0]),
        eint=np.array([0.0]), ids=np.arange(1, dtype=np.uint32))


WORKLOADS = {
    "sod": sod,
    "cylinder": cylinder,
    "blast3d": blast3d,
    "sphere3d": sphere3d,
    "quadrant": quadrant,
}


# ------------------------------------------------------------------ serving --

@dataclasses.dataclass
class RequestSpec:
    """One request of the serving stream: arrival time (s), family, sizes,
    physical parameters and step count.  The particle cloud is built on
    admission by `build_request`."""

    req_id: int
    arrival: float
    family: str            # "sod" | "quadrant" | "cylinder"
    nx: int
    ny: int
    steps: int
    seed: int
    mach: float = 3.0


def request_stream(n=1000, rate=200.0, seed=2404) -> list:
    """Poisson stream of `n` requests at `rate` per second.  Families are drawn
    uniformly: Sod tubes nx in {256, ..., 4096} with ny = max(8, nx/256);
    2x2-quadrant Riemann problems on n^2 grids, n in {128, ..., 1024}; Mach
    2-4 cylinders nx in {256, 512, 1024} by nx/2.  Steps uniform in 200..2000."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        fam = ("sod", "quadrant", "cylinder")[int(rng.integers(3))]
        if fam == "sod":
            nx = int(rng.choice([256, 512, 1024, 2048, 4096]))
            ny = max(8, nx // 256)
        elif fam == "quadrant":
            nx = int(rng.choice([128, 256, 512, 1024]))
            ny = nx
        else:
            nx = int(rng.choice([256, 512, 1024]))
            ny = nx // 2
        out.append(RequestSpec(req_id=i, arrival=t, family=fam, nx=nx, ny=ny,
                               steps=int(rng.integers(200, 2001)),
                               seed=int(rng.integers(1 << 31)),
                               mach=float(rng.uniform(2.0, 4.0))))
    return out


class LatticeCache:
    """Jittered particle lattices (and cylinder masks / normals) per grid,
    built once with the default seed and shared by all requests of that grid;
    the per-request draws set the initial states, Mach number and steps."""

    def __init__(self):
        self._c = {}

    def get(self, key, make):
        if key not in self._c:
            self._c[key] = make()
        return self._c[key]


def build_request(spec: RequestSpec, cache: Optional[LatticeCache] = None) -> Problem:
    cache = cache or LatticeCache()
    gamma = 1.4
    if spec.family == "sod":
        def make():
            return sod(nx=spec.nx, ny=spec.ny, t_end=0.0)
        base = cache.get(("sod", spec.nx, spec.ny), make)
        pb = dataclasses.replace(base, steps=spec.steps, seed=spec.seed, name=f"req{spec.req_id}_{base.name}")
        return pb
    if spec.family == "quadrant":
        def make():
            return quadrant(n=spec.nx)
        base = cache.get(("quadrant", spec.nx), make)
        rng = np.random.default_rng(spec.seed)
        q_rho = rng.uniform(0.1, 2.0, 4)
        q_p = rng.uniform(0.1, 2.0, 4)
        q_u = rng.uniform(-0.7, 0.7, (4, 2))
        x = base.x
        q = (x[0] >= 0.5).astype(int) + 2 * (x[1] >= 0.5).astype(int)
        rho = q_rho[q]
        h = base.h
        return dataclasses.replace(
            base, name=f"req{spec.req_id}_{base.name}", v=q_u[q].T.copy(), rho=rho,
            mass=rho * h * h / 4, eint=q_p[q] / ((gamma - 1.0) * rho), steps=spec.steps, seed=spec.seed)
    def make():
        return cylinder(nx=spec.nx, ny=spec.ny, mach=3.0, steps=0)
    base = cache.get(("cylinder", spec.nx), make)
    v = np.zeros_like(base.v)
    v[0] = spec.mach
    return dataclasses.replace(base, name=f"req{spec.req_id}_{base.name}", v=v,
                               inflow_u=(spec.mach, 0.0, 0.0), steps=spec.steps, seed=spec.seed)
