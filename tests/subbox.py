"""A sub-problem of the cells around one particle, for checking a full-size
launch at sampled particles with the oracle.

One step of the method reaches a bounded neighbourhood: a particle's update
reads the re-mapped momentum of its stencil nodes, which sums the updated
velocities of the particles around them, which read the nodes of the first
P2G around those.  The cells within R of a particle's cell, taken with their
particles as a problem of their own (walls on the cut faces), therefore
reproduce that particle's first steps exactly when R exceeds the reach of
those steps plus the wall layer at the cut; `tests/test_subbox.py` checks
the radius on the CPU against the whole problem.

Test support only: no method arithmetic, only the selection of cells and
particles.
"""
import dataclasses

import numpy as np


_CELLS = {}


def particle_cells(pb):
    """Cell indices (dim, N) of the initial positions, computed once per
    problem object."""
    key = id(pb)
    if key not in _CELLS or _CELLS[key][0] is not pb:
        n = np.array(pb.n[:pb.dim])
        lo = np.array(pb.lo[:pb.dim], dtype=float)
        h = (pb.hi[0] - pb.lo[0]) / pb.n[0]
        cells = np.floor((pb.x - lo[:, None]) / h).astype(np.int32)
        np.clip(cells, 0, (n - 1)[:, None], out=cells)
        _CELLS.clear()
        _CELLS[key] = (pb, cells)
    return _CELLS[key][1]


def sub_problem(pb, center_cell, radius, fp32_state=False):
    """The cells within `radius` (per axis) of `center_cell`, clipped to the
    domain, with the particles inside them.  Returns (problem, orig_ids):
    the sub-problem's ids are 0..m-1 in the order of the original ids, and
    orig_ids[i] is the original id of sub-problem id i.  fp32_state rounds
    the particle state to FP32 (the state an FP32 implementation starts
    from)."""
    assert all(f == (0, 0) for f in pb.faces[:pb.dim]), "walls on every face only"
    dim = pb.dim
    n = np.array(pb.n[:dim])
    lo = np.array(pb.lo[:dim], dtype=float)
    h = (pb.hi[0] - pb.lo[0]) / pb.n[0]
    cells = particle_cells(pb)
    c = np.asarray(center_cell[:dim], dtype=np.int64)
    c0 = np.maximum(c - radius, 0)
    c1 = np.minimum(c + radius + 1, n)
    sel = np.all((cells >= c0[:, None]) & (cells < c1[:, None]), axis=0)
    idx = np.nonzero(sel)[0]
    idx = idx[np.argsort(pb.ids[idx], kind="stable")]
    orig = pb.ids[idx].astype(np.int64)

    def st(a):
        return a.astype(np.float32).astype(np.float64) if fp32_state else a.copy()

    new_lo = tuple(float(v) for v in lo + c0 * h) + tuple(pb.lo[dim:])
    new_hi = tuple(float(v) for v in lo + c1 * h) + tuple(pb.hi[dim:])
    new_n = tuple(int(v) for v in (c1 - c0)) + tuple(pb.n[dim:])
    sub = dataclasses.replace(
        pb, name=pb.name + "_sub", n=new_n, lo=new_lo, hi=new_hi,
        x=st(pb.x[:, idx]), v=st(pb.v[:, idx]), mass=st(pb.mass[idx]), rho=st(pb.rho[idx]),
        eint=st(pb.eint[idx]), ids=np.arange(idx.size, dtype=np.uint32),
        gradv=None if pb.gradv is None else st(pb.gradv[:, idx]),
        cell_mask=None, node_normal=None, t_end=0.0)
    return sub, orig


def cell_of(pb, pid):
    """Cell of the particle whose id is pid (initial positions)."""
    k = int(np.nonzero(pb.ids == pid)[0][0])
    return tuple(int(v) for v in particle_cells(pb)[:, k])


def blast_samples(pb, radius_frac=1.0):
    """Ids of the particles nearest to seven points of the blast: six on the
    sphere of the initial pressure jump (radius 0.05 about the centre, along
    +-x, +-y, +-z) and the centre itself."""
    r = 0.05 * radius_frac
    pts = [(0.5, 0.5, 0.5)] + [tuple(0.5 + s * r * (a == b) for b in range(3)) for a in range(3) for s in (-1, 1)]
    out = []
    for p in pts:
        d2 = ((pb.x - np.array(p)[:, None]) ** 2).sum(axis=0)
        out.append(int(pb.ids[int(np.argmin(d2))]))
    return out
