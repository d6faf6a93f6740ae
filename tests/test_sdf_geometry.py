"""Obstacles from sampled surface points (Sec. 3.2, `eq:sdf`; Sec. 4.1,
transonic aerofoil): the signed distance of a sampled profile, the cell mask
and the node normals taken as its gradient, and the NACA 4-digit section
that stands in for the OAT15a profile.

The pins are independent of the code under test: the exact signed distance
of a circle, the analytic circle normals, the area of the 4-digit thickness
polynomial integrated in closed form, the mirror symmetry of a symmetric
section and the sign convention of the angle of attack.
"""
import math

import numpy as np
import pytest

from paper_2404_17057_amd import workloads as W


def _ngon(center, r, k):
    a = np.linspace(0.0, 2 * math.pi, k, endpoint=False)
    return np.stack([center[0] + r * np.cos(a), center[1] + r * np.sin(a)])


def test_polygon_sdf_of_a_fine_ngon_is_the_circle_distance():
    c, r, k = (0.31, 0.27), 0.1, 720
    poly = _ngon(c, r, k)
    sag = r * (1 - math.cos(math.pi / k))          # inscribed polygon lies within this of the circle
    rng = np.random.default_rng(5)
    q = rng.uniform(0.0, 0.6, size=(2, 4000))
    exact = np.hypot(q[0] - c[0], q[1] - c[1]) - r
    got = W.polygon_sdf(poly, q[0], q[1])
    assert np.abs(got - exact).max() <= sag + 1e-12
    far = np.abs(exact) > sag
    assert np.array_equal(np.sign(got[far]), np.sign(exact[far]))
    # vertices lie on the profile
    assert np.abs(W.polygon_sdf(poly, poly[0], poly[1])).max() < 1e-15


@pytest.mark.parametrize("shape", [W.B2, W.Q1])
def test_sdf_obstacle_reproduces_the_circle_mask_and_normals(shape):
    n, lo, h = (128, 64, 1), (0.0, 0.0, 0.0), 1.0 / 128
    c, r = (0.3, 0.25), 0.08
    mask_c, normal_c = W.circle_obstacle(n, lo, h, 2, shape, c, r)
    poly = _ngon(c, r, 2000)
    mask_s, normal_s = W.sdf_obstacle(n, lo, h, shape, poly)
    assert mask_s.shape == mask_c.shape and normal_s.shape == normal_c.shape
    # masks agree except where a cell centre is closer to the circle than the chord error
    cx = lo[0] + (np.arange(n[0]) + 0.5) * h
    cy = lo[1] + (np.arange(n[1]) + 0.5) * h
    ccx, ccy = np.meshgrid(cx, cy, indexing="xy")
    close = np.abs(np.hypot(ccx - c[0], ccy - c[1]) - r).ravel() < r * (1 - math.cos(math.pi / 2000))
    assert np.array_equal(mask_s[~close], mask_c[~close])
    assert mask_c.sum() > 300
    # the gradient of the sampled distance points along (x - c) wherever the
    # distance is smooth over the difference stencil (away from the centre)
    nodes = np.stack(W._node_positions(n, lo, h, 2, shape))
    rr = np.hypot(nodes[0] - c[0], nodes[1] - c[1])
    sel = (rr > 4 * h) & (rr < r + 3 * h)
    dots = (normal_s[:, sel] * normal_c[:, sel]).sum(axis=0)
    assert sel.sum() > 200
    assert dots.min() > 0.999
    assert np.allclose(np.hypot(normal_s[0, sel], normal_s[1, sel]), 1.0)


def test_naca0012_symmetry_thickness_and_area():
    k = 400
    poly = W.naca4_profile("0012", chord=1.0, leading_edge=(0.0, 0.0), alpha_deg=0.0, n_side=k)
    assert poly.shape == (2, 2 * k - 1)
    upper, lower = poly[:, :k][:, ::-1], poly[:, k - 1:]    # both from the leading edge aft
    assert np.allclose(upper[0], lower[0], atol=1e-15)
    assert np.allclose(upper[1], -lower[1], atol=1e-15)
    assert poly[0, 0] == pytest.approx(1.0) and poly[0, k - 1] == pytest.approx(0.0, abs=1e-15)
    assert abs(poly[1, 0]) < 1e-5 and abs(poly[1, -1]) < 1e-5   # closed trailing edge
    assert 2 * upper[1].max() == pytest.approx(0.12, rel=2e-3)
    assert upper[0][np.argmax(upper[1])] == pytest.approx(0.30, abs=0.02)
    # area: the integral of 2 y_t over the chord, in closed form, is
    # 10 t (0.2969*2/3 - 0.1260/2 - 0.3516/3 + 0.2843/4 - 0.1036/5)
    exact = 10 * 0.12 * (0.2969 * 2 / 3 - 0.1260 / 2 - 0.3516 / 3 + 0.2843 / 4 - 0.1036 / 5)
    area = 0.5 * abs(np.dot(poly[0], np.roll(poly[1], -1)) - np.dot(poly[1], np.roll(poly[0], -1)))
    assert area == pytest.approx(exact, rel=1e-4)


def test_naca_angle_of_attack_raises_the_nose():
    alpha = 10.0
    poly = W.naca4_profile("2412", chord=2.0, leading_edge=(1.0, 1.0), alpha_deg=alpha, n_side=100)
    le, te = poly[:, 99], poly[:, 0]
    ang = math.degrees(math.atan2(te[1] - le[1], te[0] - le[0]))
    assert ang == pytest.approx(-alpha, abs=1e-9)
    assert math.hypot(te[0] - le[0], te[1] - le[1]) == pytest.approx(2.0, rel=1e-12)
    # the quarter-chord point stays where the unrotated section puts it
    q = le + 0.25 * (te - le)
    assert q == pytest.approx(np.array([1.5, 1.0]), abs=1e-12)
    # a rigid rotation: every surface point keeps its distance to the
    # quarter-chord point and the traversal keeps its sense
    flat = W.naca4_profile("2412", chord=2.0, leading_edge=(1.0, 1.0), alpha_deg=0.0, n_side=100)
    d_rot = np.hypot(poly[0] - q[0], poly[1] - q[1])
    d_flat = np.hypot(flat[0] - 1.5, flat[1] - 1.0)
    assert np.allclose(d_rot, d_flat, rtol=0, atol=1e-13)
    cross = lambda P: np.dot(P[0], np.roll(P[1], -1)) - np.dot(P[1], np.roll(P[0], -1))
    assert cross(poly) == pytest.approx(cross(flat), rel=1e-12)


def test_aerofoil_workload_mask_normals_and_particles():
    pb = W.aerofoil(nx=160, steps=10)
    nx, ny = pb.n[0], pb.n[1]
    assert (nx, ny) == (160, 108)
    h = pb.h
    mask = pb.cell_mask.reshape(ny, nx)
    assert 100 < mask.sum() < 400
    # no particle starts in a masked cell
    ci = np.floor((pb.x - np.array(pb.lo[:2])[:, None]) / h).astype(int)
    assert mask[ci[1], ci[0]].sum() == 0
    assert pb.n_particles == 4 * (nx * ny - mask.sum())
    # the normals of obstacle nodes (nodes inside masked cells) are unit
    # vectors pointing out of the profile: a small move along the normal
    # increases the signed distance
    poly = W.naca4_profile("2412", 0.12, (0.1, 0.135), -3.5, 200)
    nodes = np.stack(W._node_positions(pb.n, pb.lo, h, 2, pb.shape))
    cell = np.clip(np.floor((nodes - np.array(pb.lo[:2])[:, None]) / h).astype(int),
                   0, np.array([[nx - 1], [ny - 1]]))
    obst = mask[cell[1], cell[0]] != 0
    nrm = pb.node_normal[:, obst]
    assert np.allclose(np.hypot(nrm[0], nrm[1]), 1.0)
    p = nodes[:, obst]
    sd0 = W.polygon_sdf(poly, p[0], p[1])
    near = sd0 > -0.5 * h                       # within half a cell of the surface
    eps = 0.1 * h
    sd1 = W.polygon_sdf(poly, p[0] + eps * nrm[0], p[1] + eps * nrm[1])
    assert near.sum() > 20
    assert np.all(sd1[near] > sd0[near] + 0.5 * eps)
