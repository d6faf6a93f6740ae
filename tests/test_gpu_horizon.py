"""The cylinder workloads at their full horizon against the oracle, on the
grid-projected density (sum M phi / sum (M / rho) phi at the final positions,
averaged over blocks of 16 x 16 nodes), beside the floor of the problem.

The flow is chaotic at these horizons: outflow recycling makes discrete
choices, and the time step is a maximum over the particles, so after the
workload's steps two runs differing by rounding have reached different
times.  The comparison is at equal time: the fixture holds the time t the
oracle reaches in the workload's steps, and the GPU runs to that t.  Two
floors come with it (tests/golden/horizon_*.json, written by
tests/golden/make_horizon_fixtures.py from the oracle alone): a perturbation
the size of FP32 rounding once, at the start (initial positions scaled by
1 + 1e-7 u), moves the oracle's result at t by the first; rounding the
oracle's particle state to FP32 after every step, as an FP32-state code
stores it, moves it by the second.  A GPU result whose distance to the
oracle is within twice the floor of what it carries cannot be told apart
from the oracle at this horizon; that is the bar: the first floor for the
FP64 path, the larger of the two for the FP32-state fixed-point path.
"""
import json
import os

import numpy as np
import pytest

from paper_2404_17057_amd import mpm as G
from paper_2404_17057_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MAKE = {
    "cylinder_512x256_ppc16": lambda: W.cylinder(nx=512, ny=256, per_axis=4, steps=1000),
    "cylinder_1024x512_ppc4": lambda: W.cylinder(nx=1024, ny=512, steps=2000),
}


def block_density(mass, vol, nodes, block):
    """Block mass over block volume on blocks of block x block nodes."""
    nx, ny = nodes[0], nodes[1]
    m = mass.reshape(ny, nx)
    v = vol.reshape(ny, nx)
    by, bx = -(-ny // block), -(-nx // block)
    mb = np.zeros((by, bx))
    vb = np.zeros((by, bx))
    iy = np.arange(ny)[:, None] // block
    ix = np.arange(nx)[None, :] // block
    np.add.at(mb, (iy, ix), m)
    np.add.at(vb, (iy, ix), v)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(vb > 0, mb / vb, np.nan)


@pytest.mark.parametrize("prec", [G.FP32_FIX64, G.FP64])
@pytest.mark.parametrize("name", list(MAKE))
def test_full_horizon_projected_density(name, prec):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    path = os.path.join(GOLDEN, f"horizon_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    fx = json.load(open(path))
    if "floor_rel_l1_blocks" not in fx:
        pytest.skip(f"{path} holds no floor yet")
    floor = fx["floor_rel_l1_blocks"]
    if prec != G.FP64:
        if "floor_fp32_state_rel_l1_blocks" not in fx:
            pytest.skip(f"{path} holds no FP32-state floor yet")
        floor = max(floor, fx["floor_fp32_state_rel_l1_blocks"])
    ref = np.array([np.nan if v is None else v for v in fx["density_blocks"]]).reshape(fx["shape"])
    pb = MAKE[name]()
    pb.t_end = fx["t"]
    print(f"full horizon: {name}, to t = {fx['t']:.6f} (oracle: {fx['steps']} steps), prec {prec}", flush=True)
    s = G.Simulation(pb, prec)
    s.step(0)
    st = s.status()
    # the step count to reach t is not compared: the time step follows the
    # fastest particle, whose FLIP velocity noise differs from run to run
    # (the perturbed oracle takes far more steps to the same t)
    assert st["rc"] == 0 and st["t"] == fx["t"]
    got = block_density(s.grid(G.G_MPROJ), s.grid(G.G_VOLPROJ), s.nodes, fx["block_nodes"])
    ok = np.isfinite(got) & np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), np.isfinite(ref))
    l1 = float(np.abs(got[ok] - ref[ok]).sum() / np.abs(ref[ok]).sum())
    print(f"  rel L1 of the block density vs oracle {l1:.3e}, floor {floor:.3e}, steps {st['step']}", flush=True)
    assert l1 <= 2.0 * floor
