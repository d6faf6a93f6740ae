"""The grid read-back that allocates nothing (mpm_read_grid_noalloc, fixed
32 MiB device scratch per GPU) against mpm_read_grid, through the C ABI.

Two calls in a row, the second on a smaller problem, each compared element
by element (both stage the same kernel's output, so bit for bit); a
snapshot larger than the scratch buffer is refused with MPM_E_SCRATCH.
"""
import numpy as np
import pytest

from paper_2404_17057_amd import mpm as G
from paper_2404_17057_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


WHICH = [G.G_M, G.G_P, G.G_F, G.G_PUPD, G.G_P2, G.G_FBC, G.G_FLAGS]


@pytest.mark.parametrize("prec", [G.FP32_FIX64, G.FP64])
def test_noalloc_read_grid_equals_read_grid(prec):
    _gpu()
    big = W.cylinder(nx=512, ny=256, steps=3)
    small = W.sod(nx=64, ny=2, t_end=0.0)
    for pb in (big, small):
        print(f"noalloc read-back: {pb.name}, prec {prec}", flush=True)
        s = G.Simulation(pb, prec)
        s.step(3)
        for w in WHICH:
            a = s.grid(w)
            b = s.grid_noalloc(w)
            assert a.shape == b.shape
            assert np.array_equal(a, b), (pb.name, w)
        # and again in the other order, after the other buffer's use
        b = s.grid_noalloc(G.G_P2)
        assert np.array_equal(b, s.grid(G.G_P2))
        s.close()


def test_noalloc_3d_and_too_large():
    _gpu()
    pb = W.blast3d(n=24, steps=2)
    s = G.Simulation(pb, G.FP32_FIX64)
    s.step(2)
    for w in (G.G_M, G.G_P2, G.G_FBC):
        assert np.array_equal(s.grid(w), s.grid_noalloc(w))
    s.close()
    # 1452^2 nodes x 2 components x 8 bytes > 32 MiB: refused, nothing staged
    big = W.wall_escape(n=1450)
    s = G.Simulation(big, G.FP64)
    s.step(1)
    with pytest.raises(G.MPMError) as ei:
        s.grid_noalloc(G.G_P)
    assert ei.value.code == G.E_SCRATCH
    # a scalar field of the same grid fits (16.9 MB)
    assert np.array_equal(s.grid_noalloc(G.G_M), s.grid(G.G_M))
