"""The reach of a step, which the sampled full-size comparison of the 256^3
blast relies on (tests/subbox.py): the cells within 12 of a particle's cell,
cut out as a problem of their own with walls on the cut faces, reproduce the
particle's first three steps of the whole problem to FP64 rounding when the
same time steps are used.  Checked here on a 48^3 blast at the particles the
GPU test samples (the sphere of the pressure jump and its centre); the reach
is about 3 cells per step (radius 8 already leaves 2e-14 after 3 steps)."""
import numpy as np

from oracle import oracle as O
from paper_2404_17057_amd import workloads as W

import subbox as SB

STEPS = 3
RADIUS = 12


def test_subbox_reproduces_the_whole_problem_locally():
    pb = W.blast3d(n=48, steps=STEPS)
    o = O.Oracle(pb, threads=8)
    dts = []
    for _ in range(STEPS):
        dts.append(o.status()["dt_next"])
        assert o.step(1) == 0
    fields = (O.F_X, O.F_V, O.F_RHO, O.F_E)
    full = {f: o.particles(f) for f in fields}
    o.close()
    worst = 0.0
    for pid in SB.blast_samples(pb):
        sub, orig = SB.sub_problem(pb, SB.cell_of(pb, pid), RADIUS)
        assert sub.x.shape[1] < pb.x.shape[1]
        s = O.Oracle(sub)
        for dt in dts:
            s.set_dt(dt)
            assert s.step(1) == 0
        k = int(np.nonzero(orig == pid)[0][0])
        for f in fields:
            a = s.particles(f)[..., k]
            b = full[f][..., pid]
            worst = max(worst, float(np.abs(a - b).max() / np.abs(full[f]).max()))
        s.close()
    assert worst <= 1e-13, worst
