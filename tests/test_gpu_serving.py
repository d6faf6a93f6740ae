"""Served results equal the same problems run alone (fixed-point precision,
bit for bit), with requests arriving while others run, and match the FP64
oracle within the FP32 tolerance (relative L1 of density <= 1e-3)."""
import hashlib

import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_17057_amd import mpm as G
from paper_2404_17057_amd import serving as S
from paper_2404_17057_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(11)
    specs = []
    t = 0.0
    fams = ["sod", "quadrant", "cylinder"]
    for i in range(10):
        t += rng.exponential(0.004)
        fam = fams[i % 3]
        nx = {"sod": 256, "quadrant": 64, "cylinder": 128}[fam]
        ny = {"sod": 8, "quadrant": 64, "cylinder": 64}[fam]
        specs.append(W.RequestSpec(req_id=i, arrival=t, family=fam, nx=nx, ny=ny,
                                   steps=int(rng.integers(20, 90)), seed=int(rng.integers(1 << 30)),
                                   mach=float(rng.uniform(2, 4))))
    cache = W.LatticeCache()
    build = lambda s: W.build_request(s, cache)
    be = S.GPUBackend(G.FP32_FIX64)
    srv = S.Server(be, build, hbm_budget=1 << 30, max_slots=4, steps_per_launch=16)
    done = srv.run(specs)
    assert len(done) == len(specs) and all(d.status == 0 for d in done)
    # the requests really shared launches, and some were admitted while a
    # batch was on the device
    assert max(srv.batch_sizes) > 1
    assert srv.overlapped_admissions >= 1
    for d in done:
        spec = specs[d.req_id]
        sim = G.Simulation(build(spec), G.FP32_FIX64)
        sim.step(spec.steps)
        rho = sim.field(G.F_RHO)
        sim.close()
        assert hashlib.sha256(rho.tobytes()).hexdigest() == d.digest, spec
        # the served result (the same bits) against the oracle
        o = O.Oracle(build(spec))
        o.step(spec.steps)
        ref = o.particles(O.F_RHO)
        o.close()
        assert np.abs(rho - ref).sum() / np.abs(ref).sum() <= 1e-3, spec
    summ = S.summarize(done)
    assert summ["requests"] == 10


def test_failing_request_does_not_disturb_the_others():
    """A request whose flow turns non-physical (colliding streams at 40 times
    the CFL bound: J <= 0 in its first steps) ends with MPM_E_NONPHYSICAL,
    while the requests batched with it keep results bit-identical to their
    runs alone."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bad = W.uniform_box(dim=2, n=8, jitter=0.0)
    bad.v[0] = np.where(bad.x[0] < 0.5, 5.0, -5.0)
    bad.cfl = 40.0
    fams = ["sod", "quadrant", "cylinder"]
    specs = []
    for i in range(6):
        fam = fams[i % 3]
        nx = {"sod": 256, "quadrant": 64, "cylinder": 128}[fam]
        ny = {"sod": 8, "quadrant": 64, "cylinder": 64}[fam]
        specs.append(W.RequestSpec(req_id=i, arrival=0.001 * i, family=fam, nx=nx, ny=ny,
                                   steps=40 + 5 * i, seed=100 + i, mach=3.0))
    cache = W.LatticeCache()
    build = lambda s: bad if s.req_id == 2 else W.build_request(s, cache)
    srv = S.Server(S.GPUBackend(G.FP32_FIX64), build, hbm_budget=1 << 30, max_slots=6, steps_per_launch=16)
    done = {d.req_id: d for d in srv.run(specs)}
    assert len(done) == len(specs)
    assert max(srv.batch_sizes) > 1
    assert srv.overlapped_admissions >= 1
    assert done[2].status == G.E_NONPHYSICAL
    for i, spec in enumerate(specs):
        if i == 2:
            continue
        assert done[i].status == 0, i
        sim = G.Simulation(build(spec), G.FP32_FIX64)
        sim.step(spec.steps)
        rho = sim.field(G.F_RHO)
        sim.close()
        assert hashlib.sha256(rho.tobytes()).hexdigest() == done[i].digest, spec
