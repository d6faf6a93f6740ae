"""Writes tests/golden/horizon_*.json: the oracle's grid-projected density
of the two cylinder workloads at their full horizon, and the floor of what
any other arithmetic can reach there.

Workloads (seeded inputs of paper_2404_17057_amd.workloads):
  cylinder_512x256_ppc16  Mach-3 cylinder, 512x256 cells, 4x4 particles per
                          cell, 1000 steps (the precision ablation)
  cylinder_1024x512_ppc4  Mach-3 cylinder, 1024x512 cells, 2x2 particles per
                          cell, 2000 steps (the FP32 vs FP64 throughput run)

For each: the oracle runs the workload's steps (all host cores; the P2G sums
then differ from one thread by FP64 rounding) and reaches the time t.  A
second oracle whose initial positions are scaled by (1 + 1e-7 u),
u ~ U(-1, 1) seeded -- a perturbation the size of FP32 rounding -- runs to
that same time t (its time steps, a maximum over the particles, differ).  A
third oracle rounds its particle state to FP32 after every step (FP64
arithmetic, FP32 storage) and runs to t as well: the floor of an FP32-state
implementation, which carries a rounding of that size at every step rather
than once.
The grid-projected density (sum M phi / sum (M / rho) phi at the final
positions) is averaged over blocks of 16 x 16 nodes (block mass over block
volume); the fixture holds the oracle's block densities, t, and the relative
L1 of the block densities of the perturbed and of the FP32-state run against
them (the two floors).

Only oracle/ and the input generator are used.  Run from the repository
root: python tests/golden/make_horizon_fixtures.py [name ...]; a fixture
that already holds a reference run of the same steps keeps it, and a floor
it already holds is kept.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2404_17057_amd import workloads as W  # noqa: E402

BLOCK = 16
RUNS = {
    "cylinder_512x256_ppc16": (lambda: W.cylinder(nx=512, ny=256, per_axis=4, steps=1000), 1000),
    "cylinder_1024x512_ppc4": (lambda: W.cylinder(nx=1024, ny=512, steps=2000), 2000),
}


def block_density(mass, vol, nodes, block=BLOCK):
    """Block mass over block volume on blocks of block x block nodes (the
    last block of an axis may be smaller); NaN where a block has no volume."""
    nx, ny = nodes[0], nodes[1]
    m = mass.reshape(ny, nx)
    v = vol.reshape(ny, nx)
    by, bx = -(-ny // block), -(-nx // block)
    mb = np.zeros((by, bx))
    vb = np.zeros((by, bx))
    np.add.at(mb, (np.arange(ny)[:, None] // block, np.arange(nx)[None, :] // block), m)
    np.add.at(vb, (np.arange(ny)[:, None] // block, np.arange(nx)[None, :] // block), v)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(vb > 0, mb / vb, np.nan)


def rel_l1(a, b):
    ok = np.isfinite(a) & np.isfinite(b)
    return float(np.abs(a[ok] - b[ok]).sum() / np.abs(b[ok]).sum())


def run(pb, steps, threads, fp32_state=False):
    """steps > 0: that many steps; steps = 0: to pb.t_end."""
    o = O.Oracle(pb, threads=threads)
    if fp32_state:
        o.set_fp32_state(True)
    t0 = time.time()
    rc = o.step(steps)
    assert rc == 0, rc
    st = o.status()
    m, v = o.projected()
    rho = o.particles(O.F_RHO)
    blocks = block_density(m, v, o.nodes)
    o.close()
    return blocks, rho, st, time.time() - t0


def main(names):
    threads = os.cpu_count() or 1
    for name in names:
        make, steps = RUNS[name]
        out = os.path.join(ROOT, "tests", "golden", f"horizon_{name}.json")
        rec = json.load(open(out)) if os.path.exists(out) else {}
        pb = make()
        if rec.get("steps") == steps and "density_blocks" in rec:
            blocks = np.array([np.nan if v is None else v for v in rec["density_blocks"]]).reshape(rec["shape"])
            rho = None
            print(f"{name}: reference of {steps} steps kept, t = {rec['t']:.6f}", flush=True)
        else:
            blocks, rho, st, sec = run(pb, steps, threads)
            rec = {"workload": name, "steps": steps, "t": st["t"], "step": st["step"],
                   "oracle_threads": threads, "block_nodes": BLOCK, "shape": list(blocks.shape),
                   "density_blocks": [None if not np.isfinite(x) else float(x) for x in blocks.ravel()]}
            with open(out, "w") as f:
                json.dump(rec, f, separators=(",", ":"))
            print(f"{name}: oracle {steps} steps in {sec:.0f} s, t = {st['t']:.6f}", flush=True)
        if "floor_rel_l1_blocks" not in rec:
            pp = make()
            rng = np.random.default_rng(2404)
            pp.x = pp.x * (1.0 + 1e-7 * rng.uniform(-1.0, 1.0, size=pp.x.shape))
            pp.x = np.minimum(pp.x, np.array(pp.hi[:2])[:, None] * (1 - 1e-12))
            pp.t_end = rec["t"]
            blocks_p, rho_p, st_p, sec = run(pp, 0, threads)
            print(f"{name}: perturbed oracle to t in {sec:.0f} s, {st_p['step']} steps", flush=True)
            rec.update({
                "floor_rel_l1_blocks": rel_l1(blocks_p, blocks),
                "perturbed_steps": st_p["step"],
                "perturbation": "initial positions scaled by 1 + 1e-7 U(-1,1), seed 2404; run to the same t",
            })
            if rho is not None:
                rec["floor_rel_l1_particles"] = float(np.abs(rho_p - rho).sum() / np.abs(rho).sum())
            with open(out, "w") as f:
                json.dump(rec, f, separators=(",", ":"))
            print(f"{name}: floor blocks {rec['floor_rel_l1_blocks']:.3e} -> {out}", flush=True)
        if "floor_fp32_state_rel_l1_blocks" not in rec:
            pf = make()
            pf.t_end = rec["t"]
            blocks_f, _, st_f, sec = run(pf, 0, threads, fp32_state=True)
            print(f"{name}: FP32-state oracle to t in {sec:.0f} s, {st_f['step']} steps", flush=True)
            rec.update({
                "floor_fp32_state_rel_l1_blocks": rel_l1(blocks_f, blocks),
                "fp32_state_steps": st_f["step"],
            })
            with open(out, "w") as f:
                json.dump(rec, f, separators=(",", ":"))
            print(f"{name}: FP32-state floor blocks {rec['floor_fp32_state_rel_l1_blocks']:.3e} -> {out}",
                  flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(RUNS))
