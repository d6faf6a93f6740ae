#!/usr/bin/env python3
"""Throughput of the MPM hot path on one MI355X.

Workload: Mach-3 flow past a cylinder (r = 0.05 at (0.3, 0.25)) in
[0,1]x[0,0.5], 1024x512 cells, 2x2 jittered particles per fluid cell
(2,064,184 particles), quadratic B-splines, CFL 0.3.  A step is one pass of
the whole path: cell sort, P2G, boundary conditions and grid update, G2P and
velocity update, P2G of the updated momentum, G2PD and particle update, move
with outflow recycling, time step.  Inputs are resident in HBM before the
timed region; the timed region is `--steps` steps (graph replays) bracketed
by device synchronisation, timed with HIP events on the launch stream.

Prints one JSON line: FP32 state with 64-bit fixed-point P2G (the headline
value), the plain FP64 path beside it, the per-sweep times and the roofline
of the dominant sweep, the FP64 oracle timed on the host cores on a bounded
sample of the same workload, and the relative L1 density error of both GPU
paths against the oracle after that sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (P2G+grid+G2P) FP32 vs FP64 plain at L1 err; p50/p99 serve"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes(pb, nnodes, ncells, real_sz, acc_sz):
    """Algorithmic bytes per launch of each sweep: every particle field and
    grid word the sweep must read or write, counted once (no halo re-reads,
    no clearing of the next step's buffers, no atomic retries)."""
    d = pb.dim
    N = pb.n_particles
    r = real_sz
    # grid words: 2D grids hold finished sums in the state precision, 3D
    # grids the accumulator words their atomics need
    a = real_sz if d == 2 else acc_sz
    nq = 1 + 2 * d
    return {
        # X, V, M, rho, e, tr G in; m, p, dt f out; cell offsets in
        "p2g": N * (2 * d + 4) * r + ncells * 4 + nnodes * nq * a,
        # 2D frame-node sums of the P2G (halo records in, grid out): an
        # overhead of the P2G's tiling, not algorithmic (S1 counts the grid)
        "frame_reduce": 0,
        # X, V, M in (the id only for a recycled particle); rank out; m, p,
        # dt f, flags in; p2 out; offsets in (V' and the new key are
        # recomputed by the update sweep)
        "g2p_p2g": N * ((2 * d + 1) * r + 4) + ncells * 4 + nnodes * (nq * a + 1 + d * a),
        # tile totals in, tile bases out
        "tilescan": (ncells // 256) * 8,
        # cell counts in, offsets out
        "cellscan": ncells * 8,
        # X, V, M, rho, e, tr G, id, rank in; X, V', M, rho, e, tr G, id out
        # (the whole G only in the last step of a run); m, p, dt f, p2,
        # flags in
        "update": N * ((2 * d + 4) * r + 8 + (2 * d + 4) * r + 4) + nnodes * ((1 + 3 * d) * a + 1),
        "finalize": 0,
    }


def survey_bytes(dim, N, nnodes):
    """Algorithmic bytes per launch of the three particle sweeps as the hot-
    path scope defines them: FP32 particle fields, 8-byte grid words, no
    sort, halo or clearing.  S1 reads X, V, M, rho, e and diag G and writes
    m, p, dt f; S2 reads X, V, M and those grid words and writes V and p2;
    S3 reads X, rho, e, diag G (and M in 3D), the grid words it needs, and
    writes X, rho, e, G (and Vol in 3D)."""
    d = dim
    s3_part = (2 * d + 2 + d + 2 + d * d) * 4 if d == 2 else (2 * d + 3 + d + 3 + d * d) * 4
    return {
        "p2g": N * (3 * d + 3) * 4 + nnodes * (1 + 2 * d) * 8,
        "g2p_p2g": N * (3 * d + 1) * 4 + nnodes * (1 + 3 * d) * 8,
        "update": N * s3_part + nnodes * (1 + 3 * d) * 8,
    }


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("mpm_kernels.hip", "mpm_device.hpp", "mpm_common.hpp"):
        with open(os.path.join(ROOT, "paper_2404_17057_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload, src_hash):
    """Per-launch rocprofv3 figures of a kernel from the committed counter
    summary (HBM bytes, VALU wave-instructions), valid only while the kernel
    source is the one the counters were taken from; else {}."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    try:
        data = json.load(open(path))
        rec = data.get(workload, {}).get(kernel)
        if rec and rec.get("source_hash") == src_hash:
            return rec
    except Exception:
        return {}
    return {}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Measured device-to-device copy bandwidth (GB/s, bytes read + written):
    the HBM rate a plain streaming kernel reaches on this device."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbps, 1)


def time_gpu(pb, precision, steps, warmup, profile_steps):
    """Steps/s of one precision mode.  The first mpm_step call of a problem
    captures its step graphs (host work, before anything is timed); its host
    time is reported as `graph_setup_ms`.  The warm-up is that first call,
    so the timed steps are graph replays only."""
    import torch
    from paper_2404_17057_amd import mpm as G
    sim = G.Simulation(pb, precision)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(max(warmup, 1))
    setup_ms = (time.perf_counter() - t0) * 1e3   # asynchronous call: capture + enqueue
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = sim.status()
    if st["rc"] != 0:
        raise RuntimeError(f"device error {st['rc']} during the timed steps")
    out = dict(ms_total=ms, ms_per_step=ms / steps, value=pb.n_particles * steps / (ms * 1e-3),
               nodes=sim.nnodes, counters=[int(c) for c in sim.counters()], t=st["t"], step=st["step"],
               graph_setup_ms=round(setup_ms, 3), warmup_steps=max(warmup, 1))
    sim.close()
    del sim
    # Per-sweep times over the same span of steps as the timed region (a
    # fresh run: the same warm-up, then profile_steps steps, by default as
    # many as were timed), one HIP event pair per sweep
    prof = {}
    if profile_steps != 0:
        sim = G.Simulation(pb, precision)
        sim.step(max(warmup, 1))
        prof = sim.profile(steps if profile_steps < 0 else profile_steps)
        sim.close()
        del sim
    out["sweeps_ms"] = prof
    torch.cuda.empty_cache()
    return out


def host_inclusive(pb, precision, steps):
    """Throughput with the host hand-over counted, by the host clock: the
    library's init from host arrays (checks, workspace, copy to the device,
    initial sort), `steps` steps, and the read-back of the particle state
    (X, V, M, rho, e) in id order.  Reported beside `value`, never as it."""
    import torch
    from paper_2404_17057_amd import mpm as G
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = G.Simulation(pb, precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.read([G.F_X, G.F_V, G.F_M, G.F_RHO, G.F_E])
    t3 = time.perf_counter()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"value": round(pb.n_particles * steps / (t3 - t0), 1), "unit": "particle-steps/s",
            "steps": steps, "init_s": round(t1 - t0, 4), "steps_s": round(t2 - t1, 4),
            "read_s": round(t3 - t2, 4)}


def run_sample_gpu(pb, precision, steps):
    from paper_2404_17057_amd import mpm as G
    sim = G.Simulation(pb, precision)
    sim.step(steps)
    rho = sim.field(G.F_RHO)
    sim.close()
    return rho


def ablation(args):
    """Accumulation precision on the 512x256 cylinder, 4x4 particles per cell:
    FP32 state with FP64 atomics, FP32 atomics or int64 fixed point (and
    the plain FP64 path).  Per precision: two runs of `--ablation-steps`
    steps compared bit for bit, the largest relative gap between the grid
    mass and the particle mass seen every 10 steps, throughput, and the L1
    density error against the oracle after `--ablation-oracle-steps`."""
    import numpy as np
    from paper_2404_17057_amd import mpm as G
    from paper_2404_17057_amd import workloads as W
    from oracle import oracle as O
    pb = W.cylinder(nx=512, ny=256, per_axis=4, steps=args.ablation_steps)
    # reference mass: the particle masses as the state holds them (FP32 in
    # the FP32 modes), so the drift measures the grid sums, not the rounding
    # of the inputs
    M0s = {"fp64": float(pb.mass.sum()), "fp32": float(pb.mass.astype(np.float32).astype(np.float64).sum())}
    o = O.Oracle(pb)
    o.step(args.ablation_oracle_steps)
    rho_o = o.particles(O.F_RHO)
    o.close()
    out = {"workload": f"cylinder_mach3_512x256_ppc16 ({pb.n_particles} particles)",
           "steps": args.ablation_steps, "oracle_steps": args.ablation_oracle_steps, "modes": {}}
    for name, prec in (("fp32_acc_f64", G.FP32_ACC_F64), ("fp32_acc_f32", G.FP32_ACC_F32),
                       ("fp32_fix64", G.FP32_FIX64), ("fp64", G.FP64), ("fp64_colouring", G.FP64_COLOR)):
        rec = {}
        s = G.Simulation(pb, prec)
        s.step(args.ablation_oracle_steps)
        rho = s.field(G.F_RHO)
        rec["rel_l1_density_vs_oracle"] = float(np.abs(rho - rho_o).sum() / np.abs(rho_o).sum())
        s.close()
        finals = []
        for run in range(2):
            s = G.Simulation(pb, prec)
            drift = 0.0
            done = 0
            t0 = time.perf_counter()
            while done < args.ablation_steps:
                k = min(10, args.ablation_steps - done)
                s.step(k)
                done += k
                if run == 0:
                    M0 = M0s["fp64" if prec in (G.FP64, G.FP64_COLOR) else "fp32"]
                    drift = max(drift, abs(float(s.grid(G.G_M).sum()) - M0) / M0)
            if run == 1:
                torch_sync()
                rec["particle_steps_per_s_incl_readbacks"] = pb.n_particles * done / (time.perf_counter() - t0)
            else:
                rec["max_rel_mass_drift"] = drift
            finals.append(s.read([G.F_X, G.F_RHO, G.F_V]))
            rec["status"] = s.status()["rc"]
            s.close()
        rec["bitwise_reproducible"] = all(np.array_equal(finals[0][f], finals[1][f]) for f in finals[0])
        rec["run_to_run_max_rel_density_diff"] = float(np.abs(finals[0][G.F_RHO] - finals[1][G.F_RHO]).max()
                                                      / np.abs(finals[0][G.F_RHO]).max())
        out["modes"][name] = rec
        log(f"ablation {name}: {rec}")
    return {"metric": "precision ablation (configs[3])", **out}


def blast3d(args):
    """The 3D spherical blast on the 256^3 grid (2x2x2 particles per cell,
    134M particles, FP32 state with int64 fixed-point P2G): particle-steps/s
    over `--blast-steps` steps after `--blast-warmup`, the per-sweep times and
    the step's algorithmic HBM bytes; optionally the L1 density and pressure
    error against the oracle on the 64^3 downscale after
    `--blast-oracle-steps` steps."""
    import numpy as np
    from paper_2404_17057_amd import mpm as G
    from paper_2404_17057_amd import workloads as W
    pb = W.blast3d(n=args.blast_n, steps=args.blast_steps)
    log(f"blast3d {args.blast_n}^3: {pb.n_particles} particles")
    r = time_gpu(pb, G.FP32_FIX64, args.blast_steps, args.blast_warmup, args.blast_profile_steps)
    nt = [(args.blast_n + 7) // 8, (args.blast_n + 7) // 8, (args.blast_n + 3) // 4]
    b = sweep_bytes(pb, r["nodes"], nt[0] * nt[1] * nt[2] * 256, 4, 8)
    step_bytes = sum(b.values())
    sb = survey_bytes(3, pb.n_particles, r["nodes"])
    sw = r["sweeps_ms"]
    dom = max(("p2g", "g2p_p2g", "update"), key=lambda k: sw.get(k, 0.0)) if sw else "p2g"
    roof = None
    if sw:
        dom_ms = sw[dom]
        ach = sb[dom] / (dom_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "kernel_ms": round(dom_ms, 4),
                "algorithmic_bytes_per_launch": int(sb[dom]), "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                "sweeps_frac": {k: round(sb[k] / (sw[k] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
                                for k in sb if sw.get(k)}}
        # measured HBM bytes and VALU issue of the dominant sweep from the
        # committed counters (None once the kernels changed)
        counters = measured_counters(dom, pb.name, kernel_source_hash())
        valu = counters.get("sq_insts_valu")
        roof["traffic"] = counters.get("bytes_per_launch")
        roof["valu_issue_frac"] = round(valu * 4 / (1024 * 2.4e9 * dom_ms * 1e-3), 3) if valu else None
    out = {"workload": f"blast3d_{args.blast_n}^3_ppc8", "particles": pb.n_particles,
           "steps": args.blast_steps, "warmup": r["warmup_steps"],
           "value": round(r["value"], 1), "unit": "particle-steps/s",
           "ms_per_step": round(r["ms_per_step"], 4), "graph_setup_ms": r["graph_setup_ms"],
           "sweeps_ms": sw, "roofline": roof,
           "step_algorithmic_bytes_scope": int(sum(sb.values())),
           "step_achieved_GBps_scope": round(sum(sb.values()) / (r["ms_per_step"] * 1e-3) / 1e9, 1),
           "step_algorithmic_bytes": int(step_bytes),
           "counters": r["counters"]}
    if args.blast_fp64:
        r64 = time_gpu(pb, G.FP64, args.blast_steps, args.blast_warmup, 0)
        out["fp64"] = {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 4)}
    del pb
    if args.blast_oracle_steps > 0:
        from oracle import oracle as O
        small = W.blast3d(n=64, steps=args.blast_oracle_steps)
        o = O.Oracle(small, threads=os.cpu_count() or 1)
        o.step(args.blast_oracle_steps)
        s = G.Simulation(small, G.FP32_FIX64)
        s.step(args.blast_oracle_steps)
        l1 = lambda a, ref: float(np.abs(a - ref).sum() / np.abs(ref).sum())
        out["accuracy_64^3"] = {"steps": args.blast_oracle_steps, "oracle_threads": o.threads,
                                "rel_l1_density": l1(s.field(G.F_RHO), o.particles(O.F_RHO)),
                                "rel_l1_pressure": l1(s.field(G.F_P), o.particles(O.F_P))}
        s.close()
        o.close()
    log(f"blast3d: {out}")
    return out


def aerofoil(args):
    """Transonic flow (Mach 0.73) past a NACA 2412 section on [0,0.4] x
    [0,0.27] whose mask and normals come from the sampled signed distance
    (FP32 state with int64 fixed-point P2G): particle-steps/s over
    `--aerofoil-steps` steps after the bench warm-up, the per-sweep times;
    optionally the L1 density error against the oracle on the 160-cell
    downscale after `--aerofoil-oracle-steps` steps."""
    import numpy as np
    from paper_2404_17057_amd import mpm as G
    from paper_2404_17057_amd import workloads as W
    pb = W.aerofoil(nx=args.aerofoil_nx, steps=args.aerofoil_steps)
    log(f"aerofoil {pb.n[0]}x{pb.n[1]}: {pb.n_particles} particles, {int(pb.cell_mask.sum())} masked cells")
    r = time_gpu(pb, G.FP32_FIX64, args.aerofoil_steps, args.warmup, -1)
    out = {"workload": pb.name, "particles": pb.n_particles, "masked_cells": int(pb.cell_mask.sum()),
           "steps": args.aerofoil_steps, "warmup": args.warmup,
           "value": round(r["value"], 1), "unit": "particle-steps/s",
           "ms_per_step": round(r["ms_per_step"], 5), "sweeps_ms": r["sweeps_ms"],
           "t_reached": round(r["t"], 6), "counters": r["counters"]}
    del pb
    if args.aerofoil_oracle_steps > 0:
        from oracle import oracle as O
        small = W.aerofoil(nx=160, steps=args.aerofoil_oracle_steps)
        o = O.Oracle(small)
        o.step(args.aerofoil_oracle_steps)
        s = G.Simulation(small, G.FP32_FIX64)
        s.step(args.aerofoil_oracle_steps)
        l1 = lambda a, ref: float(np.abs(a - ref).sum() / np.abs(ref).sum())
        out["accuracy_160x108"] = {"steps": args.aerofoil_oracle_steps,
                                   "rel_l1_density": l1(s.field(G.F_RHO), o.particles(O.F_RHO)),
                                   "rel_l1_pressure": l1(s.field(G.F_P), o.particles(O.F_P))}
        s.close()
        o.close()
    log(f"aerofoil: {out}")
    return out


def torch_sync():
    import torch
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--profile-steps", type=int, default=-1,
                    help="steps of the per-sweep profile (-1: as many as timed, 0: none)")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="oracle steps timed on the host (bounded sample)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving stream (Poisson, 200/s, seed 2404; 0 = skip)")
    ap.add_argument("--serve-sustained-requests", type=int, default=300,
                    help="requests of the second serving run, offered at 70 %% of the measured capacity")
    ap.add_argument("--no-serve-sustained", action="store_true",
                    help="skip the second serving run at 70 %% of the measured capacity")
    ap.add_argument("--ablation", action="store_true",
                    help="precision ablation on the 512x256 cylinder with 4x4 particles per cell "
                         "(prints its own JSON line instead of the throughput line)")
    ap.add_argument("--ablation-steps", type=int, default=1000)
    ap.add_argument("--ablation-oracle-steps", type=int, default=10)
    ap.add_argument("--no-blast3d", action="store_true",
                    help="skip the 3D blast leg (256^3 grid, 134M particles), reported beside the line")
    ap.add_argument("--only-blast3d", action="store_true",
                    help="run the 3D blast leg alone and print its JSON object (profiling runs)")
    ap.add_argument("--blast-profile-steps", type=int, default=-1,
                    help="steps of the 3D per-sweep profile (-1: as many as timed, 0: none)")
    ap.add_argument("--blast-n", type=int, default=256)
    ap.add_argument("--blast-steps", type=int, default=100)
    ap.add_argument("--blast-warmup", type=int, default=16)
    ap.add_argument("--blast-fp64", action="store_true",
                    help="also time the 3D blast with the plain FP64 state")
    ap.add_argument("--blast-oracle-steps", type=int, default=4,
                    help="oracle steps of the 64^3 downscale for the accuracy figure, on all host "
                         "cores (0 = skip)")
    ap.add_argument("--colouring", action="store_true",
                    help="also time the FP64 state with the grid-colouring P2G (no atomics) beside the "
                         "LDS-tile FP64 path, with per-sweep times")
    ap.add_argument("--all-precisions", action="store_true",
                    help="also time the FP32 state with FP64 and with FP32 accumulators on the same workload")
    ap.add_argument("--aerofoil", action="store_true",
                    help="also time the transonic aerofoil (sampled-SDF obstacle) and report it beside the line")
    ap.add_argument("--aerofoil-nx", type=int, default=1024)
    ap.add_argument("--aerofoil-steps", type=int, default=2000)
    ap.add_argument("--aerofoil-oracle-steps", type=int, default=0,
                    help="steps of the 160-cell aerofoil run against the oracle (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain device copies of 256 MiB (reference for counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent problems would shard one per GPU with no exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2404_17057_amd import mpm as G
    from paper_2404_17057_amd import workloads as W

    torch.cuda.set_device(0)
    if args.only_blast3d:
        print(json.dumps({"metric": "3D blast leg alone", **blast3d(args)}), flush=True)
        return
    if args.ablation:
        print(json.dumps(ablation(args)), flush=True)
        return
    pb = W.cylinder(nx=args.nx, ny=args.nx // 2)
    N = pb.n_particles
    log(f"workload {pb.name}: {N} particles")

    fix = time_gpu(pb, G.FP32_FIX64, args.steps, args.warmup, args.profile_steps)
    log(f"fp32_fix64: {fix['ms_per_step']:.4f} ms/step, {fix['value']:.4e} particle-steps/s, sweeps {fix['sweeps_ms']}")
    fp64 = None
    if not args.no_fp64:
        fp64 = time_gpu(pb, G.FP64, args.steps, args.warmup, args.profile_steps)
        log(f"fp64: {fp64['ms_per_step']:.4f} ms/step, {fp64['value']:.4e} particle-steps/s")

    blast3d_leg = None if args.no_blast3d else blast3d(args)

    # the grid-colouring P2G (atomic-free, bit-reproducible FP64) beside the
    # LDS-tile FP64 path on the same workload and span
    colouring = None
    if args.colouring:
        col = time_gpu(pb, G.FP64_COLOR, args.steps, args.warmup, args.profile_steps)
        colouring = {"value": round(col["value"], 1), "ms_per_step": round(col["ms_per_step"], 5),
                     "sweeps_ms": col["sweeps_ms"],
                     "lds_tile_fp64": None if fp64 is None else {"value": round(fp64["value"], 1),
                                                                "ms_per_step": round(fp64["ms_per_step"], 5),
                                                                "sweeps_ms": fp64["sweeps_ms"]}}
        log(f"fp64 colouring: {col['ms_per_step']:.4f} ms/step, {col['value']:.4e} particle-steps/s, "
            f"sweeps {col['sweeps_ms']}")

    # the other two FP32-state modes (FP64 and FP32 accumulators) on the same
    # workload and span, for the precision ablation
    modes = None
    if args.all_precisions:
        modes = {"fp32_fix64": round(fix["value"], 1), "fp64": None if fp64 is None else round(fp64["value"], 1)}
        for name, prec in (("fp32_acc_f64", G.FP32_ACC_F64), ("fp32_acc_f32", G.FP32_ACC_F32)):
            r = time_gpu(pb, prec, args.steps, args.warmup, 0)
            modes[name] = round(r["value"], 1)
        log(f"precision modes: {modes}")

    hostinc = host_inclusive(pb, G.FP32_FIX64, args.steps)
    log(f"host-inclusive: {hostinc}")

    nnodes = fix["nodes"]
    ntiles = ((pb.n[0] + 15) // 16) * ((pb.n[1] + 15) // 16)
    ncells = ntiles * 256
    bytes_fix = sweep_bytes(pb, nnodes, ncells, 4, 8)
    bytes_scope = survey_bytes(2, N, nnodes)
    sw = fix["sweeps_ms"]
    # Event cost per sweep slot.  The profiled run (an event pair around each
    # sweep slot) covers the same span as the graph-replayed timed steps, so
    # the sum of its event pairs minus the timed step is the events' cost;
    # spread over the slots that hold a kernel, it is taken off each sweep.
    # The tile-scan slot holds no kernel at this size (at most 4096 tiles):
    # its pair is pure event cost and is left out of both sums.  (It measures
    # more than the per-slot figure: around a kernel part of the event cost
    # overlaps the kernel.)
    empty = sw.get("tilescan", 0.0) if (sw and ntiles <= 4096) else 0.0
    kernel_slots = [k for k in sw if k != "tilescan" or ntiles > 4096] if sw else []
    overhead = ((sum(sw[k] for k in kernel_slots) - fix["ms_per_step"]) / len(kernel_slots)
                if kernel_slots else 0.0)
    overhead = max(overhead, 0.0)
    dominant = max(sw, key=sw.get) if sw else "update"
    dom_ms = sw.get(dominant, float("nan")) - overhead
    # achieved = the scope's algorithmic bytes of the dominant sweep per
    # launch / its kernel time; the implementation's own count beside it
    achieved = bytes_scope.get(dominant, bytes_fix[dominant]) / (dom_ms * 1e-3) / 1e9
    achieved_impl = bytes_fix[dominant] / (dom_ms * 1e-3) / 1e9
    sweeps_roofline = {}
    for k in ("p2g", "g2p_p2g", "cellscan", "update"):
        if k in sw and bytes_fix[k] > 0:
            kms = sw[k] - overhead
            b = bytes_scope.get(k, bytes_fix[k])
            gbps = b / (kms * 1e-3) / 1e9
            sweeps_roofline[k] = {"kernel_ms": round(kms, 5), "algorithmic_MB": round(b / 1e6, 2),
                                  "GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
                                  "impl_MB": round(bytes_fix[k] / 1e6, 2)}
    src_hash = kernel_source_hash()
    counters = measured_counters(dominant, pb.name, src_hash)
    traffic = counters.get("bytes_per_launch")
    # VALU issue: one wave64 VALU instruction takes 4 cycles of a SIMD;
    # 256 CUs x 4 SIMDs at 2.4 GHz
    valu = counters.get("sq_insts_valu")
    valu_frac = round(valu * 4 / (1024 * 2.4e9 * dom_ms * 1e-3), 3) if valu else None
    step_bytes = sum(bytes_fix.values())
    step_scope = sum(bytes_scope.values())
    # self-check: the timed step against the sum of the sweeps' event pairs,
    # each less the empty slot's event cost (above 1 by the launch gaps of a
    # replay and by the part of that cost that overlaps a kernel)
    sweep_sum = sum(sw[k] - empty for k in kernel_slots) if sw else None
    copy_gbps = copy_bandwidth()
    log(f"device copy: {copy_gbps} GB/s")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": dominant, "kernel_ms": round(dom_ms, 5),
                "algorithmic_bytes_per_launch": int(bytes_scope.get(dominant, bytes_fix[dominant])),
                "impl_bytes_per_launch": int(bytes_fix[dominant]),
                "frac_impl_bytes": round(achieved_impl / HBM_PEAK_GBPS, 4),
                "event_overhead_ms": round(overhead, 5),
                "empty_slot_ms": round(empty, 5),
                "measured_copy_GBps": copy_gbps,
                "valu_issue_frac": valu_frac,
                "step_algorithmic_bytes": int(step_scope),
                "step_achieved_GBps": round(step_scope / (fix["ms_per_step"] * 1e-3) / 1e9, 1),
                "step_impl_bytes": int(step_bytes),
                "step_ms_over_sweep_sum": round(fix["ms_per_step"] / sweep_sum, 4) if sweep_sum else None}

    cpu = None
    accuracy = None
    if not args.no_cpu and args.cpu_steps > 0:
        # The oracle on a bounded sample of the same problem: its first
        # --cpu-steps steps, once on one host thread (the reference order) and
        # once on every host core (OpenMP; per-thread P2G sums added in
        # thread order).
        from oracle import oracle as O
        O.build(force=False)
        ncpu = os.cpu_count() or 1
        legs = {}
        rho_o = None
        for threads in sorted({1, ncpu}):
            t0 = time.perf_counter()
            o = O.Oracle(pb, threads=threads)
            t1 = time.perf_counter()
            o.step(args.cpu_steps)
            t2 = time.perf_counter()
            legs[threads] = {"value": round(N * args.cpu_steps / (t2 - t1), 1), "seconds": round(t2 - t1, 2),
                             "setup_s": round(t1 - t0, 2)}
            if threads == 1:
                rho_o = o.particles(O.F_RHO)
            o.close()
            log(f"cpu oracle, {threads} thread(s): {legs[threads]['value']:.3e} particle-steps/s over {t2 - t1:.1f} s")
        best = max(legs, key=lambda k: legs[k]["value"])
        cpu = {"value": legs[best]["value"], "unit": "particle-steps/s", "cores": best, "kind": "oracle",
               "host_cpus": ncpu, "single_thread": legs[1]["value"],
               "threads": {str(k): v for k, v in legs.items()},
               "sample": f"first {args.cpu_steps} steps of the same {pb.name} problem "
                         f"({N} particles), FP64 C oracle on {best} host thread(s) (OpenMP; one-thread "
                         f"figure beside it); setup excluded"}
        l1 = lambda r: float(np.abs(r - rho_o).sum() / np.abs(rho_o).sum())
        accuracy = {"steps": args.cpu_steps,
                    "rel_l1_density_fp32_fix64": l1(run_sample_gpu(pb, G.FP32_FIX64, args.cpu_steps))}
        if not args.no_fp64:
            accuracy["rel_l1_density_fp64"] = l1(run_sample_gpu(pb, G.FP64, args.cpu_steps))

    serving = None
    if args.serve_requests > 0:
        from paper_2404_17057_amd import serving as S
        specs = W.request_stream(n=args.serve_requests, rate=200.0, seed=2404)
        cache = W.LatticeCache()
        prog = lambda k: log(f"serving: {k} requests done")
        srv = S.Server(S.GPUBackend(G.FP32_FIX64), lambda sp: W.build_request(sp, cache),
                       hbm_budget=64 << 30, max_slots=64, steps_per_launch=16, progress=prog)
        done = srv.run(specs)
        serving = S.summarize(done)
        serving.update({"stream": f"{args.serve_requests} requests, Poisson 200/s, seed 2404",
                        "precision": "fp32 state, int64 fixed-point P2G", "max_slots": 64,
                        "steps_per_launch": 16, "max_batch": max(srv.batch_sizes),
                        "mean_batch": round(float(np.mean(srv.batch_sizes)), 2),
                        "batched_launches": len(srv.batch_sizes),
                        "admissions_during_a_batch": srv.overlapped_admissions,
                        "failed": [dict(req_id=d.req_id, status=d.status, family=specs[d.req_id].family,
                                        nx=specs[d.req_id].nx, ny=specs[d.req_id].ny, steps=d.steps,
                                        seed=specs[d.req_id].seed, mach=specs[d.req_id].mach)
                                   for d in done if d.status != 0]})
        log(f"serving: {serving}")
        if not args.no_serve_sustained:
            # The same request mix at a rate the device sustains: 70 % of the
            # throughput just measured, divided by the mean work per request.
            mean_work = float(np.mean([d.particles * d.steps for d in done]))
            rate = 0.7 * serving["aggregate_particle_steps_per_s"] / mean_work
            specs = W.request_stream(n=args.serve_sustained_requests, rate=rate, seed=2404)
            srv = S.Server(S.GPUBackend(G.FP32_FIX64), lambda sp: W.build_request(sp, cache),
                           hbm_budget=64 << 30, max_slots=64, steps_per_launch=16, progress=prog)
            sus = S.summarize(srv.run(specs))
            sus.update({"stream": f"{args.serve_sustained_requests} requests, Poisson {rate:.2f}/s, seed 2404",
                        "max_batch": max(srv.batch_sizes),
                        "mean_batch": round(float(np.mean(srv.batch_sizes)), 2),
                        "offered_utilisation": 0.7,
                        "offered_particle_steps_per_s": rate * mean_work})
            serving["sustained"] = sus
            log(f"serving at a sustainable rate: {sus}")

    line = {
        "metric": METRIC,
        "value": round(fix["value"], 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fix["ms_per_step"], 5),
        "graph_setup_ms": fix["graph_setup_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cylinder_mach3_{pb.n[0]}x{pb.n[1]}_ppc4", "particles": N,
                   "precision": "fp32 state, int64 fixed-point P2G", "shape": "quadratic B-spline",
                   "cfl": 0.3, "steps_run": fix["step"], "t_reached": round(fix["t"], 6)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": None if fp64 is None else {"value": round(fp64["value"], 1),
                                          "ms_per_step": round(fp64["ms_per_step"], 5),
                                          "graph_setup_ms": fp64["graph_setup_ms"],
                                          "sweeps_ms": fp64["sweeps_ms"]},
        "sweeps_ms": sw,
        "sweeps_roofline": sweeps_roofline,
        "accuracy_vs_oracle": accuracy,
        "serving": serving,
        "host_inclusive": hostinc,
        "precision_modes": modes,
        "blast3d": blast3d_leg,
        "colouring": colouring,
        "aerofoil": aerofoil(args) if args.aerofoil else None,
        "kernel_source_hash": src_hash,
    }
    if args.calibrate_copy:
        # 256 MiB read + 256 MiB written per copy: the reference dispatch that
        # scales FETCH_SIZE / WRITE_SIZE readings to bytes.
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 256 << 20
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
