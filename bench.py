"""Benchmark of the R-Z PIC-MCC timestep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-poisson]

A step is one pass of the whole timestep (field gather, Boris push, walls and
secondary emission, null-collision MCC, new particles, deposit, field solve to
the configured FP64 residual, circuit, gather-field packing, and the cell sort
every sort_every steps) over the synthetic workload; the particle arrays are
resident in HBM before timing starts.  Prints one JSON line.

Value: particle-steps/s = (live electrons + ions) x steps / wall time of the
timed steps.  The roofline object covers the fused particle kernel, timed with
HIP events recorded on the library's stream around each of its launches.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
ALGO_BYTES = {             # per particle and step: read 2 positions + 3
    # velocities (+ the id that keys the random stream), write 5 words
    "f32": {"e": 44, "i": 40},
    "f64": {"e": 84, "i": 80},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile(workload):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"push_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    src = os.path.join(ROOT, "paper_2507_10727_amd", "csrc", "particles.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if t.get("source_sha256") != sha:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(prob, br, bz, sig, parts, max_seconds=40.0):
    """The FP64 oracle as it stands, single thread, one full step of the same
    workload (all particles), on this host."""
    from oracle import oracle as O
    o = O.Oracle(prob, br, bz, sig, parts, capacity=(parts[0].n + 4096, parts[1].n + 4096))
    t0 = time.perf_counter()
    o.init()
    t_init = time.perf_counter() - t0
    n = o.count(0) + o.count(1)
    t0 = time.perf_counter()
    o.step()
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 full step of {prob.name} ({n} particles, FP64, single thread; "
                      f"init excluded, {t_init:.1f} s)",
            "seconds": dt}


def poisson_bench(reps=5):
    """MG-preconditioned CG to an FP64-checked 1e-8 relative residual on the
    512 x 1024 R-Z operator, cold (phi = 0) and warm (previous solution)."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    p = W.preset("ec512x1024_f32").replace(poisson_rtol=1e-8, poisson_maxit=500)
    br, bz = W.magnetron_field(p)
    sig = W.cross_sections()
    sim = Simulation(p, br, bz, sig, None, capacity=(1024, 1024))
    rng = np.random.default_rng(250710730)
    nn = p.nodes
    # a charge snapshot shape: smooth positive bulk plus noise
    r = np.arange(p.nr + 1) * p.dr
    z = np.arange(p.nz + 1) * p.dz
    R, Z = np.meshgrid(r, z)
    base = np.exp(-((R - 0.4 * p.lr) / (0.1 * p.lr)) ** 2 - (Z / (0.1 * p.lz)) ** 2)
    out = {}
    for mode in ("cold", "warm"):
        times, its = [], []
        phi = torch.zeros(nn, dtype=torch.float64, device="cuda")
        for k in range(reps):
            q = (base * 1e-12 * (1 + 0.05 * k) + rng.normal(size=base.shape) * 1e-13).ravel()
            qd = torch.tensor(q, dtype=torch.float64, device="cuda")
            if mode == "cold":
                phi.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.poisson(qd, -500.0, phi)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            its.append(st["iterations"])
        out[mode] = {"ms": float(np.median(times[1:])), "iterations": int(np.median(its[1:])),
                     "rel_res_target": 1e-8}
    sim.close()
    return {"grid": "512x1024", "method": "MG-PCG (FP32 V-cycle, FP64 refinement)", **out,
            "learned_pc": None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ec256x512_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-poisson", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation

    if args.copy_calibration:
        # a plain device-to-device copy of known size: its FETCH_SIZE /
        # WRITE_SIZE per dispatch calibrate the counters against 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log("[bench] copy calibration: 3 x 1 GiB device copies")

    p = W.preset(args.workload)
    log(f"[bench] generating {args.workload}: {p.nr}x{p.nz} cells, {p.n_per_species} per species")
    br, bz, sig, parts = W.inputs(p)
    log("[bench] init on GPU")
    t0 = time.perf_counter()
    sim = Simulation(p, br, bz, sig, parts, timers=False)
    torch.cuda.synchronize()
    log(f"[bench] init {time.perf_counter() - t0:.1f} s; warmup {args.warmup} steps")
    sim.step(args.warmup)
    d0 = sim.diag()
    sim.lib.pic_enable_timers(sim.h, 1)
    sim.timers(reset=True)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = sim.timers(reset=True)
    d1 = sim.diag()
    n0 = d0["count"][0] + d0["count"][1]
    n1 = d1["count"][0] + d1["count"][1]
    nmean = 0.5 * (n0 + n1)
    ne = 0.5 * (d0["count"][0] + d1["count"][0])
    ni = 0.5 * (d0["count"][1] + d1["count"][1])
    value = nmean * args.steps / wall
    dtype = "f32" if p.precision == W.F32 else "f64"
    push_avg_ms = tm["push_ms"] / max(tm["push_launches"], 1)
    algo_bytes = ALGO_BYTES[dtype]["e"] * ne + ALGO_BYTES[dtype]["i"] * ni
    achieved = algo_bytes / (push_avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(args.workload),
            "kernel": "k_push (gather+Boris+walls+SEE+MCC+deposit)",
            "avg_ms": push_avg_ms, "launches": tm["push_launches"],
            "algorithmic_bytes_per_launch": algo_bytes}
    phases = {k: tm[k] / args.steps for k in ("push_ms", "children_ms", "sort_ms", "poisson_ms",
                                              "circuit_ms", "field_ms")}
    log(f"[bench] {value:.3e} particle-steps/s, {wall / args.steps * 1e3:.3f} ms/step, "
        f"push {push_avg_ms:.3f} ms ({achieved:.0f} GB/s algorithmic)")
    sim.close()
    del sim
    torch.cuda.empty_cache()

    poisson = None
    if not args.no_poisson:
        log("[bench] poisson 512x1024")
        poisson = poisson_bench()
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, 1 step)")
        cpu = cpu_baseline(p, br, bz, sig, parts)
        log(f"[bench] cpu {cpu['value']:.3e} particle-steps/s in {cpu['seconds']:.1f} s")

    line = {
        "metric": "particle-steps/s (gather+push+MCC+deposit); Poisson ms learned-PC vs MG-CG @1e-8",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{p.nr}x{p.nz}",
                   "domain_m": [p.lr, p.lz], "particles_per_species": p.n_per_species,
                   "scheme": "EC-PIC" if p.scheme == W.EC_PIC else "MC-PIC",
                   "density_m3": p.density, "pressure_mtorr": p.p_gas / W.TORR * 1e3,
                   "circuit": f"{p.v_ext} V through {p.r_ext} ohm", "dt_s": p.dt,
                   "poisson_rtol": p.poisson_rtol, "sort_every": p.sort_every},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phase_ms_per_step": phases,
        "poisson": poisson,
        "diag": {"vc": d1["vc"], "i_cathode": d1["i_cathode"], "n_coll": d1["n_coll"],
                 "deposit_fallback": d1["deposit_fallback"], "count": d1["count"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
