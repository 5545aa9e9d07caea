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


def copy_rate_gbs(bytes_moved, reps=10):
    """Rate of a device-to-device copy through torch (Tensor.copy_) that
    moves `bytes_moved` bytes (half read, half written), timed with HIP
    events: what plain streaming reaches on this GPU at the particle
    kernel's size (context for the roofline, not a bound)."""
    import torch
    n = max(1, int(bytes_moved // 2) // 4)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


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


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _time_oracle(O, prob, br, bz, sig, parts, budget_s, max_steps):
    """Whole oracle steps (push, walls, MCC, deposit, field solve, circuit)
    until about budget_s seconds have been spent; init is not timed."""
    o = O.Oracle(prob, br, bz, sig, parts, capacity=(parts[0].n + 4096, parts[1].n + 4096))
    t0 = time.perf_counter()
    o.init()
    t_init = time.perf_counter() - t0
    steps, work, spent = 0, 0, 0.0
    while steps < max_steps and spent < budget_s:
        n = o.count(0) + o.count(1)
        t0 = time.perf_counter()
        o.step()
        spent += time.perf_counter() - t0
        work += n
        steps += 1
    del o
    return {"value": work / spent, "steps": steps, "seconds": spent, "init_seconds": t_init,
            "particle_steps": work}


def cpu_baseline(prob, br, bz, sig, parts, budget_s=12.0, max_steps=64):
    """The FP64 oracle as it stands, timed on this host's cores over whole
    steps of the same workload: once with its serial build and once with its
    OpenMP build (particle loops and deposit on every thread the process may
    use, per-thread tallies combined in a fixed order).  The reported value
    is the multi-core one."""
    from oracle import oracle as O
    O.use_openmp(False)
    serial = _time_oracle(O, prob, br, bz, sig, parts, budget_s, max_steps)
    log(f"[bench] cpu serial: {serial['value']:.3e} particle-steps/s over {serial['steps']} steps")
    O.use_openmp(True)
    threads = O.thread_count()
    par = _time_oracle(O, prob, br, bz, sig, parts, budget_s, max_steps)
    O.use_openmp(False)
    n = parts[0].n + parts[1].n
    return {"value": par["value"], "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{par['steps']} whole steps of {prob.name} from its initial load "
                      f"({n} particles, FP64, {threads} OpenMP threads; init excluded); "
                      f"serial build: {serial['steps']} steps on 1 thread",
            "seconds": par["seconds"], "serial": serial, "openmp": par, **cpu_info()}


def poisson_bench(train_seconds=60.0, reps=6, n_snap=1024, train_steps=3000):
    """Field solve on the 512 x 1024 R-Z operator to an FP64-checked 1e-8
    relative residual: multigrid-preconditioned CG against flexible CG with
    the learned preconditioner, on held-out charge snapshots of a discharge
    at that grid, cold (phi = 0) and warm (previous snapshot's solution).

    The network is trained first, on the GPU, on pairs the simulation makes:
    n_snap (Q, phi0) snapshots of the same discharge and their negatives, and
    192 random potentials with Q = K phi (see pc_train): 2240 pairs by
    default, 20192 with n_snap = 10000 (--pc-snapshots).  The
    learned preconditioner's first approximation is the multigrid V-cycle
    (pc_pre = 1), which the network corrects."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import pc_train
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    # (capacity 4x the load: a long snapshot collection lets the discharge grow)
    p = W.preset("ec512x1024_f32").replace(n_per_species=2_000_000, poisson_rtol=1e-8,
                                           poisson_maxit=500, pc_batch=8, capacity_factor=4.0)
    br, bz, sig, parts = W.inputs(p)
    sim = Simulation(p, br, bz, sig, parts)
    sim.step(50)
    log(f"[bench] poisson: collecting {n_snap + 8} charge snapshots")
    # one buffer per side for the snapshots, their negatives and the random
    # potentials, filled in place (at 2e4 pairs each side holds ~85 GB)
    nf = 192
    Q = torch.empty((2 * n_snap + nf, p.nodes), dtype=torch.float64, device="cuda")
    P = torch.empty_like(Q)
    pc_train.snapshot_pairs(sim, n_snap + 8, every=2, out=(Q, P))
    held_q = Q[n_snap:n_snap + 8].clone()
    torch.neg(Q[:n_snap], out=Q[n_snap:2 * n_snap])
    torch.neg(P[:n_snap], out=P[n_snap:2 * n_snap])
    Qf, Pf = pc_train.field_pairs(sim, nf, seed=250710731)
    Q[2 * n_snap:].copy_(Qf)
    P[2 * n_snap:].copy_(Pf)
    del Qf, Pf
    log(f"[bench] poisson: training on {Q.shape[0]} pairs for <= {train_seconds:.0f} s")
    tr = pc_train.train(sim, Q, P, steps=train_steps, batch=8, lr=1e-3, seed=1,
                        time_limit=train_seconds,
                        report=lambda k, loss: log(f"[bench] poisson: step {k}, loss {loss:.4f}"))
    log(f"[bench] poisson: {tr['steps']} steps, loss {tr['loss_first']:.3f} -> "
        f"{tr['loss_last']:.4f}, {tr['ms_per_step']:.1f} ms/step")
    del Q, P
    torch.cuda.empty_cache()
    out = {"grid": "512x1024", "rtol": 1e-8, "rhs": "held-out charge snapshots",
           "pairs": 2 * n_snap + nf, "first_step": "multigrid V-cycle",
           "training": tr}
    for name, mode in (("mg_cg", W.POISSON_MGCG), ("learned_fcg", W.POISSON_LEARNED)):
        sim.set_poisson_mode(mode)
        res = {}
        for start in ("cold", "warm"):
            times, its, fb = [], [], 0
            phi = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
            for k in range(reps + 1):
                q = held_q[k % held_q.shape[0]].contiguous()
                if start == "cold":
                    phi.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = sim.poisson(q, 0.0, phi)
                torch.cuda.synchronize()
                if k == 0:
                    continue          # the first solve sets the iteration prediction
                times.append((time.perf_counter() - t0) * 1e3)
                its.append(st["iterations"])
                fb += st["fell_back"]
            res[start] = {"ms": float(np.median(times)), "iterations": int(np.median(its)),
                          "fell_back": fb, "solves": reps}
        out[name] = res
        log(f"[bench] poisson {name}: {res}")
    sim.close()
    return out


def gather_forms_bench(workload, steps=100, warmup=20, box_steps=20000, box_every=200):
    """Both gather forms of the paper (Section 2).  Throughput: the bench
    workload's full step with each form (EC-PIC is the headline value, MC-PIC
    the same discharge with the nodal-field gather).  Energy: the closed
    thermal box (workloads.thermal_box) at the workload's grid, cell and
    particle count, where the cell is three Debye lengths: EC-PIC's total
    energy stays bounded, MC-PIC heats (finite-grid instability)."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    base = W.preset(workload)
    out = {}
    for name, scheme in (("ec", W.EC_PIC), ("mc", W.MC_PIC)):
        p = base.replace(scheme=scheme)
        br, bz, sig, parts = W.inputs(p)
        sim = Simulation(p, br, bz, sig, parts)
        sim.step(warmup)
        d0 = sim.diag()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d1 = sim.diag()
        sim.close()
        del sim, parts
        n = 0.5 * (sum(d0["count"]) + sum(d1["count"]))
        res = {"particle_steps_per_s": n * steps / wall, "ms_per_step": wall / steps * 1e3}
        ppc = max(1, base.n_per_species // (base.nr * base.nz))
        bp, bparts = W.thermal_box(base.nr, base.nz, base.dr, ppc, scheme, base.precision)
        bbr, bbz = W.magnetron_field(bp)
        sim = Simulation(bp, bbr, bbz, W.cross_sections(bp.e_exc, bp.e_iz), bparts)
        ke, tot = [], []
        for _ in range(box_steps // box_every):
            sim.step(box_every)
            d = sim.diag()
            ke.append(d["ke"][0])
            tot.append(d["ke"][0] + d["w_field"])
        sim.close()
        del sim, bparts
        ke, tot = np.array(ke), np.array(tot)
        m = max(1, len(ke) // 20)
        res["box"] = {"grid": f"{bp.nr}x{bp.nz}", "particles_per_species": bp.n_per_species,
                      "density_m3": bp.density, "dt_s": bp.dt, "steps": box_steps,
                      "total_energy_drift_max": float(np.abs(tot - tot[0]).max() / tot[0]),
                      "electron_ke_growth": float(ke[-m:].mean() / ke[:m].mean() - 1.0)}
        out[name] = res
        torch.cuda.empty_cache()
        log(f"[bench] gather form {name}: {res}")
    return out


def throughput(p, steps=20, warmup=5):
    """Whole steps of one discharge: particle-steps/s, ms per step, and the
    fused particle kernel's average time (HIP events on the library's
    stream) and algorithmic HBM rate; deposit windows that fell back to
    global atomics in the last step."""
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    br, bz, sig, parts = W.inputs(p)
    sim = Simulation(p, br, bz, sig, parts, timers=False)
    del parts
    sim.step(warmup)
    d0 = sim.diag()
    sim.lib.pic_enable_timers(sim.h, 2)
    sim.timers(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = sim.timers(reset=True)
    d1 = sim.diag()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    ne = 0.5 * (d0["count"][0] + d1["count"][0])
    ni = 0.5 * (d0["count"][1] + d1["count"][1])
    dtype = "f32" if p.precision == W.F32 else "f64"
    push_ms = tm["push_ms"] / max(tm["push_launches"], 1)
    algo = ALGO_BYTES[dtype]["e"] * ne + ALGO_BYTES[dtype]["i"] * ni
    gbs = algo / (push_ms * 1e-3) / 1e9
    return {"workload": p.name, "scheme": "EC-PIC" if p.scheme == W.EC_PIC else "MC-PIC",
            "particle_steps_per_s": (ne + ni) * steps / wall, "ms_per_step": wall / steps * 1e3,
            "steps": steps, "push_avg_ms": push_ms, "push_gbs_algorithmic": gbs,
            "push_frac": gbs / HBM_PEAK_GBS, "deposit_fallback_last_step": d1["deposit_fallback"],
            "count": d1["count"]}


def high_density_bench(steps=20, warmup=5, box_steps=2000, box_every=40):
    """The high-density discharge (512 x 1024 cells, 5e7 + 5e7, n = 1e17):
    both gather forms and the clustered load (half of each species in the
    ring 0.35 R < r < 0.5 R, z < 0.1 L, about 3e3 particles per species per
    cell there).  Then the closed thermal box at this discharge's grid, cell
    (2.9 Debye lengths) and particle count with each gather form: EC-PIC's
    total energy stays bounded, MC-PIC's electrons heat (Section 5)."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    out = {}
    for name in ("ec512x1024_f32", "mc512x1024_f32", "ec512x1024_clustered_f32"):
        r = throughput(W.preset(name), steps, warmup)
        log(f"[bench] {name}: {r}")
        out[name] = r
    base = W.preset("ec512x1024_f32")
    ppc = max(1, base.n_per_species // (base.nr * base.nz))
    box = {}
    for form, scheme in (("ec", W.EC_PIC), ("mc", W.MC_PIC)):
        bp, bparts = W.thermal_box(base.nr, base.nz, base.dr, ppc, scheme, base.precision)
        bbr, bbz = W.magnetron_field(bp)
        sim = Simulation(bp, bbr, bbz, W.cross_sections(bp.e_exc, bp.e_iz), bparts)
        del bparts
        ke, tot = [], []
        for _ in range(box_steps // box_every):
            sim.step(box_every)
            d = sim.diag()
            ke.append(d["ke"][0])
            tot.append(d["ke"][0] + d["w_field"])
        sim.close()
        del sim
        torch.cuda.empty_cache()
        ke, tot = np.array(ke), np.array(tot)
        m = max(1, len(ke) // 20)
        box[form] = {"grid": f"{bp.nr}x{bp.nz}", "particles_per_species": bp.n_per_species,
                     "density_m3": bp.density, "dt_s": bp.dt, "steps": box_steps,
                     "total_energy_drift_max": float(np.abs(tot - tot[0]).max() / tot[0]),
                     "electron_ke_growth": float(ke[-m:].mean() / ke[:m].mean() - 1.0)}
        log(f"[bench] high-density box {form}: {box[form]}")
    out["thermal_box"] = box
    return out


def high_density_sweep(steps=2000, every=500):
    """The high-density discharge (512 x 1024 cells, 5e7 + 5e7, n = 1e17,
    20 mTorr) at each ion-induced yield 0.1, 0.2, 0.3 and series resistance
    10, 100 ohm, with each gather form: `steps` steps (10 ns) from the same
    seeded load, the FP64 diagnostics every `every` steps (cathode voltage
    and current, total energy = kinetic + field, collisions, emission)."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation
    base = W.preset("ec512x1024_f32")
    br, bz, sig, parts = W.inputs(base)
    runs = []
    for form, scheme in (("ec", W.EC_PIC), ("mc", W.MC_PIC)):
        for gamma in (0.1, 0.2, 0.3):
            for r_ohm in (10.0, 100.0):
                p = base.replace(scheme=scheme, gamma_i=gamma, r_ext=r_ohm)
                sim = Simulation(p, br, bz, sig, parts, timers=False)
                d = sim.diag()
                e0 = d["ke"][0] + d["ke"][1] + d["w_field"]
                hist = []
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps // every):
                    sim.step(every)
                    d = sim.diag()
                    hist.append({"step": d["step"], "vc": d["vc"], "i_cathode": d["i_cathode"],
                                 "energy_j": d["ke"][0] + d["ke"][1] + d["w_field"]})
                wall = time.perf_counter() - t0
                sim.close()
                del sim
                torch.cuda.empty_cache()
                r = {"form": form, "gamma_i": gamma, "r_ohm": r_ohm, "steps": steps,
                     "ms_per_step_with_diag": wall / steps * 1e3,
                     "vc": d["vc"], "i_cathode_a": d["i_cathode"],
                     "i_cathode_mean_a": float(np.mean([h["i_cathode"] for h in hist])),
                     "energy_change": (hist[-1]["energy_j"] - e0) / e0,
                     "n_coll": list(d["n_coll"]), "n_see": d["n_see"], "count": list(d["count"]),
                     "phi_max": d["phi_max"], "n_peak": list(d["n_peak"]), "history": hist}
                log(f"[bench] sweep {form} gamma {gamma} R {r_ohm}: vc {r['vc']:.2f} V, "
                    f"I {r['i_cathode_mean_a']:.4g} A, dE/E {r['energy_change']:+.3e}")
                runs.append(r)
    return {"grid": f"{base.nr}x{base.nz}", "particles_per_species": base.n_per_species,
            "density_m3": base.density, "dt_s": base.dt, "runs": runs}


def table1_bench(steps=200_000, chunk=2000):
    """Table 1's trends on the 3 x 3 cm geometry of Section 3: ion yield 0.1
    or 0.2 and R = 3000 or 1000 ohm (electron yield 0.1, -300 V), the four
    runs advanced together as one ensemble.  Reports per run the cathode
    voltage and the external-circuit current (V_ext - V_c) / R averaged over
    the last quarter of the steps, and the particle counts."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Ensemble, Simulation
    probs = W.table1_problems(steps)
    sims = []
    for p in probs:
        br, bz, sig, parts = W.inputs(p)
        sims.append(Simulation(p, br, bz, sig, parts))
    ens = Ensemble(sims)
    hist = [[] for _ in probs]
    t0 = time.perf_counter()
    for k in range(steps // chunk):
        ens.step(chunk)
        for r, s in enumerate(sims):
            d = s.diag()
            hist[r].append((d["vc"], d["i_cathode"], d["count"][0], d["count"][1]))
        if (k + 1) % 10 == 0:
            log(f"[bench] table1 step {(k + 1) * chunk}: vc "
                + " ".join(f"{h[-1][0]:.1f}" for h in hist)
                + " counts " + " ".join(f"{h[-1][2]}" for h in hist))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"steps": steps, "dt_s": probs[0].dt, "wall_s": wall, "runs": []}
    for p, h in zip(probs, hist):
        a = np.array(h)
        q = a[len(a) * 3 // 4:]
        vc = float(q[:, 0].mean())
        out["runs"].append({"gamma_i": p.gamma_i, "r_ohm": p.r_ext, "vc_v": vc,
                            "i_circuit_a": (p.v_ext - vc) / p.r_ext,
                            "i_cathode_sampled_a": float(q[:, 1].mean()),
                            "electrons": int(q[-1, 2]), "ions": int(q[-1, 3])})
    ens.close()
    for s in sims:
        s.close()
    return out


def ensemble_bench(n_runs=64, steps=10, scale=1.0):
    """The yield / resistance sweep (workloads.ensemble_problems): the runs
    advanced one after another through pic_step, then the same runs advanced
    together as one ensemble (one captured graph per step), aggregate
    particle-steps/s for each.  Launch shapes come from the autotuner (one
    tuning per run size, cached), the stream count from timing 2..16."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import autotune
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Ensemble, Simulation
    ps = W.ensemble_problems(n_runs=n_runs, scale=scale)
    t0 = time.perf_counter()
    sims = []
    for p in ps:
        br, bz, sig, parts = W.inputs(p)
        sims.append(Simulation(p, br, bz, sig, parts))
    torch.cuda.synchronize()
    log(f"[bench] ensemble: {n_runs} runs initialised in {time.perf_counter() - t0:.1f} s")
    cache = autotune.TuningCache()
    tuned = 0
    for sim in sims:
        _, now = cache.apply_or_tune(sim, steps_per_trial=2)
        tuned += int(now)
    log(f"[bench] ensemble: {tuned} sizes tuned: {cache.table}")

    def live():
        return [sim.diag()["count"] for sim in sims]

    # one after another
    c0 = live()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    c1 = live()
    ps_seq = sum(0.5 * (a[0] + a[1] + b[0] + b[1]) for a, b in zip(c0, c1)) * steps
    # together
    ens = Ensemble(sims, nstreams=1)
    ens.step(1)
    c0 = live()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(steps)
    torch.cuda.synchronize()
    t_ens = time.perf_counter() - t0
    c1 = live()
    ps_ens = sum(0.5 * (a[0] + a[1] + b[0] + b[1]) for a, b in zip(c0, c1)) * steps
    ens.close()
    runs = []
    for p, sim in zip(ps, sims):
        d = sim.diag()
        runs.append({"grid": p.nr, "gamma": p.gamma_i, "r_ohm": p.r_ext,
                     "particles": d["count"][0] + d["count"][1], "step": d["step"],
                     "i_cathode_a": d["i_cathode"], "v_cathode": d["vc"],
                     "n_e_peak_m3": d["n_peak"][0], "n_i_peak_m3": d["n_peak"][1]})
        sim.close()
    seq = ps_seq / t_seq
    bat = ps_ens / t_ens
    log(f"[bench] ensemble: sequential {seq:.3e}, batched {bat:.3e} particle-steps/s "
        f"({bat / seq:.2f}x)")
    return {"runs": n_runs, "steps": steps, "total_particles": int(sum(r["particles"] for r in runs)),
            "sequential_particle_steps_per_s": seq, "batched_particle_steps_per_s": bat,
            "speedup": bat / seq, "sequential_ms_per_step": t_seq / steps * 1e3,
            "batched_ms_per_step": t_ens / steps * 1e3, "tuning": cache.table,
            "note": "per-run values after the measured steps (a few tens of ps of a discharge "
                    "that needs ~4 us to reach steady state)",
            "per_run": runs}


def ensemble_long(n_runs=64, steps=200_000, every=2000):
    """The yield / resistance sweep advanced as one ensemble for `steps`
    steps (2e5 steps of 5 ps: 1 us), each run's cathode current, voltage and
    peak densities sampled every `every` steps; per run, the means and
    spread of current and voltage over the last quarter of the samples.
    Capacity 2x the initial load per species, for a discharge that grows."""
    import numpy as np
    import torch
    from paper_2507_10727_amd import autotune
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Ensemble, Simulation
    ps = [p.replace(capacity_factor=2.0) for p in W.ensemble_problems(n_runs=n_runs)]
    sims = []
    for p in ps:
        br, bz, sig, parts = W.inputs(p)
        sims.append(Simulation(p, br, bz, sig, parts))
    cache = autotune.TuningCache()
    for sim in sims:
        cache.apply_or_tune(sim, steps_per_trial=2)
    log(f"[bench] ensemble-long: {n_runs} runs initialised and tuned")
    ens = Ensemble(sims, nstreams=1)
    samples = [[] for _ in sims]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        ens.step(k)
        done += k
        tot = 0
        for j, sim in enumerate(sims):
            d = sim.diag()
            samples[j].append((d["step"], d["i_cathode"], d["vc"], d["n_peak"][0], d["n_peak"][1],
                               d["count"][0] + d["count"][1]))
            tot += d["count"][0] + d["count"][1]
        log(f"[bench] ensemble-long: {done} steps, {tot} particles, "
            f"{(time.perf_counter() - t0):.1f} s")
    wall = time.perf_counter() - t0
    ens.close()
    runs = []
    for p, sim, sm in zip(ps, sims, samples):
        a = np.array(sm, dtype=np.float64)
        tail = a[-max(1, len(a) // 4):]
        runs.append({"grid": p.nr, "gamma": p.gamma_i, "r_ohm": p.r_ext,
                     "density_m3": p.density, "particles_start": p.n_per_species * 2,
                     "particles_end": int(a[-1, 5]), "step": int(a[-1, 0]),
                     "i_cathode_mean_a": float(tail[:, 1].mean()),
                     "i_cathode_std_a": float(tail[:, 1].std()),
                     "v_cathode_mean": float(tail[:, 2].mean()),
                     "v_cathode_std": float(tail[:, 2].std()),
                     "n_e_peak_m3": float(a[-1, 3]), "n_i_peak_m3": float(a[-1, 4])})
        sim.close()
    return {"runs": n_runs, "steps": steps, "sample_every": every,
            "ms_per_step_with_sampling": wall / steps * 1e3, "per_run": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ec256x512_f32")
    ap.add_argument("--solver", choices=("direct", "mgcg"), default="direct",
                    help="field solve of the timed steps: the direct sine-transform solve "
                         "(default) or multigrid-preconditioned CG")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-poisson", action="store_true")
    ap.add_argument("--poisson-only", action="store_true",
                    help="only the field-solve comparison (prints its JSON)")
    ap.add_argument("--train-seconds", type=float, default=60.0)
    ap.add_argument("--train-steps", type=int, default=3000,
                    help="most Adam steps of the network training (the time limit may stop it first)")
    ap.add_argument("--pc-snapshots", type=int, default=1024,
                    help="charge snapshots of the training set (with their negatives and 192 "
                         "random potentials: 2 N + 192 pairs)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the EC-PIC / MC-PIC throughput and energy comparison")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the batched sweep of 64 runs")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the batched sweep against sequential runs (prints its JSON)")
    ap.add_argument("--ensemble-runs", type=int, default=64)
    ap.add_argument("--table1-only", type=int, default=0, metavar="STEPS",
                    help="only the Table 1 trend runs on the 3 x 3 cm geometry, STEPS steps "
                         "(prints their JSON)")
    ap.add_argument("--no-high-density", action="store_true",
                    help="skip the 512 x 1024 discharges (uniform EC/MC and clustered)")
    ap.add_argument("--high-density-only", action="store_true",
                    help="only the 512 x 1024 discharges (prints their JSON)")
    ap.add_argument("--ensemble-long", type=int, default=0, metavar="STEPS",
                    help="only the 64-run sweep as one ensemble for STEPS steps with per-run "
                         "current / voltage sampling (prints its JSON)")
    ap.add_argument("--hd-sweep-only", action="store_true",
                    help="only the 512 x 1024 discharge at ion yields 0.1/0.2/0.3 and "
                         "10/100 ohm with each gather form, 2000 steps each (prints its JSON)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_10727_amd import workloads as W
    from paper_2507_10727_amd.sim import Simulation

    if args.poisson_only:
        print(json.dumps({"poisson": poisson_bench(args.train_seconds, n_snap=args.pc_snapshots,
                                                   train_steps=args.train_steps)}), flush=True)
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble": ensemble_bench(args.ensemble_runs)}), flush=True)
        return
    if args.table1_only:
        print(json.dumps({"table1": table1_bench(args.table1_only)}), flush=True)
        return
    if args.high_density_only:
        print(json.dumps({"high_density": high_density_bench()}), flush=True)
        return
    if args.hd_sweep_only:
        print(json.dumps({"high_density_sweep": high_density_sweep()}), flush=True)
        return
    if args.ensemble_long:
        print(json.dumps({"ensemble_long": ensemble_long(steps=args.ensemble_long)}), flush=True)
        return

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

    p = W.preset(args.workload).replace(
        poisson_mode=W.POISSON_DIRECT if args.solver == "direct" else W.POISSON_MGCG)
    log(f"[bench] generating {args.workload}: {p.nr}x{p.nz} cells, {p.n_per_species} per species")
    br, bz, sig, parts = W.inputs(p)
    log("[bench] init on GPU")
    t0 = time.perf_counter()
    sim = Simulation(p, br, bz, sig, parts, timers=False)
    torch.cuda.synchronize()
    log(f"[bench] init {time.perf_counter() - t0:.1f} s; warmup {args.warmup} steps")
    sim.step(args.warmup)
    d0 = sim.diag()
    # the timed steps time the particle kernel alone (two HIP events a step)
    sim.lib.pic_enable_timers(sim.h, 2)
    sim.timers(reset=True)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = sim.timers(reset=True)
    d1 = sim.diag()
    # phase breakdown from further steps with every phase timed (the events
    # around each phase cost time of their own, so they stay out of the
    # timed steps); one cell sort falls in every sort_every steps
    n_ph = max(p.sort_every, 20)
    sim.lib.pic_enable_timers(sim.h, 1)
    sim.step(n_ph)
    tm_all = sim.timers(reset=True)
    sim.lib.pic_enable_timers(sim.h, 0)
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
    copy_gbs = copy_rate_gbs(algo_bytes)
    log(f"[bench] device copy of the same bytes: {copy_gbs:.0f} GB/s")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(args.workload),
            "kernel": "k_push (gather+Boris+walls+SEE+MCC+deposit)",
            "avg_ms": push_avg_ms, "launches": tm["push_launches"],
            "algorithmic_bytes_per_launch": algo_bytes,
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs}
    phases = {k: tm_all[k] / n_ph for k in ("push_ms", "children_ms", "sort_ms", "poisson_ms",
                                            "circuit_ms", "field_ms")}
    phases["steps"] = n_ph
    log(f"[bench] {value:.3e} particle-steps/s, {wall / args.steps * 1e3:.3f} ms/step, "
        f"push {push_avg_ms:.3f} ms ({achieved:.0f} GB/s algorithmic)")
    log(f"[bench] last field solve: {d1['poisson']}")
    sim.close()
    del sim
    torch.cuda.empty_cache()

    poisson = None
    if not args.no_poisson:
        log("[bench] poisson 512x1024")
        poisson = poisson_bench(args.train_seconds)
    forms = None
    if not args.no_forms:
        log("[bench] gather forms (EC-PIC / MC-PIC)")
        forms = gather_forms_bench(args.workload)
    hd = None
    if not args.no_high_density:
        log("[bench] 512 x 1024 discharges")
        hd = high_density_bench()
    ensemble = None
    if not args.no_ensemble:
        log(f"[bench] ensemble of {args.ensemble_runs} runs")
        ensemble = ensemble_bench(args.ensemble_runs)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle: serial build, then OpenMP build)")
        cpu = cpu_baseline(p, br, bz, sig, parts)
        log(f"[bench] cpu {cpu['value']:.3e} particle-steps/s on {cpu['cores']} threads "
            f"in {cpu['seconds']:.1f} s")

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
                   "poisson_rtol": p.poisson_rtol, "sort_every": p.sort_every,
                   "field_solve": args.solver},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phase_ms_per_step": phases,
        "poisson": poisson,
        "gather_forms": forms,
        "high_density": hd,
        "ensemble": ensemble,
        "diag": {"vc": d1["vc"], "i_cathode": d1["i_cathode"], "n_coll": d1["n_coll"],
                 "deposit_fallback": d1["deposit_fallback"], "count": d1["count"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
