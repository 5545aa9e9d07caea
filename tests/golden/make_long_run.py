"""Write tests/golden/long_run_small64.json: long-run statistics of the small
discharge (64 x 64 cells over 2 x 2 cm, MC-PIC, FP64, cathode fixed at
-400 V, 5 mTorr argon, peak B 0.03 T) with 1e5 + 1e5 macroparticles over
20000 steps (100 ns), computed by the oracle alone.

Recorded over the last 25% of the steps (every step for the current, every
10th step for the rest): the mean cathode current, the mean peak electron
and ion densities (node charge summed over blocks of 8 x 8 nodes, divided by
the blocks' volume), the mean peak potential, the mean live particle counts
and the collisions per step.

    python tests/golden/make_long_run.py      (about 10 minutes, one core)
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_2507_10727_amd import workloads as W     # noqa: E402

STEPS = 20000
N_PER_SPECIES = 100_000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_run_small64.json")


def problem():
    return W.scaled(W.preset("small_mc64_f64"), N_PER_SPECIES).replace(steps=STEPS)


def block_peak(q, p, qs):
    """Peak density of charge q (node array) over blocks of 8 x 8 nodes."""
    g = q.reshape(p.nz + 1, p.nr + 1)[:p.nz, :p.nr]
    b = g.reshape(p.nz // 8, 8, p.nr // 8, 8).sum(axis=(1, 3))
    r0 = np.maximum(np.arange(0, p.nr, 8) - 0.5, 0.0) * p.dr
    r1 = (np.arange(0, p.nr, 8) + 7.5) * p.dr
    vol = math.pi * (r1 ** 2 - r0 ** 2) * 8 * p.dz
    return float((b / (qs * vol[None, :])).max())


def stats_window(p):
    return int(0.75 * p.steps), p.steps


def main():
    p = problem()
    br, bz, sig, parts = W.inputs(p)
    o = O.Oracle(p, br, bz, sig, parts, capacity=(4 * N_PER_SPECIES, 4 * N_PER_SPECIES))
    o.init()
    lo, hi = stats_window(p)
    cur, ne, ni, phim, cnt, coll = [], [], [], [], [], []
    t0 = time.time()
    sp = p.species()
    for k in range(1, p.steps + 1):
        d = o.step()
        if k > lo:
            cur.append(d["i_cathode"])
            coll.append(list(d["n_coll"]))
            if k % 10 == 0:
                ne.append(block_peak(o.q[0], p, sp[0][0]))
                ni.append(block_peak(o.q[1], p, sp[1][0]))
                phim.append(d["phi_max"])
                cnt.append([o.count(0), o.count(1)])
        if k % 1000 == 0:
            print(f"step {k}: {time.time() - t0:.0f} s, counts {o.count(0)} {o.count(1)}, "
                  f"I {d['i_cathode']:.3e} A", flush=True)
    out = {
        "source": "tests/golden/make_long_run.py (oracle only)",
        "workload": "small_mc64_f64 scaled to 1e5 + 1e5 particles, 20000 steps",
        "steps": p.steps, "window": [lo, hi], "n_per_species": N_PER_SPECIES,
        "i_cathode_mean_a": float(np.mean(cur)),
        "i_cathode_sem_a": float(np.std(cur) / math.sqrt(len(cur))),
        "n_e_peak_m3": float(np.mean(ne)), "n_i_peak_m3": float(np.mean(ni)),
        "phi_max_v": float(np.mean(phim)),
        "count_e": float(np.mean([c[0] for c in cnt])), "count_i": float(np.mean([c[1] for c in cnt])),
        "collisions_per_step": [float(x) for x in np.mean(np.array(coll), axis=0)],
        "v_cathode_v": p.v_fixed,
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
