"""Launch tuning with a cache: the particle kernel's shape per run size
(pic_autotune, timed on the GPU; the simulation's state is restored after
the trials).

Choices are keyed by what sets the kernels' cost: grid, state precision,
gather scheme and the particle count to within a factor of two.  The cache
is a JSON file when a path is given.
"""
from __future__ import annotations

import json
import math
import os

from . import workloads as W


def key(p: W.Problem, particles: int) -> str:
    prec = "f64" if p.precision == W.F64 else "f32"
    scheme = "ec" if p.scheme == W.EC_PIC else "mc"
    bucket = int(round(math.log2(max(particles, 1))))
    return f"{p.nr}x{p.nz}:{prec}:{scheme}:2^{bucket}"


class TuningCache:
    def __init__(self, path=None):
        self.path = path
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def save(self):
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)

    def apply_or_tune(self, sim, steps_per_trial=2):
        """Apply the cached shape for sim's size, else tune sim (it advances
        by 9 * steps_per_trial steps) and cache the result.  Returns
        (choice, tuned_now)."""
        d = sim.diag()
        k = key(sim.prob, d["count"][0] + d["count"][1])
        if k in self.table:
            t = self.table[k]
            sim.set_tuning(t["push_blocks"], t["push_e_weight"])
            return t, False
        t = sim.autotune(steps_per_trial)
        self.table[k] = {"push_blocks": t["push_blocks"], "push_e_weight": t["push_e_weight"],
                         "push_ms": t["push_ms"]}
        return self.table[k], True
