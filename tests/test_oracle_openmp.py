"""The oracle's multi-core timing build (liborc_omp.so, OpenMP over the
particle loops and the deposit) computes the serial oracle's step: every
particle (positions, velocities, ids, new particles) bit for bit, and the
sums (node charge, energies) to round-off of their different summation
order."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
from oracle import oracle as O
from paper_2507_10727_amd import workloads as W
if OMP:
    O.use_openmp(True)
p = W.scaled(W.preset("small_mc64_f64"), 20000).replace(gamma_e=0.2, n_meta=1e19,
                                                           field_solve=0)
br, bz, sig, parts = W.inputs(p)
o = O.Oracle(p, br, bz, sig, parts)
o.init()
# a potential that does not depend on the deposit's summation order (the
# initial solve amplifies round-off of the charge sum to its tolerance)
r = np.tile(np.arange(p.nr + 1) * p.dr, p.nz + 1)
z = np.repeat(np.arange(p.nz + 1) * p.dz, p.nr + 1)
o.phi[:] = -400.0 * (1.0 - z / p.lz) + 2.0e5 * r * r
for _ in range(3):
    d = o.step()
out = {"d": d, "q": [o.q[0].tolist(), o.q[1].tolist()]}
for s in range(2):
    a = o.particles(s)
    out[f"p{s}"] = {k: v.tolist() for k, v in a.items()}
print(json.dumps(out))
"""


def _run(omp, threads):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    code = SCRIPT.replace("ROOT", repr(ROOT)).replace("OMP", str(bool(omp)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=300, check=True)
    return json.loads(r.stdout.splitlines()[-1])


def test_openmp_build_matches_serial():
    a = _run(False, 1)
    b = _run(True, 4)
    for s in range(2):
        for k in a[f"p{s}"]:
            assert a[f"p{s}"][k] == b[f"p{s}"][k], (s, k)
    for s in range(2):
        qa, qb = np.array(a["q"][s]), np.array(b["q"][s])
        assert np.abs(qa - qb).max() <= 1e-13 * np.abs(qa).max()
    da, db = a["d"], b["d"]
    for k in ("n_abs", "n_cand", "n_coll", "n_see", "n_see_e", "n_child"):
        assert da[k] == db[k], k
    for k in ("ke", "pz"):
        for s in range(2):
            assert abs(da[k][s] - db[k][s]) <= 1e-12 * max(abs(da[k][s]), 1e-30), k
    assert abs(da["dq_conv"] - db["dq_conv"]) <= 1e-12 * max(abs(da["dq_conv"]), 1e-30)
