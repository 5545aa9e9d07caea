"""The paper's central comparison on the GPU path (Sections 2 and 5): in a
closed box (reflecting walls, grounded, no collisions or emission, frozen
ions, quiet neutral start) whose cell is three Debye lengths, EC-PIC keeps
the total energy (kinetic + field) bounded while MC-PIC heats the electrons
(finite-grid instability).  The same check runs on the oracle at a smaller
size in test_oracle_plasma.py; here the state is FP32 as in production.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_sim, say
from paper_2507_10727_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_box(scheme, n_cells, steps, every):
    p, parts = W.thermal_box(n_cells, n_cells, 0.01 / 16, 32, scheme)
    br, bz = W.magnetron_field(p)
    sim = gpu_sim(p, br, bz, W.cross_sections(p.e_exc, p.e_iz), parts)
    ke, tot = [], []
    for _ in range(steps // every):
        sim.step(every)
        d = sim.diag()
        ke.append(d["ke"][0])
        tot.append(d["ke"][0] + d["w_field"])
    sim.close()
    return np.array(ke), np.array(tot)


def test_ec_energy_bounded_mc_heats():
    steps, every = 8000, 20
    say("case thermal box 64x64 cells, 131072 per species, FP32, EC then MC")
    ke_ec, tot_ec = run_box(W.EC_PIC, 64, steps, every)
    ke_mc, tot_mc = run_box(W.MC_PIC, 64, steps, every)
    drift_ec = np.abs(tot_ec - tot_ec[0]).max() / tot_ec[0]
    m = len(ke_mc) // 40
    growth_mc = ke_mc[-m:].mean() / ke_mc[:m].mean() - 1.0
    say(f"EC total-energy drift {drift_ec:.2e}, MC kinetic-energy growth {growth_mc:.2%}")
    assert drift_ec < 0.01, drift_ec
    assert growth_mc > 0.10, growth_mc
