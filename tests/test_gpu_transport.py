"""Transport of slow particles in the FP32 state.

The FP32 state keeps a particle's in-cell offset on a grid of 2^-21 cell.
A step's displacement is rounded to that grid without bias (down after a
dither of the particle slot and step), so a particle of steady velocity
covers v dt per step on average however slow it is; rounding the new offset
to nearest would stop any particle that moves less than half a quantum per
step and shorten every steady displacement by the same fraction of a
quantum.  The FP64 state runs the same case as the control (no rounding).

Setup: ions only, no field (no field solve, cathode at 0 V, no magnetic
field), no collisions or emission, 10^4 steps of 5 ps.  Three groups of
2000 ions at rest radially with v_z = 2, 20 and 200 m/s: 0.021, 0.21 and
2.1 quanta per step on a 1 mm cell."""
import numpy as np
import pytest

from gpu_helpers import gpu_sim, say
from paper_2507_10727_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 10_000
SPEEDS = (2.0, 20.0, 200.0)
PER_GROUP = 2000


def _case(prec):
    p = W.Problem(name="drift", nr=16, nz=16, lr=0.016, lz=0.016, n_per_species=0,
                  precision=prec, field_solve=0, circuit=W.FIXED_V, v_fixed=0.0,
                  mcc_on=0, see_on=0, gamma_i=0.0, gamma_e=0.0, b_peak=0.0, dt=5e-12)
    rng = np.random.default_rng(3)
    n = PER_GROUP * len(SPEEDS)
    r = 0.004 + 0.008 * rng.random(n)
    z = 0.004 + 0.008 * rng.random(n)
    vz = np.repeat(SPEEDS, PER_GROUP)
    ions = W.SpeciesArrays(r, z, np.zeros(n), np.zeros(n), vz, np.arange(n, dtype=np.uint32))
    none = W.SpeciesArrays(*(np.zeros(0) for _ in range(5)), np.zeros(0, np.uint32))
    nn = p.nodes
    return p, np.zeros(nn), np.zeros(nn), W.cross_sections(), [none, ions]


def _drift(prec):
    p, br, bz, sig, parts = _case(prec)
    sim = gpu_sim(p, br, bz, sig, [x.copy() for x in parts], capacity=(1024, 8192))
    sim.step(STEPS)
    g = sim.particles(1)
    sim.close()
    o = np.argsort(g["id"])
    dz = g["z"][o] - parts[1].z
    dr = g["r"][o] - parts[1].r
    return p, dz, dr


@pytest.mark.parametrize("prec", [W.F32, W.F64])
def test_slow_ions_drift_the_analytic_distance(prec):
    """Mean axial drift of each group within 1% of v dt N (FP32; the dither
    noise of a group mean is about 0.2%); FP64 within 2e-8 (each step adds a
    displacement of 1e-8 cell or more to an offset below one cell, rounding
    the sum by at most 2^-53 cell); no radial motion beyond one quantum per
    particle."""
    p, dz, dr = _drift(prec)
    tol = 1e-2 if prec == W.F32 else 2e-8
    for g, v in enumerate(SPEEDS):
        sl = slice(g * PER_GROUP, (g + 1) * PER_GROUP)
        want = v * p.dt * STEPS
        got = float(dz[sl].mean())
        say(f"  {prec} v_z = {v:6.1f} m/s: drift {got:.6e} m, expected {want:.6e} m "
            f"({got / want - 1:+.2e})")
        assert abs(got / want - 1.0) <= tol
    assert np.abs(dr).max() <= p.dr * 2.0 ** -21 * 1.01
