"""Collective pins for the oracle (whole timesteps, fields solved).

* cold plasma oscillation: frozen ions, quiet start, an electron displacement
  grad(psi) with psi = A J0(j01 r/R) sin(pi z/L); the field energy oscillates
  at twice the leapfrog plasma frequency (2/dt) asin(w_pe dt / 2);
* EC-PIC conserves total energy in a grounded, reflecting box when the cell
  is 3 Debye lengths, while MC-PIC heats (finite-grid instability) -- the
  paper's central comparison (Sections 2 and 5).
"""
import math

import numpy as np
import pytest
from tol import approx
from scipy.special import j0, j1, jn_zeros

from oracle_helpers import make_oracle, species
from paper_2507_10727_amd import workloads as W

QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12


def _box(**kw):
    base = dict(name="box", nr=16, nz=16, lr=0.01, lz=0.01, circuit=W.FIXED_V,
                v_fixed=0.0, v_ext=0.0, mcc_on=0, see_on=0, frozen_ions=1,
                wall_bc=(W.REFLECT, W.REFLECT, W.REFLECT), gamma_i=0.0)
    base.update(kw)
    return W.Problem(**base)


def test_cold_plasma_frequency():
    n0 = 1e14
    wpe = math.sqrt(n0 * QE * QE / (EPS0 * ME))
    dt = 0.2 / wpe
    R = L = 0.01
    nr_, nz_ = 96, 96
    rk = R * np.sqrt((np.arange(nr_) + 0.5) / nr_)
    zk = L * (np.arange(nz_) + 0.5) / nz_
    Rg, Zg = np.meshgrid(rk, zk)
    r, z = Rg.ravel(), Zg.ravel()
    n = r.shape[0]
    p = _box(dt=dt, density=n0, n_per_species=n)
    k1 = jn_zeros(0, 1)[0]
    kr, kz = k1 / R, math.pi / L
    amp = 0.03 * p.dr / kr
    dr_ = -amp * kr * j1(kr * r) * np.sin(kz * z)
    dz_ = amp * kz * j0(kr * r) * np.cos(kz * z)
    el = species(r + dr_, z + dz_, 0.0, 0.0, 0.0)
    io = species(r, z, 0.0, 0.0, 0.0)
    o = make_oracle(p, [el, io], b=None, capacity=(n + 16, n + 16))
    o.init()
    steps = 240
    w = np.array([o.step()["w_field"] for _ in range(steps)])
    t = np.arange(steps)
    best, wbest = None, None
    for om in np.linspace(0.8, 1.2, 4001) * wpe:
        A = np.stack([np.ones(steps), np.cos(2 * om * dt * t), np.sin(2 * om * dt * t)], 1)
        coef, res, *_ = np.linalg.lstsq(A, w, rcond=None)
        err = np.sum((A @ coef - w) ** 2)
        if best is None or err < best:
            best, wbest = err, om
    expect = 2.0 / dt * math.asin(wpe * dt / 2)
    assert wbest == approx(expect, rel=0.02)


def _thermal_box(scheme, steps):
    te = 2.0
    lam = 0.01 / 16 / 3.0            # cell = 3 Debye lengths
    n0 = EPS0 * te / (QE * lam * lam)
    wpe = math.sqrt(n0 * QE * QE / (EPS0 * ME))
    npart = 16 * 16 * 32
    p = _box(scheme=scheme, dt=0.1 / wpe, density=n0, n_per_species=npart, te_ev=te,
             ti_ev=0.0, seed=99)
    el, io = W.load_uniform(p)
    io.vr[:] = 0; io.vt[:] = 0; io.vz[:] = 0
    el.r[:] = io.r; el.z[:] = io.z      # start neutral
    o = make_oracle(p, [el, io], capacity=(npart + 16, npart + 16))
    o.init()
    ke, tot = [], []
    for _ in range(steps):
        d = o.step()
        ke.append(d["ke"][0])
        tot.append(d["ke"][0] + d["w_field"])
    return np.array(ke), np.array(tot)


@pytest.mark.slow
def test_ec_energy_bounded_mc_heats():
    steps = 8000
    ke_ec, tot_ec = _thermal_box(W.EC_PIC, steps)
    ke_mc, tot_mc = _thermal_box(W.MC_PIC, steps)
    e0 = tot_ec[1]
    drift_ec = np.abs(tot_ec[1:] - e0).max() / e0
    assert drift_ec < 0.01, drift_ec
    growth_mc = ke_mc[-200:].mean() / ke_mc[1:201].mean() - 1.0
    assert growth_mc > 0.10, growth_mc
