"""Pins for the oracle's particle side: deposit, gather, push, walls.

* deposit: total charge, single-particle tent weights, uniform load gives the
  uniform density at every node (exact cylindrical volume of the tent);
* gather: EC field = minus the gradient of the bilinear interpolant of phi
  (finite differences of an independent interpolant); MC momentum identity
  sum_p q w E(x_p) = sum_n Q_n E_n; linear phi gives the exact uniform field;
* push: discrete Boris gyration (closed form of the rotated-velocity orbit,
  with the R-Z mapping), straight-line motion through the axis, E x B drift.
"""
import math

import numpy as np
import pytest
from tol import approx

from oracle_helpers import empty, make_oracle, species, zero_field_problem
from paper_2507_10727_amd import workloads as W

QE = 1.602176634e-19
ME = 9.1093837015e-31


# ---------------------------------------------------------------- deposit ---
def test_deposit_total_charge():
    p = zero_field_problem(nr=20, nz=30, lr=0.02, lz=0.03)
    o = make_oracle(p)
    rng = np.random.default_rng(3)
    n = 50000
    r = p.lr * np.sqrt(rng.random(n))
    z = p.lz * rng.random(n)
    q = o.deposit(r, z, -3.7e-14)
    assert q.sum() == approx(-3.7e-14 * n, rel=1e-13)


def test_deposit_single_particle_weights():
    p = zero_field_problem(nr=8, nz=8, lr=0.008, lz=0.008)
    o = make_oracle(p)
    q = o.deposit([2.25e-3], [3.5e-3], 1.0).reshape(9, 9)  # (j, i)
    expect = {(3, 2): 0.75 * 0.5, (3, 3): 0.25 * 0.5, (4, 2): 0.75 * 0.5, (4, 3): 0.25 * 0.5}
    for (j, i), v in expect.items():
        assert q[j, i] == approx(v, rel=1e-14)
    assert np.count_nonzero(q) == 4


def test_uniform_load_gives_uniform_density():
    """E[Q_n] = q n * integral of the tent over the node's support, whose
    closed form in cylindrical geometry is pi dr^2 dz_j / 3 on the axis,
    2 pi r_i dr dz_j inside and (pi dr R - pi dr^2 / 3) dz_j at r = R."""
    p = zero_field_problem(nr=8, nz=8, lr=0.01, lz=0.01)
    o = make_oracle(p)
    rng = np.random.default_rng(4)
    n = 2_000_000
    r = p.lr * np.sqrt(rng.random(n))
    z = p.lz * rng.random(n)
    dens = n / (math.pi * p.lr ** 2 * p.lz)
    q = o.deposit(r, z, 1.0).reshape(p.nz + 1, p.nr + 1)
    dr, dz = p.dr, p.dz
    i = np.arange(p.nr + 1)
    vr = 2 * math.pi * i * dr * dr
    vr[0] = math.pi * dr * dr / 3
    vr[-1] = math.pi * dr * p.lr - math.pi * dr * dr / 3
    vz = np.full(p.nz + 1, dz)
    vz[0] = vz[-1] = dz / 2
    expect = dens * vz[:, None] * vr[None, :]
    # statistical: each weight <= 1, so var(Q_n) <= E[Q_n]
    z5 = (q - expect) / np.sqrt(expect)
    assert np.abs(z5).max() < 5.0


# ----------------------------------------------------------------- gather ---
def _bilinear(phi2, p, r, z):
    """Independent bilinear interpolant of nodal values (scipy)."""
    from scipy.interpolate import RegularGridInterpolator
    f = RegularGridInterpolator((np.arange(p.nz + 1) * p.dz, np.arange(p.nr + 1) * p.dr), phi2)
    return f(np.stack([z, r], axis=-1))


def test_ec_field_is_gradient_of_interpolant():
    p = zero_field_problem(nr=10, nz=12, lr=0.01, lz=0.012, scheme=W.EC_PIC)
    o = make_oracle(p)
    rng = np.random.default_rng(5)
    phi = rng.normal(size=p.nodes) * 10
    # points away from cell edges so a centred difference stays in one cell
    ci = rng.integers(0, p.nr, 400)
    cj = rng.integers(0, p.nz, 400)
    r = (ci + 0.1 + 0.8 * rng.random(400)) * p.dr
    z = (cj + 0.1 + 0.8 * rng.random(400)) * p.dz
    er, ez, _, _ = o.gather(phi, r, z)
    phi2 = phi.reshape(p.nz + 1, p.nr + 1)
    h = 1e-4 * p.dr
    fd_r = -(_bilinear(phi2, p, r + h, z) - _bilinear(phi2, p, r - h, z)) / (2 * h)
    fd_z = -(_bilinear(phi2, p, r, z + h) - _bilinear(phi2, p, r, z - h)) / (2 * h)
    scale = np.abs(phi).max() / p.dr
    assert np.abs(er - fd_r).max() < 1e-7 * scale
    assert np.abs(ez - fd_z).max() < 1e-7 * scale


def test_ec_er_is_ngp_in_r():
    """E_r is constant across a cell in r (nearest edge), linear in z."""
    p = zero_field_problem(nr=6, nz=6, lr=0.006, lz=0.006, scheme=W.EC_PIC)
    o = make_oracle(p)
    rng = np.random.default_rng(6)
    phi = rng.normal(size=p.nodes)
    z = np.full(5, 2.3e-3)
    r = np.array([3.01, 3.2, 3.5, 3.8, 3.99]) * 1e-3
    er, ez, _, _ = o.gather(phi, r, z)
    assert np.ptp(er) < 1e-12 * np.abs(er).max()
    assert np.ptp(ez) > 1e-6  # varies in r


def test_linear_phi_gives_uniform_field():
    for scheme in (W.MC_PIC, W.EC_PIC):
        p = zero_field_problem(nr=10, nz=10, lr=0.01, lz=0.01, scheme=scheme)
        o = make_oracle(p)
        r = np.arange(p.nr + 1) * p.dr
        z = np.arange(p.nz + 1) * p.dz
        a, b = 1234.0, -567.0
        phi = (a * r[None, :] + b * z[:, None]).ravel()
        rng = np.random.default_rng(7)
        rr = (1 + (p.nr - 2) * rng.random(100)) * p.dr   # keep off the axis cell
        zz = p.lz * rng.random(100)
        er, ez, _, _ = o.gather(phi, rr, zz)
        assert np.abs(er + a).max() < 1e-9 * abs(a)
        assert np.abs(ez + b).max() < 1e-9 * abs(a)


def test_mc_momentum_identity():
    p = zero_field_problem(nr=12, nz=14, lr=0.012, lz=0.014, scheme=W.MC_PIC)
    o = make_oracle(p)
    rng = np.random.default_rng(8)
    phi = rng.normal(size=p.nodes)
    n = 5000
    r = p.lr * np.sqrt(rng.random(n))
    z = p.lz * rng.random(n)
    er, ez, _, _ = o.gather(phi, r, z)
    qn = o.deposit(r, z, 1.0)
    ern, ezn = o.nodal_e(phi)
    assert er.sum() == approx((qn * ern).sum(), rel=1e-11)
    assert ez.sum() == approx((qn * ezn).sum(), rel=1e-11)


# ------------------------------------------------------------------- push ---
def _push_problem(**kw):
    base = dict(nr=40, nz=40, lr=0.02, lz=0.02, field_solve=0, mcc_on=0, see_on=0,
                frozen_ions=1, wall_bc=(W.REFLECT, W.REFLECT, W.REFLECT), weight=1.0,
                v_fixed=0.0, v_ext=0.0)
    base.update(kw)
    return zero_field_problem(**base)


def _run_single(p, part, phi=None, b=None, steps=100, record=("r",)):
    o = make_oracle(p, [part, empty()], b=b)
    o.init()
    o.phi[:] = 0.0 if phi is None else phi
    out = {k: [] for k in record}
    for _ in range(steps):
        o.step()
        a = o.particles(0)
        for k in record:
            out[k].append(a[k][0])
    return {k: np.array(v) for k, v in out.items()}


def test_boris_gyration_discrete_orbit():
    b0 = 0.02
    p = _push_problem()
    nn = p.nodes
    r0, vr0, vt0 = 0.01, 3e5, 1e5
    steps = 800
    out = _run_single(p, species(r0, 0.01, vr0, vt0, 0.0), b=(np.zeros(nn), np.full(nn, b0)),
                      steps=steps, record=("r", "vr", "vt", "z"))
    # closed form: v^{n+1/2} = Rot(theta)^(n+1) v^{-1/2}, theta = -2 atan(q B dt / 2m)
    theta = -2 * math.atan(-QE * b0 * p.dt / (2 * ME))
    x = np.array([r0, 0.0])
    v = np.array([vr0, vt0])
    c, s = math.cos(theta), math.sin(theta)
    rs = []
    for _ in range(steps):
        v = np.array([c * v[0] - s * v[1], s * v[0] + c * v[1]])
        x = x + v * p.dt
        rs.append(math.hypot(*x))
    rs = np.array(rs)
    assert np.abs(out["r"] - rs).max() < 1e-10 * r0
    speed = np.hypot(out["vr"], out["vt"])
    assert np.abs(speed - math.hypot(vr0, vt0)).max() < 1e-9 * math.hypot(vr0, vt0)
    assert np.all(out["z"] == 0.01)
    # orbit radius of the discrete Boris map vs the analytic Larmor radius
    wc = QE * b0 / ME
    rl = math.hypot(vr0, vt0) / wc
    xs = []
    x = np.array([r0, 0.0]); v = np.array([vr0, vt0])
    for _ in range(int(2 * math.pi / abs(theta)) + 2):
        v = np.array([c * v[0] - s * v[1], s * v[0] + c * v[1]]); x = x + v * p.dt; xs.append(x)
    xs = np.array(xs)
    ctr = xs.mean(axis=0)
    rad = np.hypot(*(xs - ctr).T).mean()
    assert rad == approx(rl * math.sqrt(1 + (wc * p.dt / 2) ** 2), rel=2e-3)


def test_straight_line_through_axis():
    p = _push_problem()
    r0, vr, vt = 5e-4, -1.0e5, 2.0e3
    steps = 2000
    out = _run_single(p, species(r0, 0.01, vr, vt, 0.0), steps=steps, record=("r", "vr", "vt"))
    t = p.dt * np.arange(1, steps + 1)
    exact = np.hypot(r0 + vr * t, vt * t)
    assert np.abs(out["r"] - exact).max() < 1e-11 * r0
    # the particle crossed the axis: radial velocity changes sign, speed kept
    assert out["vr"][0] < 0 < out["vr"][-1]
    assert np.abs(np.hypot(out["vr"], out["vt"]) - math.hypot(vr, vt)).max() < 1e-6


def test_exb_drift():
    e0, b0 = 100.0, 0.05
    p = _push_problem(lr=0.02)
    r = np.arange(p.nr + 1) * p.dr
    phi = np.tile(-e0 * r, p.nz + 1)
    nn = p.nodes
    steps = 3000
    out = _run_single(p, species(0.01, 0.01, 0.0, 0.0, 0.0), phi=phi,
                      b=(np.zeros(nn), np.full(nn, b0)), steps=steps, record=("vt",))
    theta = 2 * math.atan(QE * b0 * p.dt / (2 * ME))
    n = np.arange(steps)
    A = np.stack([np.ones(steps), np.cos(theta * n), np.sin(theta * n)], axis=1)
    coef, *_ = np.linalg.lstsq(A, out["vt"], rcond=None)
    assert coef[0] == approx(-e0 / b0, rel=1e-3)
