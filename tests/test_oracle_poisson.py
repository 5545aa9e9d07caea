"""Pins for the oracle's R-Z field solve (charge-form finite volumes).

* symmetry and zero row sums of the full operator (a Gauss-law operator);
* face areas tile the disk and the cylinder exactly (geometry);
* Gauss's law over the whole box: induced wall charge = -(free charge);
* the separable case solved by a different algorithm (DST-I in z + banded
  tridiagonal in r, scipy) agrees with the oracle's conjugate gradients;
* a manufactured solution J0(j01 r/R) sin(pi z/L) converges at second order.
"""
import math

import numpy as np
import pytest
from tol import approx
from scipy import fft as sfft
from scipy.linalg import solve_banded
from scipy.special import j0, jn_zeros

from oracle_helpers import make_oracle, zero_field_problem

EPS0 = 8.8541878128e-12


def full_matrix(o):
    n = o.prob.nodes
    K = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        K[:, c] = o.apply_k(e)
    return K


def test_operator_symmetric_zero_rowsum():
    p = zero_field_problem(nr=5, nz=6, lr=0.01, lz=0.013, cathode_rmax=0.006)
    o = make_oracle(p)
    K = full_matrix(o)
    scale = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-14 * scale
    assert np.abs(K.sum(axis=1)).max() <= 1e-14 * scale
    # positive diagonal, non-positive off-diagonal
    assert (np.diag(K) > 0).all()
    off = K - np.diag(np.diag(K))
    assert (off <= 0).all()


def test_face_areas_tile_domain():
    p = zero_field_problem(nr=7, nz=9, lr=0.03, lz=0.05)
    o = make_oracle(p)
    ce, cn = o.couplings()
    ce = ce.reshape(p.nz + 1, p.nr + 1)
    cn = cn.reshape(p.nz + 1, p.nr + 1)
    # axial faces at each z_{j+1/2} tile the disk pi R^2
    for j in range(p.nz):
        area = cn[j].sum() * p.dz / EPS0
        assert area == approx(math.pi * p.lr ** 2, rel=1e-13)
    # radial faces at each r_{i+1/2} tile the side 2 pi r L
    for i in range(p.nr):
        area = ce[:, i].sum() * p.dr / EPS0
        assert area == approx(2 * math.pi * (i + 0.5) * p.dr * p.lz, rel=1e-13)


def test_gauss_law_total_charge():
    p = zero_field_problem(nr=12, nz=10, cathode_rmax=0.012)
    o = make_oracle(p)
    kind = o.node_kind()
    rng = np.random.default_rng(1)
    q = rng.normal(size=p.nodes) * 1e-12
    q[kind != 0] = 0.0
    phi, rc, it, res = o.solve(q, 0.0, rtol=1e-14)
    assert rc == 0
    kp = o.apply_k(phi)
    induced = kp[kind != 0].sum()
    assert induced == approx(-q.sum(), rel=1e-10)


def dst_solve(o, q):
    """Exact solve of the oracle's operator for the all-Dirichlet-z case."""
    p = o.prob
    nr, nz = p.nr, p.nz
    ce, cn = o.couplings()
    ce = ce.reshape(nz + 1, nr + 1)
    cn = cn.reshape(nz + 1, nr + 1)
    # separability: interior-row couplings independent of j
    assert np.allclose(ce[1:nz], ce[1], rtol=0, atol=0)
    assert np.allclose(cn[1:nz], cn[1], rtol=0, atol=0)
    a = ce[1, :nr]          # coupling i <-> i+1 (a[nr-1] couples to the wall)
    c = cn[1, :nr]
    Q = q.reshape(nz + 1, nr + 1)[1:nz, :nr]       # (nz-1, nr) unknowns
    Qh = sfft.dst(Q, type=1, axis=0)
    lam = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, nz) / nz)
    out = np.zeros_like(Qh)
    for k in range(nz - 1):
        diag = a + np.concatenate([[0.0], a[:-1]]) + c * lam[k]
        ab = np.zeros((3, nr))
        ab[0, 1:] = -a[:-1]
        ab[1] = diag
        ab[2, :-1] = -a[:-1]
        out[k] = solve_banded((1, 1), ab, Qh[k])
    phi_u = sfft.idst(out, type=1, axis=0)
    phi = np.zeros((nz + 1, nr + 1))
    phi[1:nz, :nr] = phi_u
    return phi.ravel()


def test_matches_dst_banded_solver():
    p = zero_field_problem(nr=24, nz=40, lr=0.02, lz=0.03)
    o = make_oracle(p)
    kind = o.node_kind()
    rng = np.random.default_rng(2)
    q = rng.normal(size=p.nodes) * 1e-12
    q[kind != 0] = 0.0
    phi, rc, it, res = o.solve(q, 0.0, rtol=1e-14)
    assert rc == 0
    ref = dst_solve(o, q)
    assert np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()


def _manufactured_error(n):
    R, L = 0.02, 0.03
    p = zero_field_problem(nr=n, nz=n, lr=R, lz=L)
    o = make_oracle(p)
    k1 = jn_zeros(0, 1)[0]
    r = np.arange(n + 1) * p.dr
    z = np.arange(n + 1) * p.dz
    Rm, Zm = np.meshgrid(r, z)
    exact = j0(k1 * Rm / R) * np.sin(np.pi * Zm / L)
    rho = EPS0 * ((k1 / R) ** 2 + (np.pi / L) ** 2) * exact
    # control-volume size of each node (clipped to the domain)
    rlo = np.clip(r - 0.5 * p.dr, 0, R)
    rhi = np.clip(r + 0.5 * p.dr, 0, R)
    zlo = np.clip(z - 0.5 * p.dz, 0, L)
    zhi = np.clip(z + 0.5 * p.dz, 0, L)
    vol = np.pi * (rhi ** 2 - rlo ** 2)[None, :] * (zhi - zlo)[:, None]
    phi, rc, it, res = o.solve((rho * vol).ravel(), 0.0, rtol=1e-13)
    assert rc == 0
    return np.abs(phi.reshape(Rm.shape) - exact).max()


def test_manufactured_second_order():
    e = [_manufactured_error(n) for n in (16, 32, 64)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.5 < r1 < 4.6, e
    assert 3.5 < r2 < 4.6, e
    assert e[2] < 2e-3


def test_laplace_cathode_potential_bounded():
    # cathode at 1 V, other walls 0, Neumann block for r > 0.6 R at z = 0
    p = zero_field_problem(nr=20, nz=20, cathode_rmax=0.012)
    o = make_oracle(p)
    kind = o.node_kind()
    phi, rc, it, res = o.solve(np.zeros(p.nodes), 1.0, rtol=1e-14)
    assert rc == 0
    assert (phi[kind == 1] == 1.0).all() and (phi[kind == 2] == 0.0).all()
    inner = phi[kind == 0]
    assert inner.min() > 0.0 and inner.max() < 1.0     # maximum principle
