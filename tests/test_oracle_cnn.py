"""Pins for the learned-preconditioner oracle (oracle/cnn_oracle.py).

* the convolution equals scipy's 2-D correlation summed over input channels;
* pooling and upsampling equal their brute-force definitions, and each
  backward is the adjoint of its forward (<L x, y> = <x, L^T y>);
* the full network gradient matches central finite differences of the loss;
* the loss is exactly 1/2 when the network outputs zero;
* the first Adam step equals its closed form -lr g / (|g| + eps);
* flexible CG reaches the direct solution of the field operator, with the
  identity, a Jacobi and a nonlinear (Jacobi plus network) preconditioner;
* a few Adam steps on solved pairs lower the loss.
"""
import math

import numpy as np
import pytest
from tol import approx
from scipy.signal import correlate2d

from oracle import cnn_oracle as N
from oracle_helpers import make_oracle, zero_field_problem

EPS0 = 8.8541878128e-12


def operator(p):
    o = make_oracle(p)
    kind = o.node_kind()
    unk = kind == 0

    def apply_a(v):
        return np.where(unk, o.apply_k(np.where(unk, v, 0.0)) / (2 * math.pi * EPS0), 0.0)

    return o, kind, apply_a


def dense(apply_a, kind):
    idx = np.flatnonzero(kind == 0)
    n = kind.size
    A = np.zeros((idx.size, idx.size))
    for c, node in enumerate(idx):
        e = np.zeros(n)
        e[node] = 1.0
        A[:, c] = apply_a(e)[idx]
    return A, idx


def test_param_count():
    assert N.param_count() == 196753
    assert 1.5e5 < N.param_count() < 2.5e5


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 3, 7, 9))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = N.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.abs(y[n, o] - ref).max() < 1e-12


@pytest.mark.parametrize("H,W", [(6, 8), (7, 9), (5, 4), (1, 3)])
def test_pool_up_definitions(H, W):
    rng = np.random.default_rng(H * 10 + W)
    x = rng.normal(size=(2, 3, H, W))
    p = N.pool2(x)
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    assert p.shape == (2, 3, Hc, Wc)
    for Y in range(Hc):
        for X in range(Wc):
            win = x[:, :, 2 * Y:min(2 * Y + 2, H), 2 * X:min(2 * X + 2, W)]
            assert np.allclose(p[:, :, Y, X], win.mean(axis=(2, 3)), rtol=0, atol=1e-14)
    c = rng.normal(size=(2, 3, Hc, Wc))
    u = N.up2(c, H, W)
    for y in range(H):
        for xx in range(W):
            assert np.array_equal(u[:, :, y, xx], c[:, :, y // 2, xx // 2])


@pytest.mark.parametrize("H,W", [(6, 8), (7, 9), (5, 5)])
def test_backward_is_adjoint(H, W):
    rng = np.random.default_rng(11 + H)
    x = rng.normal(size=(2, 3, H, W))
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    g = rng.normal(size=(2, 3, Hc, Wc))
    assert np.isclose((N.pool2(x) * g).sum(), (x * N.pool2_backward(g, H, W)).sum(), rtol=1e-13)
    gf = rng.normal(size=(2, 3, H, W))
    assert np.isclose((N.up2(g, H, W) * gf).sum(), (g * N.up2_backward(gf, Hc, Wc)).sum(),
                      rtol=1e-13)
    w = rng.normal(size=(5, 3, 3, 3))
    gy = rng.normal(size=(2, 5, H, W))
    y0 = N.conv3x3(x, w, np.zeros(5))
    gx, gw, gb = N.conv3x3_backward(x, w, gy)
    lhs = (y0 * gy).sum()
    assert np.isclose(lhs, (x * gx).sum(), rtol=1e-12)
    assert np.isclose(lhs, (w * gw).sum(), rtol=1e-12)
    assert np.allclose(gb, gy.sum(axis=(0, 2, 3)), rtol=1e-14)


def pairs(p, o, kind, nb, seed):
    """Right-hand sides b (scaled operator units) and their exact solutions."""
    rng = np.random.default_rng(seed)
    unk = kind == 0
    bs, phis = [], []
    r = (np.arange(p.nr + 1) * p.dr)[None, :]
    z = (np.arange(p.nz + 1) * p.dz)[:, None]
    for k in range(nb):
        smooth = np.exp(-((r - rng.uniform(0.2, 0.8) * p.lr) ** 2 + (z - 0.5 * p.lz) ** 2)
                        / (0.2 * p.lr) ** 2)
        b = (smooth + 0.3 * rng.normal(size=smooth.shape)).ravel() * 1e-12
        b = np.where(unk, b, 0.0)
        phi, rc, it, res = o.solve(b, 0.0, rtol=1e-13)
        assert rc == 0
        bs.append(b / (2 * math.pi * EPS0))
        phis.append(phi)
    return bs, phis


def test_loss_gradient_finite_differences():
    """Per layer, the derivative of the loss along a random direction in that
    layer's parameters: central differences with Richardson extrapolation,
    steps small enough that no ReLU changes sign, agree to 1e-6."""
    p = zero_field_problem(nr=10, nz=12, lr=0.01, lz=0.012)
    o, kind, apply_a = operator(p)
    bs, phis = pairs(p, o, kind, 2, 5)
    unk = kind == 0
    rng = np.random.default_rng(7)
    theta = N.init_params(rng)
    theta[-N.CONVS[-1][0] * 9 - 1:] *= 10.0   # make the output layer matter
    rms = [np.sqrt(np.mean(b[unk] ** 2)) for b in bs]
    scale = float(np.mean([np.sqrt(np.mean((ph[unk] / r) ** 2)) for ph, r in zip(phis, rms)]))
    loss = lambda th: N.loss_and_grad(th, scale, bs, phis, kind, p.nr, p.nz, apply_a)[0]
    L, g = N.loss_and_grad(theta, scale, bs, phis, kind, p.nr, p.nz, apply_a)
    assert L > 0.01
    offs = np.cumsum([0] + [ci * co * 9 + co for ci, co in N.CONVS])
    h = 1e-6
    for k in range(len(N.CONVS)):
        v = np.zeros_like(theta)
        v[offs[k]:offs[k + 1]] = rng.normal(size=offs[k + 1] - offs[k])
        v *= np.linalg.norm(theta[offs[k]:offs[k + 1]]) / np.linalg.norm(v)
        d = lambda s: (loss(theta + s * v) - loss(theta - s * v)) / (2 * s)
        fd = (4 * d(h / 2) - d(h)) / 3
        assert abs(fd - g @ v) <= 1e-6 * abs(g @ v), (k, fd, g @ v)


def test_loss_is_half_for_zero_output():
    p = zero_field_problem(nr=8, nz=8, lr=0.01, lz=0.01)
    o, kind, apply_a = operator(p)
    bs, phis = pairs(p, o, kind, 3, 9)
    theta = N.init_params(np.random.default_rng(1))
    ci, co = N.CONVS[-1]
    theta[-(ci * co * 9 + co):] = 0.0
    L, g = N.loss_and_grad(theta, 1.0, bs, phis, kind, p.nr, p.nz, apply_a)
    assert L == approx(0.5, abs=1e-13)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    st = N.adam_init(th)
    lr = 1e-3
    th1 = N.adam_step(th, g, st, lr)
    assert np.allclose(th1, th - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


@pytest.mark.parametrize("pc", ["identity", "jacobi", "network", "sgs", "sandwich"])
def test_fpcg_reaches_direct_solution(pc):
    p = zero_field_problem(nr=12, nz=14, lr=0.012, lz=0.014, cathode_rmax=0.006)
    o, kind, apply_a = operator(p)
    A, idx = dense(apply_a, kind)
    bs, phis = pairs(p, o, kind, 1, 21)
    b = bs[0]
    x_direct = np.zeros(kind.size)
    x_direct[idx] = np.linalg.solve(A, b[idx])
    if pc == "identity":
        M = lambda r: r.copy()
    elif pc == "jacobi":
        d = np.zeros(kind.size)
        d[idx] = np.diag(A)
        M = lambda r: np.where(kind == 0, r / np.where(d > 0, d, 1.0), 0.0)
    elif pc == "sgs":
        theta = np.zeros(N.param_count())
        M = lambda r: N.precondition(theta, 1.0, r, kind, p.nr, p.nz, apply_a)
    elif pc == "sandwich":
        theta = N.init_params(np.random.default_rng(4))
        M = lambda r: N.precondition(theta, 1e-3, r, kind, p.nr, p.nz, apply_a)
    else:
        # nonlinear: Jacobi plus an untrained network's output at 30% of it
        # (an untrained network alone need not give descent directions)
        theta = N.init_params(np.random.default_rng(4))
        d = np.zeros(kind.size)
        d[idx] = np.diag(A)
        jac = lambda r: np.where(kind == 0, r / np.where(d > 0, d, 1.0), 0.0)

        def M(r):
            zj = jac(r)
            zn = N.network_correction(theta, 1.0, r, kind, p.nr, p.nz)
            nn = np.linalg.norm(zn)
            return zj + (0.3 * np.linalg.norm(zj) / nn) * zn if nn > 0 else zj
    x, it, rel = N.fpcg(apply_a, M, b, np.zeros(kind.size), 1e-10, 2000)
    assert rel <= 1e-10
    assert np.abs(x - x_direct).max() <= 1e-8 * np.abs(x_direct).max()
    if pc in ("identity", "jacobi", "sgs"):
        # finite termination for a fixed SPD preconditioner (up to rounding)
        assert it <= idx.size + 5


def test_training_lowers_loss():
    p = zero_field_problem(nr=16, nz=16, lr=0.016, lz=0.016)
    o, kind, apply_a = operator(p)
    bs, phis = pairs(p, o, kind, 4, 31)
    rng = np.random.default_rng(8)
    theta = N.init_params(rng)
    # output scale from the data: rms of the scaled targets
    unk = kind == 0
    rms = [np.sqrt(np.mean(b[unk] ** 2)) for b in bs]
    scale = float(np.mean([np.sqrt(np.mean((ph[unk] / r) ** 2)) for ph, r in zip(phis, rms)]))
    st = N.adam_init(theta)
    L0, g = N.loss_and_grad(theta, scale, bs, phis, kind, p.nr, p.nz, apply_a)
    for _ in range(25):
        L, g = N.loss_and_grad(theta, scale, bs, phis, kind, p.nr, p.nz, apply_a)
        theta = N.adam_step(theta, g, st, 2e-3)
    L1, _ = N.loss_and_grad(theta, scale, bs, phis, kind, p.nr, p.nz, apply_a)
    assert L1 < 0.7 * L0


def test_zero_network_is_symmetric_gauss_seidel():
    """With a zero network the preconditioner is red-black symmetric
    Gauss-Seidel: z1 = (D + L)^-1 r, z = z1 + (D + U)^-1 (r - A z1) in the
    ordering red nodes first, from a dense matrix; and it is symmetric."""
    from scipy.linalg import solve_triangular
    p = zero_field_problem(nr=9, nz=11, lr=0.009, lz=0.011, cathode_rmax=0.005)
    o, kind, apply_a = operator(p)
    A, idx = dense(apply_a, kind)
    red, black = N.colours(kind, p.nr, p.nz)
    order = np.concatenate([np.flatnonzero(red[idx]), np.flatnonzero(black[idx])])
    Ao = A[np.ix_(order, order)]
    rng = np.random.default_rng(3)
    r = np.zeros(kind.size)
    r[idx] = rng.normal(size=idx.size)
    theta = np.zeros(N.param_count())
    z = N.precondition(theta, 1.0, r, kind, p.nr, p.nz, apply_a)
    ro = r[idx][order]
    z1 = solve_triangular(np.tril(Ao), ro, lower=True)
    zo = z1 + solve_triangular(np.triu(Ao), ro - Ao @ z1, lower=False)
    ref = np.zeros(kind.size)
    ref[idx[order]] = zo
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()
    s2 = np.zeros(kind.size)
    s2[idx] = rng.normal(size=idx.size)
    z2 = N.precondition(theta, 1.0, s2, kind, p.nr, p.nz, apply_a)
    assert abs(s2 @ z - r @ z2) <= 1e-12 * abs(r @ z2)
