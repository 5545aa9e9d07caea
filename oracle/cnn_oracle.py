"""FP64 NumPy oracle of the learned Poisson preconditioner (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module; the GPU library never does, and
this module shares no code with it.

What is computed.  The paper solves an electrostatic R-Z field every step
(Section 3, the field solve behind the explicit scheme) but does not name a
solver.  This project accelerates that solve with a preconditioned conjugate
gradient method whose preconditioner is a small convolutional network; the
network and its training are this project's reading, not the paper's:

* Operator.  A = K / (2 pi eps0) on the unknown nodes, K the charge-form
  finite-volume R-Z operator of the field solve (Gauss's law over each
  node's control volume, Section 3).  Dirichlet nodes carry zero.
* Network (4 levels, 196,753 parameters, about 2e5).  Node grid H = nz + 1
  rows by W = nr + 1 columns.  Input channels: r / rms(r) on unknown nodes
  (0 on Dirichlet nodes) and the radial node index i / 256.  Every
  convolution is 3x3 with zero padding and a bias; ``relu`` marks a ReLU
  after it.  Channels per level 16, 16, 48, 80:

      level 0:  c0a = relu(conv(x, 2->16));   e0 = relu(conv(c0a, 16->16))
      level 1:  p1 = pool(e0);  c1a = relu(conv(p1, 16->16));  e1 = relu(conv(c1a, 16->16))
      level 2:  p2 = pool(e1);  c2a = relu(conv(p2, 16->48));  e2 = relu(conv(c2a, 48->48))
      level 3:  p3 = pool(e2);  c3a = relu(conv(p3, 48->80));  e3 = relu(conv(c3a, 80->80))
      level 2:  d2a = relu(conv(up(e3), 80->48) + e2);  d2 = relu(conv(d2a, 48->48))
      level 1:  d1a = relu(conv(up(d2), 48->16) + e1);  d1 = relu(conv(d1a, 16->16))
      level 0:  d0a = relu(conv(up(d1), 16->16) + e0);  d0 = relu(conv(d0a, 16->16))
      out = conv(d0, 16->1)

  pool = 2x2 average over the nodes present (a last odd row or column
  averages fewer nodes), coarse size ceil(n / 2); up = nearest neighbour,
  fine (y, x) <- coarse (y // 2, x // 2).
* Smoothing.  A red-black Gauss-Seidel half sweep of colour c (red: i + j
  even) sets x_p <- x_p + (b - A x)_p / A_pp on the unknown nodes of that
  colour (nodes of one colour do not couple, so the order within a colour
  does not matter).  pre(b): red then black from x = 0; post(x, b): black
  then red.
* Preconditioner.  x1 = pre(r), r1 = r - A x1, the network correction
  c = out_scale * rms(r1) * net(r1 / rms(r1)) on unknown nodes (0 on
  Dirichlet nodes), z = post(x1 + c, r).  With a zero network this is the
  symmetric Gauss-Seidel preconditioner; the network supplies the smooth
  part of the error that the sweeps leave.
* Loss of one pair (b, phi) with A phi = b: x1 = pre(b), r1 = b - A x1,
  e1 = phi - x1 (so A e1 = r1), rho = rms(r1) over the unknown nodes,
  input r1 / rho, target t = e1 / rho, e = out_scale * out - t on unknown
  nodes, L = (1/2) e.A e / (t.A t); a batch averages L.
* Adam with the usual bias corrections.
* Flexible conjugate gradients: beta = z_k.(r_k - r_{k-1}) / z_{k-1}.r_{k-1}
  (the Polak-Ribiere form), which stays convergent with a preconditioner
  that changes between iterations, as a nonlinear network does.

Parameters are one flat FP64 vector: for each convolution in the order
above, its weights [cout][cin][3][3] followed by its bias [cout].
"""
from __future__ import annotations

import numpy as np

EPS0 = 8.8541878128e-12

# (cin, cout) of the 15 convolutions, in order
CONVS = [(2, 16), (16, 16),
         (16, 16), (16, 16),
         (16, 48), (48, 48),
         (48, 80), (80, 80),
         (80, 48), (48, 48),
         (48, 16), (16, 16),
         (16, 16), (16, 16),
         (16, 1)]


def param_count():
    return sum(ci * co * 9 + co for ci, co in CONVS)


def unpack(theta):
    """Flat vector -> list of (w [cout][cin][3][3], b [cout]) views."""
    out, o = [], 0
    for ci, co in CONVS:
        w = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((w, b))
    assert o == theta.size
    return out


def init_params(rng):
    """He-normal weights, zero biases; the output layer starts small."""
    parts = []
    for k, (ci, co) in enumerate(CONVS):
        std = np.sqrt(2.0 / (9 * ci))
        if k == len(CONVS) - 1:
            std *= 0.1
        parts.append(rng.normal(size=co * ci * 9) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# ---- layers (x: [B][C][H][W]) ----------------------------------------------

def conv3x3(x, w, b):
    """y[n, o, i, j] = b[o] + sum_c sum_{u,v} w[o, c, u, v] x[n, c, i+u-1, j+v-1]
    with x = 0 outside the grid."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    y = np.zeros((B, w.shape[0], H, W))
    for u in range(3):
        for v in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, u, v], xp[:, :, u:u + H, v:v + W])
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, gy):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for u in range(3):
        for v in range(3):
            gw[:, :, u, v] = np.einsum("bohw,bchw->oc", gy, xp[:, :, u:u + H, v:v + W])
            gxp[:, :, u:u + H, v:v + W] += np.einsum("oc,bohw->bchw", w[:, :, u, v], gy)
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:H + 1, 1:W + 1], gw, gb


def pool2(x):
    """2x2 average over the nodes present; coarse size ceil(n / 2)."""
    B, C, H, W = x.shape
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    s = np.zeros((B, C, Hc, Wc))
    cnt = np.zeros((Hc, Wc))
    for a in range(2):
        for c in range(2):
            part = x[:, :, a::2, c::2]
            s[:, :, :part.shape[2], :part.shape[3]] += part
            cnt[:part.shape[2], :part.shape[3]] += 1
    return s / cnt


def pool2_backward(g, H, W):
    Hc, Wc = g.shape[2], g.shape[3]
    cnt = np.zeros((Hc, Wc))
    for a in range(2):
        for c in range(2):
            cnt[:len(range(a, H, 2)), :len(range(c, W, 2))] += 1
    gs = g / cnt
    gx = np.zeros(g.shape[:2] + (H, W))
    for a in range(2):
        for c in range(2):
            ny, nx = len(range(a, H, 2)), len(range(c, W, 2))
            gx[:, :, a::2, c::2] = gs[:, :, :ny, :nx]
    return gx


def up2(x, H, W):
    """Nearest neighbour to an H x W grid: fine (y, x) <- coarse (y // 2, x // 2)."""
    return x[:, :, np.arange(H) // 2][:, :, :, np.arange(W) // 2]


def up2_backward(g, Hc, Wc):
    B, C, H, W = g.shape
    gc = np.zeros((B, C, Hc, Wc))
    for a in range(2):
        for c in range(2):
            part = g[:, :, a::2, c::2]
            gc[:, :, :part.shape[2], :part.shape[3]] += part
    return gc


def relu(x):
    return np.maximum(x, 0.0)


# ---- network ---------------------------------------------------------------

def forward(theta, x):
    """Network output [B][1][H][W] and the activations the backward pass needs."""
    P = unpack(theta)
    a = {"x": x}
    a["c0a"] = relu(conv3x3(x, *P[0]))
    a["e0"] = relu(conv3x3(a["c0a"], *P[1]))
    a["p1"] = pool2(a["e0"])
    a["c1a"] = relu(conv3x3(a["p1"], *P[2]))
    a["e1"] = relu(conv3x3(a["c1a"], *P[3]))
    a["p2"] = pool2(a["e1"])
    a["c2a"] = relu(conv3x3(a["p2"], *P[4]))
    a["e2"] = relu(conv3x3(a["c2a"], *P[5]))
    a["p3"] = pool2(a["e2"])
    a["c3a"] = relu(conv3x3(a["p3"], *P[6]))
    a["e3"] = relu(conv3x3(a["c3a"], *P[7]))
    a["u2"] = up2(a["e3"], *a["e2"].shape[2:])
    a["d2a"] = relu(conv3x3(a["u2"], *P[8]) + a["e2"])
    a["d2"] = relu(conv3x3(a["d2a"], *P[9]))
    a["u1"] = up2(a["d2"], *a["e1"].shape[2:])
    a["d1a"] = relu(conv3x3(a["u1"], *P[10]) + a["e1"])
    a["d1"] = relu(conv3x3(a["d1a"], *P[11]))
    a["u0"] = up2(a["d1"], *a["e0"].shape[2:])
    a["d0a"] = relu(conv3x3(a["u0"], *P[12]) + a["e0"])
    a["d0"] = relu(conv3x3(a["d0a"], *P[13]))
    out = conv3x3(a["d0"], *P[14])
    return out, a


def backward(theta, a, g_out):
    """Gradient of sum(g_out * forward(theta, x)) with respect to theta (flat)."""
    P = unpack(theta)
    grads = [None] * len(CONVS)

    def conv_b(k, inp, gy):
        gx, gw, gb = conv3x3_backward(inp, P[k][0], gy)
        grads[k] = (gw, gb)
        return gx

    mask = lambda g, act: g * (act > 0)
    g = conv_b(14, a["d0"], g_out)
    g = conv_b(13, a["d0a"], mask(g, a["d0"]))
    g_h = mask(g, a["d0a"])                  # pre-activation of d0a
    g_e0 = g_h.copy()
    g = conv_b(12, a["u0"], g_h)
    g = up2_backward(g, *a["d1"].shape[2:])
    g = conv_b(11, a["d1a"], mask(g, a["d1"]))
    g_h = mask(g, a["d1a"])
    g_e1 = g_h.copy()
    g = conv_b(10, a["u1"], g_h)
    g = up2_backward(g, *a["d2"].shape[2:])
    g = conv_b(9, a["d2a"], mask(g, a["d2"]))
    g_h = mask(g, a["d2a"])
    g_e2 = g_h.copy()
    g = conv_b(8, a["u2"], g_h)
    g = up2_backward(g, *a["e3"].shape[2:])
    g = conv_b(7, a["c3a"], mask(g, a["e3"]))
    g = conv_b(6, a["p3"], mask(g, a["c3a"]))
    g = pool2_backward(g, *a["e2"].shape[2:]) + g_e2
    g = conv_b(5, a["c2a"], mask(g, a["e2"]))
    g = conv_b(4, a["p2"], mask(g, a["c2a"]))
    g = pool2_backward(g, *a["e1"].shape[2:]) + g_e1
    g = conv_b(3, a["c1a"], mask(g, a["e1"]))
    g = conv_b(2, a["p1"], mask(g, a["c1a"]))
    g = pool2_backward(g, *a["e0"].shape[2:]) + g_e0
    g = conv_b(1, a["c0a"], mask(g, a["e0"]))
    conv_b(0, a["x"], mask(g, a["c0a"]))
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


# ---- preconditioner and loss -------------------------------------------------

def diagonal(apply_a, kind, nr, nz):
    """A_pp of every unknown node: A applied to the indicator of one colour
    equals the diagonal on that colour (same-colour nodes do not couple)."""
    red, black = colours(kind, nr, nz)
    return np.where(red, apply_a(red * 1.0), 0.0) + np.where(black, apply_a(black * 1.0), 0.0)


def colours(kind, nr, nz):
    j, i = np.divmod(np.arange((nr + 1) * (nz + 1)), nr + 1)
    unk = kind == 0
    return unk & ((i + j) % 2 == 0), unk & ((i + j) % 2 == 1)


def half_sweep(x, b, colour, apply_a, diag):
    return np.where(colour, x + (b - apply_a(x)) / np.where(colour, diag, 1.0), x)


def pre_smooth(b, kind, nr, nz, apply_a, diag):
    red, black = colours(kind, nr, nz)
    x = half_sweep(np.zeros_like(b), b, red, apply_a, diag)
    return half_sweep(x, b, black, apply_a, diag)


def post_smooth(x, b, kind, nr, nz, apply_a, diag):
    red, black = colours(kind, nr, nz)
    x = half_sweep(x, b, black, apply_a, diag)
    return half_sweep(x, b, red, apply_a, diag)


def features(r, kind, nr, nz):
    """Network input [2][H][W] of one node vector r, and rms(r) over unknowns."""
    unk = kind == 0
    rms = np.sqrt(np.mean(r[unk] ** 2)) if unk.any() else 0.0
    x = np.zeros((2, nz + 1, nr + 1))
    if rms > 0:
        x[0] = np.where(unk, r / rms, 0.0).reshape(nz + 1, nr + 1)
    x[1] = (np.arange(nr + 1) / 256.0)[None, :]
    return x, rms


def network_correction(theta, out_scale, r, kind, nr, nz):
    """out_scale * rms(r) * net(r / rms(r)) on unknown nodes."""
    x, rms = features(r, kind, nr, nz)
    out, _ = forward(theta, x[None])
    z = out_scale * rms * out[0, 0].ravel()
    return np.where(kind == 0, z, 0.0)


def precondition(theta, out_scale, r, kind, nr, nz, apply_a):
    """z = post(x1 + network_correction(r - A x1), r) with x1 = pre(r)."""
    diag = diagonal(apply_a, kind, nr, nz)
    x1 = pre_smooth(r, kind, nr, nz, apply_a, diag)
    r1 = np.where(kind == 0, r - apply_a(x1), 0.0)
    x2 = x1 + network_correction(theta, out_scale, r1, kind, nr, nz)
    return post_smooth(x2, r, kind, nr, nz, apply_a, diag)


def loss_and_grad(theta, out_scale, b, phi, kind, nr, nz, apply_a):
    """Mean relative A-norm error of the network correction over a batch of
    pairs (b[k], phi[k]) with A phi = b (after pre-smoothing), and its
    gradient in theta.  ``apply_a`` maps a node vector
    (zero on Dirichlet nodes) to A times it on the unknown nodes."""
    unk = kind == 0
    nb = len(b)
    diag = diagonal(apply_a, kind, nr, nz)
    xs, scaled_phi = [], []
    for k in range(nb):
        x1 = pre_smooth(b[k], kind, nr, nz, apply_a, diag)
        r1 = np.where(unk, b[k] - apply_a(x1), 0.0)
        x, rho = features(r1, kind, nr, nz)
        xs.append(x)
        scaled_phi.append(np.where(unk, (phi[k] - x1) / rho, 0.0))
    out, acts = forward(theta, np.stack(xs))
    L = 0.0
    g_out = np.zeros_like(out)
    for k in range(nb):
        z = np.where(unk, out_scale * out[k, 0].ravel(), 0.0)
        e = z - scaled_phi[k]
        ae = np.where(unk, apply_a(e), 0.0)
        den = scaled_phi[k] @ np.where(unk, apply_a(scaled_phi[k]), 0.0)
        L += 0.5 * (e @ ae) / den / nb
        g_out[k, 0] = (out_scale * ae / den / nb).reshape(nz + 1, nr + 1)
    return L, backward(theta, acts, g_out)


def adam_init(theta):
    return {"m": np.zeros_like(theta), "v": np.zeros_like(theta), "t": 0}


def adam_step(theta, grad, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias-corrected moments."""
    state["t"] += 1
    t = state["t"]
    state["m"] = b1 * state["m"] + (1 - b1) * grad
    state["v"] = b2 * state["v"] + (1 - b2) * grad * grad
    mhat = state["m"] / (1 - b1 ** t)
    vhat = state["v"] / (1 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)


def fpcg(apply_a, precond, b, x0, rtol, maxit):
    """Flexible preconditioned CG with the Polak-Ribiere beta.  Returns
    (x, iterations, relative residual ||b - A x|| / ||b||)."""
    x = x0.copy()
    r = b - apply_a(x)
    nb = np.linalg.norm(b)
    if nb == 0:
        return np.zeros_like(b), 0, 0.0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < maxit:
        q = apply_a(p)
        pq = p @ q
        if not (pq > 0 and rz != 0):      # breakdown: no usable direction
            break
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        z_old_r_old = rz
        z = precond(r)
        beta = (z @ (r - r_old)) / z_old_r_old
        rz = r @ z
        p = z + beta * p
    return x, it, np.linalg.norm(r) / nb
