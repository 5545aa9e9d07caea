"""Training of the learned field-solve preconditioner from pairs the
simulation produces (library calls only; the arithmetic runs in libpic.so).

Pairs (Q, phi) with K phi = Q and phi = 0 on the Dirichlet nodes:
  * snapshots of a running discharge: the deposited charge Q of a step and
    the cathode-at-0-V potential phi0 its field solve returned, and their
    negatives;
  * random potentials smoothed over 0.7 to 24 cells with Q = K phi from the
    library's operator; they cover the part of the spectrum that conjugate-
    gradient residuals visit and smooth discharge snapshots do not.
"""
from __future__ import annotations

import time

import numpy as np

from . import workloads as W


def snapshot_pairs(sim, n, every=2, out=None):
    """n (Q, phi0) pairs from sim, one every `every` steps: device tensors
    [n, nodes] (float64), or written into the first n rows of out = (Q, P)."""
    torch = sim.torch
    nodes = sim.prob.nodes
    if out is None:
        Q = torch.empty((n, nodes), dtype=torch.float64, device=sim.device)
        P = torch.empty_like(Q)
    else:
        Q, P = out
    for k in range(n):
        sim.step(every)
        f = sim.fields()
        with torch.cuda.stream(sim.stream):
            Q[k].copy_(f["q_e"].double() + f["q_i"].double())
            P[k].copy_(f["phi0"])
        sim.stream.synchronize()
    return Q, P


def field_pairs(sim, n, seed):
    """n (K phi, phi) pairs for random potentials (device tensors)."""
    torch = sim.torch
    p = sim.prob
    P = torch.tensor(np.stack(W.random_potentials(p, n, seed)), dtype=torch.float64,
                     device=sim.device)
    Q = torch.empty_like(P)
    for k in range(n):
        sim.apply_operator(P[k], Q[k])
    return Q, P


def output_scale(Q, P, unknown, rows=64):
    """Typical size of phi / rms(Q / (2 pi eps0)): the network output scale
    (the mean over pairs, taken `rows` pairs at a time)."""
    two_pi_eps0 = 2 * np.pi * 8.8541878128e-12
    total = 0.0
    for a in range(0, Q.shape[0], rows):
        q = Q[a:a + rows][:, unknown].double() / two_pi_eps0
        ph = P[a:a + rows][:, unknown].double()
        rho = q.pow(2).mean(dim=1).sqrt()
        total += float((ph / rho[:, None]).pow(2).mean(dim=1).sqrt().sum())
    return total / Q.shape[0]


def train(sim, Q, P, steps=2000, batch=8, lr=1e-3, seed=0, time_limit=None, theta=None,
          report=None, report_seconds=30.0):
    """Adam on random batches of the pairs; the last quarter of the steps
    at 0.3 lr.  report(steps_done, loss), if given, is called about every
    report_seconds.  Returns a summary dict."""
    torch = sim.torch
    rng = np.random.default_rng(seed)
    n = Q.shape[0]
    unknown = torch.tensor(W.unknown_mask(sim.prob), device=sim.device)
    if theta is None:
        theta = init_params(rng)
    sim.pc_set_weights(theta, output_scale(Q, P, unknown))
    losses = []
    t0 = t_rep = time.perf_counter()
    done = 0
    for s in range(steps):
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        idx = torch.tensor(rng.choice(n, size=min(batch, n), replace=False), device=sim.device)
        rate = lr if s < 0.75 * steps else 0.3 * lr
        losses.append(sim.pc_train_step(Q[idx].contiguous(), P[idx].contiguous(), rate))
        done += 1
        if report is not None and time.perf_counter() - t_rep > report_seconds:
            report(done, losses[-1])
            t_rep = time.perf_counter()
    secs = time.perf_counter() - t0
    return {"steps": done, "batch": min(batch, n), "pairs": n, "seconds": secs,
            "ms_per_step": secs / max(done, 1) * 1e3,
            "loss_first": float(np.mean(losses[:10])), "loss_last": float(np.mean(losses[-20:]))}


# (cin, cout) of the 15 convolutions, in the library's order
CONVS = [(2, 16), (16, 16), (16, 16), (16, 16), (16, 48), (48, 48), (48, 80), (80, 80),
         (80, 48), (48, 48), (48, 16), (16, 16), (16, 16), (16, 16), (16, 1)]


def init_params(rng):
    """He-normal weights, zero biases, the output layer at a tenth: the flat
    [cout][cin][3][3] + [cout] vector pic_pc_set_weights takes."""
    parts = []
    for k, (ci, co) in enumerate(CONVS):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if k == len(CONVS) - 1 else 1.0)
        parts.append(rng.normal(size=co * ci * 9) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
