"""Helpers for the GPU parity tests (HIP library vs the FP64 oracle)."""
import math
import sys

import numpy as np

from oracle import oracle as O
from paper_2507_10727_amd import workloads as W

QE = 1.602176634e-19
ME = 9.1093837015e-31


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_sim(p, br, bz, sig, parts, **kw):
    from paper_2507_10727_amd.sim import Simulation
    return Simulation(p, br, bz, sig, parts, **kw)


def to_species(d):
    return W.SpeciesArrays(d["r"].copy(), d["z"].copy(), d["vr"].copy(), d["vt"].copy(),
                           d["vz"].copy(), d["id"].astype(np.uint32).copy())


def vth(p, s):
    t = p.te_ev if s == 0 else p.ti_ev
    m = ME if s == 0 else W.M_AR - ME
    return math.sqrt(max(t, 1e-3) * QE / m)


def compare_particles(p, g, o, s, tol, max_mismatch=0):
    """Compare GPU and oracle particles of species s by id.

    Positions relative to the cell size, velocities relative to
    (v_th,s + |v|).  Returns (worst position error, worst velocity error,
    number of ids present on only one side)."""
    gi = np.argsort(g["id"])
    oi = np.argsort(o["id"])
    gid, oid = g["id"][gi], o["id"][oi]
    common, ga, ob = np.intersect1d(gid, oid, assume_unique=True, return_indices=True)
    only = len(gid) + len(oid) - 2 * len(common)
    assert only <= max_mismatch, (s, only, np.setxor1d(gid, oid)[:20])
    G = {k: g[k][gi][ga] for k in ("r", "z", "vr", "vt", "vz")}
    Ov = {k: o[k][oi][ob] for k in ("r", "z", "vr", "vt", "vz")}
    ep = max(np.abs(G["r"] - Ov["r"]).max(initial=0) / p.dr,
             np.abs(G["z"] - Ov["z"]).max(initial=0) / p.dz)
    vt = vth(p, s)
    ev = 0.0
    for k in ("vr", "vt", "vz"):
        e = np.abs(G[k] - Ov[k]) / (vt + np.abs(Ov[k]))
        ev = max(ev, e.max(initial=0))
    return ep, ev, only


def oracle_from_gpu(p, br, bz, sig, sim, **kw):
    """An oracle run whose particles are the GPU's current particles."""
    parts = [to_species(sim.particles(s)) for s in range(2)]
    cap = (max(parts[0].n * 2, 1024), max(parts[1].n * 2, 1024))
    o = O.Oracle(p, br, bz, sig, parts, capacity=cap, **kw)
    return o
