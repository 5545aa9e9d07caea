"""Shared helpers for the oracle's CPU tests (no method arithmetic here)."""
import numpy as np

from oracle import oracle as O
from paper_2507_10727_amd import workloads as W


def zero_field_problem(**kw):
    """A small problem with no magnetic field (override b arrays separately)."""
    base = dict(name="t", nr=16, nz=16, lr=0.02, lz=0.02, n_per_species=0)
    base.update(kw)
    return W.Problem(**base)


def make_oracle(p, parts=None, b=None, capacity=None, sigma=None):
    nn = p.nodes
    if b is None:
        br = np.zeros(nn)
        bz = np.zeros(nn)
    else:
        br, bz = b
    sig = W.cross_sections(p.e_exc, p.e_iz, e_iz_meta=p.e_iz_meta) if sigma is None else sigma
    if parts is None:
        parts = [W.SpeciesArrays(*(np.zeros(0) for _ in range(5)), np.zeros(0, np.uint32))
                 for _ in range(2)]
    cap = capacity or (max(parts[0].n, 16) * 2 + 64, max(parts[1].n, 16) * 2 + 64)
    return O.Oracle(p, br, bz, sig, parts, capacity=cap)


def species(r, z, vr, vt, vz, ids=None):
    r = np.atleast_1d(np.asarray(r, np.float64))
    n = r.shape[0]
    f = lambda a: np.broadcast_to(np.asarray(a, np.float64), (n,)).copy()
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.asarray(ids, np.uint32)
    return W.SpeciesArrays(f(r), f(z), f(vr), f(vt), f(vz), ids)


def empty():
    return species(np.zeros(0), 0, 0, 0, 0)
