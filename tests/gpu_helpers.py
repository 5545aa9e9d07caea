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


# ---- decision parity (FP32): the oracle's decision evaluated on the GPU's
# own pre-decision values, mismatches allowed only within a band of the
# threshold ---------------------------------------------------------------
BAND_ULPS = 4
ULP32 = 2.0 ** -23           # relative spacing of binary32 numbers in [1, 2)
POS_QUANTUM = 2.0 ** -21     # position resolution of the FP32 state (cells)


def twin(sim, prob, br, bz, sig, capacity):
    """A second simulation of `prob` holding a bitwise copy of sim's particle
    arrays, scalar state and potential (its push then gives the same values
    particle for particle)."""
    import torch
    t = gpu_sim(prob, br, bz, sig, None, capacity=capacity)
    st = sim.get_state()
    t.set_state(st)
    torch.cuda.synchronize()
    for s in range(2):
        a, b = sim.particle_tensors(s), t.particle_tensors(s)
        assert a.keys() == b.keys()
        for k in a:
            b[k].copy_(a[k])
    torch.cuda.synchronize()
    phi = sim.fields_host()["phi"]
    sim.set_phi(phi)
    t.set_phi(phi)
    return t


def energy_ev(d):
    return 0.5 * ME * (d["vr"] ** 2 + d["vt"] ** 2 + d["vz"] ** 2) / QE


def gpu_processes(after, pushed, ids, o=None, step=0, new_from=2 ** 32):
    """The collision each electron of `ids` underwent on the GPU, from its
    velocity after the step (`after`) and after the push alone (`pushed`, a
    run without collisions from the same state): -1 none; otherwise the
    process whose energy outcome is nearest the GPU's -- 0 elastic (E
    (1 - 2 m/M (1 - cos)), within 4 m/M E), 1 excitation (E - E_exc), 2 and 3
    ionization from the ground state and from the metastable ((1 - U)(E -
    E_thr), U the first word of the electron's ionization draw from the
    oracle's generator); 8 when two outcomes are too close to tell apart, 9
    when none fits."""
    from oracle import oracle as O
    p = o.prob
    def pick(d):
        order = np.argsort(d["id"])
        k = order[np.searchsorted(d["id"][order], ids)]
        assert np.array_equal(d["id"][k], ids)
        return {n: d[n][k] for n in ("vr", "vt", "vz")}
    a, b = pick(after), pick(pushed)
    pa = {n: pick_pos(after, ids, n) for n in ("r", "z")}
    changed = (a["vr"] != b["vr"]) | (a["vt"] != b["vt"]) | (a["vz"] != b["vz"])
    ea, eb = energy_ev(a), energy_ev(b)
    proc = np.full(ids.shape[0], -1, np.int32)
    key = [p.seed & 0xffffffff, p.seed >> 32]
    m_ratio = 4 * ME / (39.948 * 1.66053906660e-27)
    # new electrons (ejected ones sit exactly at their parent's position)
    kids = after["id"] >= new_from
    kid_pos = {}
    for r_, z_, e_ in zip(after["r"][kids], after["z"][kids], energy_ev(after)[kids]):
        kid_pos.setdefault((r_, z_), []).append(e_)
    for k in np.flatnonzero(changed):
        u = O.philox([int(ids[k]), (p.run << 8) | 1, int(step) & 0xffffffff, 0], key)
        split = (int(u[0]) >> 8) / 2 ** 24
        tol = 1e-4 * eb[k] + 1e-4
        err = {1: abs(ea[k] - (eb[k] - p.e_exc)) if eb[k] >= p.e_exc else np.inf,
               2: abs(ea[k] - (1 - split) * (eb[k] - p.e_iz)) if eb[k] >= p.e_iz else np.inf,
               3: (abs(ea[k] - (1 - split) * (eb[k] - p.e_iz_meta))
                   if eb[k] >= p.e_iz_meta and p.n_meta > 0 else np.inf)}
        loss = eb[k] - ea[k]
        err[0] = 0.0 if -tol <= loss <= m_ratio * eb[k] + tol else np.inf
        near = [c for c in err if err[c] <= 10 * tol]
        if len(near) > 1:
            # outcomes too close to tell by the scattered energy: an
            # ionization leaves an ejected electron with split (E - E_thr) at
            # the parent's (exact) position, the other processes none
            ej = kid_pos.get((pa["r"][k], pa["z"][k]), [])
            thr = {2: p.e_iz, 3: p.e_iz_meta}
            for c in near:
                if c in thr:
                    ok_c = any(abs(x - split * (eb[k] - thr[c])) <= tol for x in ej)
                else:
                    ok_c = len(ej) == 0
                if not ok_c:
                    err[c] = np.inf
        order = sorted(err, key=lambda c: err[c])
        best, second = order[0], order[1]
        if err[best] > tol:
            proc[k] = 9
        elif err[second] <= 10 * tol:
            proc[k] = 8
        else:
            proc[k] = best
    return proc


def pick_pos(d, ids, name):
    order = np.argsort(d["id"])
    k = order[np.searchsorted(d["id"][order], ids)]
    return d[name][k]


def check_mcc_decisions(o, after, pushed, pre_next_id, step, band=BAND_ULPS * ULP32):
    """Every electron that existed before the step and survived its push:
    the oracle's decision (orc_mcc_select) on the GPU's pushed velocity must
    equal the GPU's outcome, unless the deciding comparison lies within
    `band` (relative) of its threshold.  Returns (candidates, collisions per
    process, cases within the band)."""
    sel = pushed["id"] < pre_next_id
    ids = np.sort(pushed["id"][sel])
    o_sorted = np.argsort(pushed["id"])
    k = o_sorted[np.searchsorted(pushed["id"][o_sorted], ids)]
    code, margin = o.mcc_select(ids, step, pushed["vr"][k], pushed["vt"][k], pushed["vz"][k])
    gproc = gpu_processes(after, pushed, ids, o, step, pre_next_id)
    assert not np.any(gproc == 9), ids[gproc == 9][:10]
    n_amb = int((gproc == 8).sum())
    assert n_amb <= 2, n_amb
    expect = np.where(code < 0, -1, code)
    bad = (expect != gproc) & (gproc != 8)
    in_band = bad & (margin <= band)
    say(f"  mcc decisions: candidates {int((code >= -1).sum())}, collisions "
        f"{[int((gproc == q).sum()) for q in range(4)]}, mismatches {int(bad.sum())} "
        f"(within {band:.2e} of a threshold: {int(in_band.sum())})")
    assert not np.any(bad & ~in_band), (ids[bad & ~in_band][:10], margin[bad & ~in_band][:10])
    return int((code >= -1).sum()), [int((expect == q).sum()) for q in range(4)], int(in_band.sum())


def wall_margin_cells(p, r, z):
    """Distance (in cells) of positions to the nearest absorbing boundary."""
    return np.minimum.reduce([np.abs(z) / p.dz, np.abs(p.lz - z) / p.dz, np.abs(p.lr - r) / p.dr])


def check_wall_decisions(p, g, o, pre_ids, band=BAND_ULPS * POS_QUANTUM):
    """Particles of `pre_ids` (present before the step) alive after it on the
    GPU (g) and in the oracle (o): any particle alive on one side only must
    sit within `band` cells of an absorbing wall on the side that kept it.
    Returns the number of such cases."""
    ga = np.isin(pre_ids, g["id"])
    oa = np.isin(pre_ids, o["id"])
    only_g, only_o = pre_ids[ga & ~oa], pre_ids[oa & ~ga]
    n = 0
    for ids, side in ((only_g, g), (only_o, o)):
        if ids.size == 0:
            continue
        k = np.isin(side["id"], ids)
        m = wall_margin_cells(p, side["r"][k], side["z"][k])
        say(f"  wall decision on one side only: {ids.size}, margins (cells) {m[:8]}")
        assert (m <= band).all(), (ids[:10], m[:10])
        n += ids.size
    return n


def check_cells(p, g, o, band=BAND_ULPS * POS_QUANTUM):
    """Same cell for every particle of both (matched by id), except where
    the oracle's position lies within `band` cells of a cell face.  Returns
    the number of such cases."""
    gi, oi = np.argsort(g["id"]), np.argsort(o["id"])
    assert np.array_equal(g["id"][gi], o["id"][oi])
    xr, xz = o["r"][oi] / p.dr, o["z"][oi] / p.dz
    ci, cj = np.floor(xr).astype(np.int64), np.floor(xz).astype(np.int64)
    diff = (g["i"][gi] != ci) | (g["j"][gi] != cj)
    fr, fz = xr - np.floor(xr), xz - np.floor(xz)
    edge = np.minimum.reduce([fr, 1 - fr, fz, 1 - fz])
    if diff.any():
        say(f"  cells differ for {int(diff.sum())}, face distances {edge[diff][:8]}")
    assert (edge[diff] <= band).all(), (g["id"][gi][diff][:10], edge[diff][:10])
    return int(diff.sum())


def sample_oracle(p, br, bz, sig, sim, n_sample, seed, rtol=1e-11):
    """An oracle run holding a random sample of sim's current particles (up to
    n_sample per species), sim's potential and circuit state.  A particle's
    push, walls and collision depend only on its own state, its random stream
    and the fields, so the sample can be stepped alone and compared one by
    one (children, whose ids follow the global order, are left out)."""
    from oracle import oracle as O
    f = sim.fields_host()
    st = sim.get_state()
    rng = np.random.default_rng(seed)
    sample, ids = [], []
    for s in range(2):
        g = sim.particles(s)
        n = g["id"].shape[0]
        pick = np.sort(rng.choice(n, min(n, n_sample), replace=False))
        sample.append(to_species({k: g[k][pick] for k in ("r", "z", "vr", "vt", "vz", "id")}))
        ids.append(np.sort(g["id"][pick]))
    cap = tuple(max(2 * x.n, 1024) for x in sample)
    o = O.Oracle(p, br, bz, sig, sample, capacity=cap, rtol=rtol)
    o.init()
    o.phi[:] = f["phi"]
    o.phi0[:] = f["phi0"]
    o.set_state(step=st["step"], vc=st["vc"])
    o.state.qc = st["qc"]
    return o, ids


def check_sample(p, sim, o, ids, tol=1e-5):
    """After one step of both: the sampled particles of sim and the oracle
    agree one by one (positions to tol cells, velocities to tol of
    v_th + |v|); absorptions and cells agree except within the FP32 band of
    a wall or cell face.  Returns the number of band cases."""
    n_band = 0
    for s in range(2):
        g = sim.particles(s)
        keep = np.isin(g["id"], ids[s])
        g = {k: v[keep] for k, v in g.items()}
        r = o.particles(s)
        keep = np.isin(r["id"], ids[s])
        r = {k: v[keep] for k, v in r.items()}
        n_wall = check_wall_decisions(p, g, r, ids[s])
        both = np.intersect1d(g["id"], r["id"])
        g = {k: v[np.isin(g["id"], both)] for k, v in g.items()}
        r = {k: v[np.isin(r["id"], both)] for k, v in r.items()}
        ep, ev, only = compare_particles(p, g, r, s, tol)
        say("  species", s, "sample", len(ids[s]), "kept", g["id"].shape[0], "pos", ep, "vel", ev,
            "wall band", n_wall)
        assert only == 0 and ep < tol and ev < tol
        assert g["id"].shape[0] >= 0.98 * len(ids[s])
        n_cell = check_cells(p, g, r)
        n_band += n_wall + n_cell
    return n_band
