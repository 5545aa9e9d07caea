"""Bit-reproducible runs and checkpoint/resume on the GPU.

With the fixed-point deposit (deposit_fixed = 1, FP64 state) the node charge
is an integer sum of rounded tent weights and the cathode charge is formed
from integer tallies, so no step result depends on the order in which the
GPU's threads happen to add.  Two runs from the same inputs are then
bit-identical, and a run stopped after N steps, checkpointed (scalar state,
particle arrays, phi0 and its predecessor) and resumed in a fresh handle
reaches the same bits after 2N steps as the uninterrupted run.  The
fixed-point deposit itself is checked against the oracle like the floating
one (FP64 tolerance 1e-12)."""
import numpy as np
import pytest

from gpu_helpers import compare_particles, gpu_sim, say
from oracle import oracle as O
from paper_2507_10727_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(scheme, n=40000):
    # every process of the step active: collisions including the metastable
    # channel, ion- and electron-induced emission, the resistor circuit
    p = W.scaled(W.preset("small_mc64_f64"), n)
    return p.replace(scheme=scheme, deposit_fixed=1, circuit=W.RESISTOR, v_ext=-400.0,
                     r_ext=100.0, gamma_i=0.2, gamma_e=0.1, n_meta=2.5e17, sort_every=20,
                     poisson_rtol=1e-13)


def _snapshot(sim):
    out = {"state": sim.get_state()}
    for s in range(2):
        d = sim.particles(s)
        o = np.argsort(d["id"], kind="stable")
        out[s] = {k: d[k][o] for k in ("id", "key", "fr", "fz", "vr", "vt", "vz")}
    f = sim.fields_host()
    for k in ("phi", "phi0", "phi0_prev", "q_e", "q_i"):
        out[k] = f[k]
    return out


def _assert_same_bits(a, b, what):
    sa, sb = a["state"], b["state"]
    for k in ("step", "vc", "qc", "next_id"):
        assert sa[k] == sb[k], (what, k, sa[k], sb[k])
    for s in range(2):
        assert a[s]["id"].shape == b[s]["id"].shape, (what, s)
        for k, v in a[s].items():
            assert np.array_equal(v.view(np.uint8), b[s][k].view(np.uint8)), (what, s, k)
    for k in ("phi", "phi0", "phi0_prev", "q_e", "q_i"):
        assert np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)), (what, k)


@pytest.mark.parametrize("scheme", [W.MC_PIC, W.EC_PIC])
def test_fixed_deposit_matches_oracle(scheme):
    """Ten steps with the fixed-point deposit against the oracle: particles,
    potential and node charge to 1e-12 (the weights are rounded to 2^-42,
    well inside it), every decision identical."""
    p = _problem(scheme, 20000)
    br, bz, sig, parts = W.inputs(p)
    say("case fixed-point deposit against the oracle", p.name, "scheme", scheme)
    sim = gpu_sim(p, br, bz, sig, [x.copy() for x in parts])
    o = O.Oracle(p, br, bz, sig, [x.copy() for x in parts])
    o.init()
    for k in range(1, 11):
        sim.step(1)
        d_o = o.step()
        d_g = sim.diag()
        for key in ("n_coll", "n_cand", "n_see", "n_see_e", "n_abs"):
            assert np.array_equal(np.array(d_g[key]), np.array(d_o[key])), (k, key)
        assert abs(d_g["dq_conv"] - d_o["dq_conv"]) <= 1e-12 * max(abs(d_o["dq_conv"]), 1e-30)
    for s in range(2):
        ep, ev, only = compare_particles(p, sim.particles(s), o.particles(s), s, 1e-12)
        say("  species", s, "pos", ep, "vel", ev)
        assert ep < 2e-12 and ev < 2e-12 and only == 0
    f = sim.fields_host()
    ephi = np.abs(f["phi"] - o.phi).max() / np.abs(o.phi).max()
    eq = max(np.abs(f["q_e"] - o.q[0]).max() / np.abs(o.q[0]).max(),
             np.abs(f["q_i"] - o.q[1]).max() / np.abs(o.q[1]).max())
    say("  phi", ephi, "q", eq)
    assert ephi < 2e-12 and eq < 1e-12
    st = sim.get_state()
    assert st["next_id"] == (o.state.next_id[0], o.state.next_id[1])
    assert abs(st["vc"] - o.state.vc) <= 1e-12 * abs(o.state.vc)
    sim.close()


@pytest.mark.parametrize("scheme", [W.MC_PIC, W.EC_PIC])
def test_fixed_deposit_runs_bit_identical(scheme):
    """Two runs of the same inputs, 60 steps (three cell sorts), agree bit
    for bit: particles by id, potential, node charge, circuit state."""
    p = _problem(scheme)
    br, bz, sig, parts = W.inputs(p)
    say("case two runs bit-identical", p.name, "scheme", scheme)
    snaps = []
    for r in range(2):
        sim = gpu_sim(p, br, bz, sig, [x.copy() for x in parts])
        sim.step(60)
        snaps.append(_snapshot(sim))
        sim.close()
    say("  counts", snaps[0]["state"]["count"], "vc", snaps[0]["state"]["vc"])
    _assert_same_bits(snaps[0], snaps[1], "second run")


@pytest.mark.parametrize("scheme", [W.MC_PIC, W.EC_PIC])
def test_resume_bit_exact(scheme):
    """Run 2N = 70 steps; separately run N = 35, checkpoint, resume in a fresh
    handle (created without particles) and run N more.  The two end states
    agree bit for bit.  N is not a multiple of the sort interval, so the
    resumed run must also take over the sort phase."""
    p = _problem(scheme)
    br, bz, sig, parts = W.inputs(p)
    n = 35
    say("case resume bit-exact", p.name, "scheme", scheme, "N", n)
    cap = (4 * p.n_per_species, 4 * p.n_per_species)
    a = gpu_sim(p, br, bz, sig, [x.copy() for x in parts], capacity=cap)
    a.step(2 * n)
    ref = _snapshot(a)
    a.close()

    b = gpu_sim(p, br, bz, sig, [x.copy() for x in parts], capacity=cap)
    b.step(n)
    ck = b.checkpoint()
    assert ck["state"]["sort_phase"] == n % p.sort_every
    b.close()

    c = gpu_sim(p, br, bz, sig, None, capacity=cap)
    c.restore(ck)
    st = c.get_state()
    assert st["step"] == n and st["sort_phase"] == n % p.sort_every
    c.step(n)
    got = _snapshot(c)
    c.close()
    say("  counts", got["state"]["count"], "vc", got["state"]["vc"])
    _assert_same_bits(ref, got, "resumed run")


def test_autotune_leaves_the_run_where_it_was():
    """pic_autotune steps the live simulation through its trials (nine
    shapes, two steps each) and then puts the state back: the state right
    after the call equals the state before it, and 30 further steps reach
    the same bits as a run that was never tuned (the fixed-point deposit
    makes the launch shape irrelevant to the result)."""
    p = _problem(W.EC_PIC)
    br, bz, sig, parts = W.inputs(p)
    say("case autotune restores the state", p.name)
    a = gpu_sim(p, br, bz, sig, [x.copy() for x in parts])
    a.step(25)
    before = _snapshot(a)
    t = a.autotune(steps_per_trial=2)
    say("  tuning", t)
    after = _snapshot(a)
    _assert_same_bits(before, after, "right after autotune")
    a.step(30)
    tuned = _snapshot(a)
    a.close()
    b = gpu_sim(p, br, bz, sig, [x.copy() for x in parts])
    b.step(55)
    ref = _snapshot(b)
    b.close()
    _assert_same_bits(ref, tuned, "tuned run")
