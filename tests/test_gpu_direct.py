"""The direct sine-transform field solve (PIC_DIRECT) against the oracle.

The solve (sine transform over z as FP64 matrix products, one tridiagonal
system in r per sine mode) must reproduce the oracle's field equation to
FP64 round-off: its residual, recomputed with the oracle's own operator, is
checked at 1e-11 (a direct solve from phi = 0 leaves a forward error of a
few units of FP64 round-off in every mode, so its residual relative to
||b|| grows with the operator's condition number, measured 4e-10 at 256x512
for a charge without Dirichlet drive; the solve corrects from the residual
of its current potential, and a second correction reaches the FP64 floor),
and on grids the oracle solves in seconds the potentials are compared node
by node to 1e-9.  Grids include sizes that are not multiples of
the 32-row / 32-column tiles (ragged tails) and a single tile.
"""
import numpy as np
import pytest

from gpu_helpers import compare_particles, gpu_sim, say
from oracle import oracle as O
from paper_2507_10727_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(nr, nz, **kw):
    base = dict(name="direct", nr=nr, nz=nz, lr=nr * 1.5625e-4, lz=nz * 1.5625e-4,
                n_per_species=0, poisson_mode=W.POISSON_DIRECT, poisson_rtol=1e-11)
    base.update(kw)
    return W.Problem(**base)


def _charge(p, kind, rng):
    r = (np.arange(p.nr + 1) * p.dr)[None, :]
    z = (np.arange(p.nz + 1) * p.dz)[:, None]
    smooth = np.exp(-((r - 0.4 * p.lr) / (0.2 * p.lr)) ** 2 - ((z - 0.3 * p.lz) / (0.2 * p.lz)) ** 2)
    q = (smooth + 0.3 * rng.normal(size=smooth.shape)).ravel() * 1e-12
    return q


@pytest.mark.parametrize("nr,nz", [(2, 2), (5, 3), (37, 53), (32, 33), (100, 60), (256, 512),
                                   (512, 1024)])
def test_direct_solve_matches_oracle(nr, nz):
    import torch
    p = _problem(nr, nz)
    br, bz, sig, _ = W.inputs(p, n=0)
    say("case direct solve", nr, nz)
    sim = gpu_sim(p, br, bz, sig, None, capacity=(1024, 1024))
    o = O.Oracle(p, br, bz, sig, None, capacity=(16, 16))
    kind = o.node_kind()
    rng = np.random.default_rng(nr * 1000 + nz)
    q = _charge(p, kind, rng)
    for vcat in (-500.0, 0.0, 1.0):
        phi = torch.full((p.nodes,), 7.0, dtype=torch.float64, device="cuda")
        st = sim.poisson(torch.tensor(q, dtype=torch.float64, device="cuda"), vcat, phi)
        g = phi.cpu().numpy()
        assert np.all(g[kind == 1] == vcat) and np.all(g[kind == 2] == 0.0)
        unk = kind == 0
        r = (q - o.apply_k(g))[unk]
        b = (q - o.apply_k(np.where(unk, 0.0, g)))[unk]
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        say(f"  v_cathode {vcat}: stats {st}, residual with the oracle's operator {rel:.3e}")
        assert st["converged"] == 1 and st["rel_res"] <= 1e-11 and st["iterations"] == 0
        assert rel <= 1e-11
        if p.nodes <= 140_000:
            ref, rc, it, res = o.solve(q, vcat, rtol=1e-12)
            scale = np.abs(ref).max()
            d = np.abs(g - ref).max() / scale
            say(f"  max |phi - oracle| / max |phi| = {d:.3e} (oracle residual {res:.1e})")
            assert d <= 1e-9
    sim.close()


def test_direct_rejects_neumann_block():
    from paper_2507_10727_amd import _lib as L
    p = _problem(64, 64)
    p = p.replace(cathode_rmax=0.85 * p.lr)
    br, bz, sig, _ = W.inputs(p, n=0)
    with pytest.raises(L.PicError) as e:
        gpu_sim(p, br, bz, sig, None, capacity=(1024, 1024))
    assert e.value.status == L.PIC_EINVAL


@pytest.mark.parametrize("scheme", [W.MC_PIC, W.EC_PIC])
def test_f64_steps_direct(scheme):
    """The small configuration (64x64, FP64, 2e4 + 2e4 particles) stepped
    with the direct solve against the oracle: every 5 steps for 20 steps,
    identical decisions, and positions and velocities within 2e-13 per step
    (the oracle solves to a 1e-13 residual, so each step's fields differ by
    that order and the particles' differences grow with the step count, as
    in the 200-step comparison)."""
    p = W.scaled(W.preset("small_mc64_f64"), 20000).replace(
        scheme=scheme, poisson_mode=W.POISSON_DIRECT, poisson_rtol=1e-11)
    br, bz, sig, parts = W.inputs(p)
    say("case f64 direct steps", scheme)
    sim = gpu_sim(p, br, bz, sig, [x.copy() for x in parts])
    o = O.Oracle(p, br, bz, sig, [x.copy() for x in parts])
    o.init()
    for k in range(1, 21):
        sim.step(1)
        d_o = o.step()
        if k % 5:
            continue
        d_g = sim.diag()
        for s in range(2):
            ep, ev, only = compare_particles(p, sim.particles(s), o.particles(s), s, 1e-12)
            say(f"  step {k} species {s}: pos {ep:.2e} vel {ev:.2e}")
            assert ep < 2e-13 * k and ev < 2e-13 * k and only == 0
        f = sim.fields_host()
        ephi = np.abs(f["phi"] - o.phi).max() / np.abs(o.phi).max()
        say(f"  step {k}: phi {ephi:.2e}, solve {d_g['poisson']}")
        assert ephi < max(1e-12, 2e-13 * k)
        assert d_g["poisson"]["converged"] == 1 and d_g["poisson"]["rel_res"] <= 1e-11
        assert d_g["n_coll"] == d_o["n_coll"] and d_g["n_see"] == d_o["n_see"]
        assert abs(d_g["vc"] - o.state.vc) <= 1e-12 * abs(o.state.vc)
    sim.close()
