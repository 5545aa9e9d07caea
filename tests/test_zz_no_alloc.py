"""pic_poisson_static: the direct field solve with the library's static
scratch (no device allocation) against pic_poisson on the same handle.

Two calls in a row share the GPU's scratch array, the second on a smaller
grid (its transform buffers then hold the first call's values beyond its
own extent); each must equal pic_poisson's solution to the FP64 bar
(1e-12 of the largest potential; the two run the same kernels on the same
inputs, so they normally agree bit for bit), and its residual, recomputed
with the oracle's operator, must meet the solve tolerance.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_sim, say
from oracle import oracle as O
from paper_2507_10727_amd import _lib as L
from paper_2507_10727_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(nr, nz, mode=W.POISSON_DIRECT):
    p = W.Problem(name="static", nr=nr, nz=nz, lr=nr * 1.5625e-4, lz=nz * 1.5625e-4,
                  n_per_species=0, poisson_mode=mode, poisson_rtol=1e-11)
    br, bz, sig, _ = W.inputs(p, n=0)
    sim = gpu_sim(p, br, bz, sig, None, capacity=(1024, 1024))
    o = O.Oracle(p, br, bz, sig, None, capacity=(16, 16))
    return p, sim, o


def _charge(p, seed):
    rng = np.random.default_rng(seed)
    r = (np.arange(p.nr + 1) * p.dr)[None, :]
    z = (np.arange(p.nz + 1) * p.dz)[:, None]
    smooth = np.exp(-((r - 0.3 * p.lr) / (0.25 * p.lr)) ** 2 - ((z - 0.6 * p.lz) / (0.3 * p.lz)) ** 2)
    return (smooth + 0.2 * rng.normal(size=smooth.shape)).ravel() * 1e-12


def test_static_scratch_solve_equals_pic_poisson():
    import torch
    for (nr, nz), vcat, seed in (((256, 512), -500.0, 1), ((60, 90), -300.0, 2)):
        p, sim, o = _setup(nr, nz)
        say("case static-scratch solve", nr, nz, vcat)
        q = torch.tensor(_charge(p, seed), dtype=torch.float64, device="cuda")
        phi_a = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
        st_a = sim.poisson(q, vcat, phi_a)
        phi_b = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
        status, st_b = sim.poisson_static(q, vcat, phi_b)
        say("  pic_poisson", st_a, "\n  pic_poisson_static", status, st_b)
        assert status == L.PIC_OK and st_b["converged"] == 1 and st_b["rel_res"] <= 1e-11
        a, b = phi_a.cpu().numpy(), phi_b.cpu().numpy()
        d = np.abs(a - b).max() / np.abs(a).max()
        say(f"  max |static - pic_poisson| / max |phi| = {d:.3e}, identical: {np.array_equal(a, b)}")
        assert d <= 1e-12
        kind = o.node_kind()
        unk = kind == 0
        qh = q.cpu().numpy()
        r = (qh - o.apply_k(b))[unk]
        rhs = (qh - o.apply_k(np.where(unk, 0.0, b)))[unk]
        assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(rhs)
        sim.close()


def test_static_scratch_rejects_other_modes_and_large_grids():
    import torch
    p, sim, _ = _setup(32, 32, mode=W.POISSON_MGCG)
    q = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
    phi = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
    status, _ = sim.poisson_static(q, 0.0, phi)
    assert status == L.PIC_ESTATE
    sim.close()
    # 1024 x 2048 cells: 2.1e6 nodes + 2 x 2048 x 1024 transform doubles
    # exceed the 32 MiB array
    p, sim, _ = _setup(1024, 2048)
    q = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
    phi = torch.zeros(p.nodes, dtype=torch.float64, device="cuda")
    status, _ = sim.poisson_static(q, 0.0, phi)
    assert status == L.PIC_EINVAL
    assert b"scratch" in sim.lib.pic_last_error(sim.h)
    sim.close()
