"""Synthetic inputs: the clustered load of the high-density discharge."""
import numpy as np

from paper_2507_10727_amd import workloads as W


def test_clustered_load_fills_the_ring():
    p = W.preset("ec512x1024_clustered_f32").replace(n_per_species=100_000)
    assert p.cluster == 0.5
    for sp in W.load_uniform(p):
        ring = (sp.r > 0.35 * p.lr) & (sp.r < 0.5 * p.lr) & (sp.z < 0.1 * p.lz)
        # half loaded in the ring, plus the uniform half's share of it
        share = (0.5 ** 2 - 0.35 ** 2) * 0.1
        assert abs(ring.mean() - (0.5 + 0.5 * share)) < 0.01
        assert np.all(ring[:50_000])
        assert sp.r.max() < p.lr and sp.z.max() < p.lz and sp.r.min() >= 0
        assert np.unique(sp.id).size == sp.n
    # per-cell load in the ring: about 3e3 per species at full size
    full = W.preset("ec512x1024_clustered_f32")
    cells = (0.5 - 0.35) * full.nr * 0.1 * full.nz
    assert 2e3 < 0.5 * full.n_per_species / cells < 5e3


def test_uniform_presets_have_no_cluster():
    for name in ("small_mc64_f64", "ec256x512_f32", "ec512x1024_f32", "mc512x1024_f32"):
        assert W.preset(name).cluster == 0.0
