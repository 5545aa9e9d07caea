"""Pins for the oracle's Philox4x32-10 generator.

* known-answer vectors published with the generator (tests/golden);
* rocRAND's independent implementation, on a grid of counters and keys;
* uniformity of the 24-bit uniforms (chi-square).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(O.philox(ctr, key)) == out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand(tmp_path):
    exe = tmp_path / "rr"
    subprocess.check_call(["hipcc", "-O1", "-o", str(exe),
                           os.path.join(HERE, "rocrand_philox_ref.cpp")])
    rng = np.random.default_rng(5)
    lines, cases = [], []
    for _ in range(200):
        c = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
             int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        k = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        cases.append((c, k))
        lines.append(" ".join("%08x" % v for v in c + k))
    out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for (c, k), line in zip(cases, out):
        ref = [int(x, 16) for x in line.split()]
        assert list(O.philox(c, k)) == ref


def test_uniformity_chi2():
    # u24 of each output word over consecutive ids at a fixed step: 64 bins
    n = 20000
    vals = np.array([O.philox([i, 0x10, 7, 0], [0x12345678, 0x9abcdef0]) for i in range(n)])
    u = (vals >> 8).astype(np.float64) / 2**24
    for w in range(4):
        h, _ = np.histogram(u[:, w], bins=64, range=(0, 1))
        e = n / 64
        chi2 = ((h - e) ** 2 / e).sum()
        # 63 dof: mean 63, sd ~11.2; 5 sigma band
        assert chi2 < 63 + 5 * 11.3
