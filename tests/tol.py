"""Relative comparison without pytest.approx's default absolute tolerance
(1e-12), which would swallow the small SI magnitudes of this code (charges
of 1e-9 C, energies of 1e-8 J, areas of 1e-3 m^2)."""
import pytest


def approx(expected, rel=1e-12, abs=0.0):
    return pytest.approx(expected, rel=rel, abs=abs)
