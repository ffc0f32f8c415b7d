"""CPU checks of the learned-bound encoding (library host helpers)."""
import math
import os

import numpy as np
import pytest

A = pytest.importorskip("paper_2307_12276_amd")
if not os.path.exists(A.LIB_PATH):
    pytest.skip("libadl.so not built", allow_module_level=True)


def raw(kpar=1.0, kperp=1e-3, amax=0.2, h=1 / 256, dt=1e-4):
    return [math.log10(kpar), math.log10(0.7 * kpar), math.log10(kperp), math.log10(0.5 * kperp),
            amax, 0.5 * amax, math.log10(h), math.log10(h), math.log10(dt)]


def test_targets_decode_roundtrip():
    f = raw()
    for rho, m, K in [(1e6, 40, 1), (3.3e5, 95, 2), (2e4, 12, 4)]:
        g = 1.3 * rho
        y = A.learned_targets(f, g, rho, m, K)
        r, m2, K2 = A.learned_decode(f, g, y)
        assert r == pytest.approx(rho, rel=1e-6)
        assert K2 == K
        assert abs(m2 - m) <= 1


def test_features_are_dimensionless():
    """Scaling the grid spacing and the step together (same rho dt) leaves
    the inputs unchanged except the spacing-ratio entry stays zero."""
    g1 = 8 * 256 ** 2
    x1 = np.array(A.learned_features(raw(h=1 / 256, dt=1e-4), g1))
    x2 = np.array(A.learned_features(raw(h=1 / 512, dt=0.25e-4, amax=0.0), 4 * g1))
    x1b = np.array(A.learned_features(raw(h=1 / 256, dt=1e-4, amax=0.0), g1))
    assert np.allclose(x2, x1b, atol=1e-5)
    assert x1[5] == 0.0
    assert np.all(np.isfinite(x1))
