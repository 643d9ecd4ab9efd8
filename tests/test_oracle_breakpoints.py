"""Pins for the oracle's Gaussian breakpoints (Section 2.2 regions; equiprobable N(0,1) reading)."""
import math

import numpy as np
import pytest

from oracle import breakpoints, breakpoints_at_cardinality

UPPER_QUARTILE = 0.6744897501960817  # Phi^{-1}(3/4), standard normal tables (0.67448975019608...)


def test_ends_and_centre():
    b = breakpoints()
    assert b.shape == (257,)
    assert b[0] == -np.inf and b[256] == np.inf
    assert b[128] == 0.0
    assert np.all(np.diff(b[1:256]) > 0)


def test_symmetry_exact():
    b = breakpoints()
    for k in range(1, 256):
        assert b[256 - k] == -b[k]


def test_quartiles():
    b = breakpoints()
    assert b[192] == UPPER_QUARTILE
    assert b[64] == -UPPER_QUARTILE


def test_against_scipy_quantile():
    from scipy.stats import norm
    b = breakpoints()
    ref = norm.ppf(np.arange(1, 256) / 256.0)
    ulp = np.spacing(np.abs(ref))
    ulp[ref == 0] = 5e-324
    assert np.all(np.abs(b[1:256] - ref) <= 2 * ulp)


def test_correctly_rounded_by_root_finding():
    """Independent route: solve Phi(z) = k/256 with a root finder on the normal CDF at 50 digits,
    then check the table entry is the float64 nearest to that root."""
    import mpmath
    ctx = mpmath.mp.clone()
    ctx.dps = 50
    b = breakpoints()
    for k in list(range(1, 256, 7)) + [1, 2, 127, 129, 254, 255]:
        p = ctx.mpf(k) / 256
        z = ctx.findroot(lambda t: ctx.ncdf(t) - p, ctx.mpf(float(b[k])))
        v = float(b[k])
        for nb in (math.nextafter(v, math.inf), math.nextafter(v, -math.inf)):
            assert abs(ctx.mpf(v) - z) <= abs(ctx.mpf(nb) - z)


@pytest.mark.parametrize("bits", [1, 2, 3, 5, 8])
def test_lower_cardinality_is_subset(bits):
    b = breakpoints()
    bb = breakpoints_at_cardinality(bits)
    assert bb.shape == ((1 << bits) + 1,)
    step = 1 << (8 - bits)
    assert np.array_equal(bb, b[::step])


def test_cardinality_four():
    bb = breakpoints_at_cardinality(2)
    assert list(bb[1:4]) == [-UPPER_QUARTILE, 0.0, UPPER_QUARTILE]
