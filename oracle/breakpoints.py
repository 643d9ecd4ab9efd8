"""Gaussian breakpoints for the iSAX alphabet (oracle side; test infrastructure only).

Section 2.2 ("iSAX Representation") divides the value axis into regions, one symbol per region,
with 256 symbols (8 bits) as the maximum cardinality. The region boundaries are not printed in
the paper; the iSAX convention it cites makes the regions equiprobable under N(0,1). Reading:
``beta_k = Phi^{-1}(k / 256)`` for ``k = 1..255``, ``beta_0 = -inf``, ``beta_256 = +inf``.

Computed here with mpmath's inverse error function at 60 significant digits and rounded to the
nearest float64 (``Phi^{-1}(p) = sqrt(2) * erfinv(2p - 1)``). The tests pin the table against
scipy's quantile function, against an independent root-finding of mpmath's normal CDF, and
against the closed forms ``beta_128 = 0``, ``beta_{256-k} = -beta_k`` and the upper quartile.
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=None)
def _table8() -> np.ndarray:
    import mpmath

    ctx = mpmath.mp.clone()
    ctx.dps = 60
    out = np.empty(257, dtype=np.float64)
    out[0] = -np.inf
    out[256] = np.inf
    for k in range(1, 256):
        z = ctx.sqrt(2) * ctx.erfinv(ctx.mpf(2 * k) / 256 - 1)
        out[k] = float(z)  # mpmath rounds to nearest on conversion
    out.setflags(write=False)
    return out


def breakpoints() -> np.ndarray:
    """float64[257]: beta_0 = -inf, beta_1..beta_255, beta_256 = +inf (8-bit alphabet)."""
    return _table8()


def breakpoints_at_cardinality(bits: int) -> np.ndarray:
    """float64[2^bits + 1] boundaries of the 2^bits-symbol alphabet.

    The 2^b-level boundaries are the subset ``beta_{k * 2^(8-b)}`` of the 8-bit ones (both are
    quantiles at multiples of 1/2^b), which is what makes a lower-cardinality symbol a bit prefix
    of the 8-bit symbol (Section 2.2, variable cardinalities in the ADS+ index).
    """
    if not 1 <= bits <= 8:
        raise ValueError("bits must be in 1..8")
    step = 1 << (8 - bits)
    return np.ascontiguousarray(_table8()[::step])
