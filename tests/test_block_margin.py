"""The block bound's float32 evaluation never drops a pair whose exact bound is within its
threshold (CPU emulation of the kernel's arithmetic: numpy float32 operations round to nearest
like the GPU's; the fused square-add is emulated by an exact float64 product and sum rounded
once to float32). Adversarial cases: query means on region edges, inside, far outside, large
and tiny magnitudes, thresholds equal to the exact bound."""
import numpy as np

from oracle.breakpoints import breakpoints

U32 = 2.0 ** -24


def _down(x):
    f = np.float32(x)
    return f if float(f) <= x else np.nextafter(f, np.float32(-np.inf))


def _up(x):
    f = np.float32(x)
    return f if float(f) >= x else np.nextafter(f, np.float32(np.inf))


def _kernel_bound(p, lo, hi, L):
    acc = np.float32(0.0)
    pf = [np.float32(v) for v in p]
    for s in range(16):
        g = max(max(np.float32(_down(lo[s]) - pf[s]), np.float32(pf[s] - _up(hi[s]))), np.float32(0.0))
        acc = np.float32(float(g) * float(g) + float(acc))
    return float(np.float32(acc * np.float32(L)))


def _kernel_threshold(V, p, L):
    A = float(np.sum(np.asarray(p, np.float64) ** 2)) * L
    r = np.sqrt(V) * (1 + 2 * U32) + U32 * np.sqrt(A) * (1 + 2 * U32)
    return float(_up((1 + 24 * U32) * r * r * (1 + 4 * U32)))


def _exact_bound(p, lo, hi, L):
    g = np.maximum(np.maximum(lo - p, p - hi), 0.0)
    return L * float(np.sum(g * g))


def test_float32_block_bound_never_drops_a_pair_within_its_threshold():
    b = breakpoints()
    rng = np.random.default_rng(11)
    worst = 0.0
    for trial in range(4000):
        L = int(rng.choice([1, 4, 16, 17, 64]))
        mn = rng.integers(0, 256, 16)
        mx = np.minimum(255, mn + rng.integers(0, 40, 16))
        lo, hi = b[mn], b[mx + 1]
        kind = trial % 4
        if kind == 0:     # on the edges
            p = np.where(rng.random(16) < 0.5, lo, hi)
            p = np.where(np.isfinite(p), p, 0.0)
        elif kind == 1:   # just outside the edges
            p = np.where(rng.random(16) < 0.5, lo - 1e-7 * rng.random(16), hi + 1e-7 * rng.random(16))
            p = np.where(np.isfinite(p), p, 1.0)
        elif kind == 2:   # anywhere, moderate
            p = rng.standard_normal(16) * 2.0
        else:             # large magnitudes
            p = rng.standard_normal(16) * 50.0
        B = _exact_bound(p, lo, hi, L)
        for V in (B, B * (1 + 1e-12), B + 1e-30):
            T = _kernel_threshold(V, p, L)
            Bk = _kernel_bound(p, lo, hi, L)
            assert Bk <= T, (trial, kind, L, B, V, Bk, T)
            if B >= 1.0 and kind != 3:
                worst = max(worst, (T - B) / B)
    # for thresholds of ordinary size the inflation is tiny
    assert worst < 1e-4


def test_float32_block_bound_still_prunes():
    """A pair whose exact bound clearly exceeds the threshold is dropped (the margin is not vacuous)."""
    b = breakpoints()
    lo = b[np.full(16, 200)]
    hi = b[np.full(16, 210)]
    p = np.zeros(16)
    L = 16
    B = _exact_bound(p, lo, hi, L)
    assert _kernel_bound(p, lo, hi, L) > _kernel_threshold(B * 0.999, p, L)
