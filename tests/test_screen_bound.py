"""The batched screen's accumulator brackets the squared distance.

CPU emulation of the screen's arithmetic for one (query, series) pair: operands rounded to
bfloat16 (nearest even), their products exact in float32, the folded constants a_q and b_x
entering as directed-rounded bfloat16 pairs through the bias k-step, everything summed in
float32 in random orders and as a pairwise tree (the matrix cores' order is not specified, so
the bound must hold for any). With P = 1 every pair satisfies

    U - 2A <= d^2 <= U - 2A + 2c (qn + xn),

and with the projected screen (segment means over P points, threshold U / P) P (U/P - 2A) <= d^2.
The screen keeps a pair iff A >= 0; the batched re-score skips a candidate when the left side,
from the accumulator truncated to 16 bits, exceeds an upper bound on the nearest distance
(the right side for another survivor, or a computed distance). Adversarial pairs: the query
equal to the series, near duplicates, thresholds at the tiny floor and far above the distance.
"""
import numpy as np
import pytest

import synth

U24 = 2.0 ** -24
U23 = 2.0 ** -23
UB = 2.0 ** -8


def _gam(k, u):
    return k * u / (1.0 - k * u)


def _margin(nd, np_):
    """The screen's relative error budget c for nd screened points padded to np_."""
    c = (2 * UB + UB * UB) + 6 * _gam(np_ + 48, U23) * (1 + UB) ** 2 + 2 * _gam(nd, U24) + 16 * U24
    return float(np.float32(1.05 * c + 32 * U24))


def _bf16_rne(v):
    b = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _bf16_dir(t, up):
    """bfloat16 of float32 t rounded toward +inf (up) or -inf."""
    b = int(np.float32(t).view(np.uint32))
    h = b >> 16
    neg = b >> 31
    if b & 0xFFFF and (neg == (0 if up else 1)):
        h += 1
    return np.uint32(h << 16).view(np.float32)


def _bias_pair(t):
    t = np.float32(t)
    hi = _bf16_dir(t, up=False)
    rem = np.float32(t - hi)          # exact
    lo = _bf16_dir(rem, up=True)
    assert float(hi) + float(lo) >= float(t)
    return hi, lo


def _rd32(x):
    f = np.float32(x)
    return f if float(f) <= x else np.nextafter(f, np.float32(-np.inf))


def _proj(v, P):
    if P == 1:
        return v.astype(np.float32)
    return (v.astype(np.float64).reshape(-1, P).sum(1) / P).astype(np.float32)


def _sum32_seq(terms):
    return np.cumsum(terms.astype(np.float32), dtype=np.float32)[-1]


def _sum32_tree(terms):
    t = terms.astype(np.float32)
    while t.size > 1:
        if t.size % 2:
            t = np.append(t, np.float32(0))
        t = (t[0::2] + t[1::2]).astype(np.float32)
    return t[0]


def _accumulators(q, x, U, P, np_, rng, orders=4):
    """(A for several summation orders, qn, xn, U/P) as the screen forms them."""
    vq, vx = _proj(q, P), _proj(x, P)
    nd = vq.size
    c = _margin(nd, np_)
    qn = _sum32_seq(rng.permutation((vq * vq).astype(np.float32)))
    xn = _sum32_seq(rng.permutation((vx * vx).astype(np.float32)))
    Up = U if P == 1 else U / P * (1.0 + 2.0 ** -50)
    a = _rd32(((1.0 - c) * float(qn) - Up) * 0.5)
    b = _rd32((1.0 - c) * float(xn) * 0.5)
    hq, lq = _bias_pair(-a)
    hx, lx = _bias_pair(-b)
    prods = (_bf16_rne(vq).astype(np.float64) * _bf16_rne(vx).astype(np.float64)).astype(np.float32)
    assert np.array_equal(prods.astype(np.float64), _bf16_rne(vq).astype(np.float64) * _bf16_rne(vx))
    terms = np.concatenate([prods, np.zeros(np_ - nd, np.float32), np.array([hq, lq, hx, lx], np.float32)])
    accs = [_sum32_tree(terms)]
    for _ in range(orders):
        accs.append(_sum32_seq(rng.permutation(terms)))
    return accs, float(qn), float(xn), Up, c


def _cases(n, rng):
    X = synth.random_walks(300, n, seed=5)
    Q, src, _ = synth.noisy_queries(X, 60, seed=6, sigma=(0.0, 0.5))
    out = []
    for m in range(Q.shape[0]):
        q = Q[m]
        d_src = float(np.sum((q.astype(np.float64) - X[src[m]]) ** 2))
        out.append((q, X[src[m]], d_src))                              # the nearest, usually
        out.append((q, X[rng.integers(0, X.shape[0])], d_src))         # another series
    for i in range(10):
        x = X[i]
        out.append((x.copy(), x, 1e-20))                               # d = 0, U at its floor
        y = x.copy()
        y[rng.integers(0, n)] = np.nextafter(y[rng.integers(0, n)], np.float32(9))
        out.append((y, x, 1e-20))                                      # near duplicate
        out.append((x, X[i + 1], 1e3))                                 # threshold far above
    return out


@pytest.mark.parametrize("n,P,np_", [(256, 1, 256), (128, 1, 128), (512, 1, 512),
                                     (1024, 2, 512), (2048, 4, 512)])
def test_screen_accumulator_brackets_the_distance(n, P, np_):
    rng = np.random.default_rng(n + P)
    seed_rel = 3.0 * _gam(n + 2, U24) + 2.0 ** -30
    worst_lo = worst_hi = -np.inf
    for q, x, d_seed in _cases(n, rng):
        U = d_seed * (1.0 + seed_rel) + 1e-20
        d2 = float(np.sum((q.astype(np.float64) - x.astype(np.float64)) ** 2))
        accs, qn, xn, Up, c = _accumulators(q, x, U, P, np_, rng)
        u_lo = float(_rd32(Up))
        for A in accs:
            A = float(A)
            # lower side (the screen's pruning and the re-score's skip), from the truncated copy
            at = float(np.uint32(np.float32(A).view(np.uint32) & 0xFFFF0000).view(np.float32))
            a_hi = at * (1.0 + 2.0 ** -7) if at > 0 else at
            assert A <= a_hi
            lb = P * (u_lo - 2.0 * a_hi) * (1.0 - 2.0 ** -40)
            assert lb <= d2 * (1 + 1e-12) + 1e-12, (n, P, lb, d2)
            assert P * (Up - 2.0 * A) <= d2 * (1 + 1e-12) + 1e-12
            worst_lo = max(worst_lo, P * (Up - 2.0 * A) - d2)
            if P == 1:
                # upper side (the certified bound on the nearest distance)
                ub = (U - 2.0 * A + 2.0 * c * (qn + xn)) * (1.0 + 2.0 ** -40)
                assert d2 <= ub, (n, d2, ub)
                worst_hi = max(worst_hi, d2 - (U - 2.0 * A))
    assert worst_lo <= 0.0
