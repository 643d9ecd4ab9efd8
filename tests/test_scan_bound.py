"""CPU emulation of the lower-bound scan's float32 arithmetic (no GPU): the fine table (entries
L * delta^2 rounded toward zero), the coarse tables of the first pass (the minimum of the 64 fine
entries sharing a symbol's 2-bit prefix, 4 segments summed per table as ((a + b) + (c + d))), the
coarse bound ((t0 + t1) + (t2 + t3)) and the fine bound (16 terms in the kernel's tree). Both
must stay within (1 + gamma_15) of the float64 bound of the oracle, so that the scan's threshold
margin covers pruning on either, and the coarse bound must never exceed the float64 bound over
the cardinality-4 regions by more than that."""
import numpy as np

import synth
from oracle import isax, lb_table, lower_bound_sq, paa

G15 = 15 * 2.0 ** -24 / (1 - 15 * 2.0 ** -24)


def _round_toward_zero_f32(x):
    f = x.astype(np.float32)
    over = f.astype(np.float64) > x
    f[over] = np.nextafter(f[over], np.float32(0))
    return f


def _fine32(T8, S):
    t = T8[np.arange(16)[None, :], S]                     # [N][16] float32
    part = [(t[:, 4 * k] + t[:, 4 * k + 1]) + (t[:, 4 * k + 2] + t[:, 4 * k + 3]) for k in range(4)]
    return (part[0] + part[1]) + (part[2] + part[3])


def _coarse32(T8, S):
    t2 = T8.reshape(16, 4, 64).min(axis=2)                # float32
    c = (S >> 6).astype(np.int64)
    g = [(t2[4 * j][c[:, 4 * j]] + t2[4 * j + 1][c[:, 4 * j + 1]]) +
         (t2[4 * j + 2][c[:, 4 * j + 2]] + t2[4 * j + 3][c[:, 4 * j + 3]]) for j in range(4)]
    return (g[0] + g[1]) + (g[2] + g[3])


def test_two_pass_bound_within_the_margin():
    X = synth.random_walks(40000, 256, seed=71)
    S = isax(paa(X)).astype(np.int64)
    Qn, _, _ = synth.noisy_queries(X, 6, seed=72, sigma=(0.01, 0.8))
    Q = np.concatenate([Qn, synth.fresh_walk_queries(3, 256, seed=73)])
    for q in Q:
        qp = paa(q)
        T8 = _round_toward_zero_f32(lb_table(qp, 16))
        lb = lower_bound_sq(qp, S, 16)
        fine = _fine32(T8, S).astype(np.float64)
        coarse = _coarse32(T8, S).astype(np.float64)
        assert np.all(fine <= lb * (1 + G15) + 1e-30)
        assert np.all(coarse <= lb * (1 + G15) + 1e-30)
        # the coarse bound is the cardinality-4 bound (up to rounding): never above it by more
        t4 = lb_table(qp, 16, bits=2)
        lb4 = sum(t4[s][S[:, s] >> 6] for s in range(16))
        assert np.all(coarse <= lb4 * (1 + G15) + 1e-30)
        assert np.all(lb4 <= lb * (1 + 1e-12))
        # at any threshold, a series within it by a relative 1e-6 passes both bounds
        for thr in np.quantile(lb, [0.001, 0.05, 0.5]):
            keep = lb <= thr * (1 - 1e-6)
            assert np.all(coarse[keep] <= thr) and np.all(fine[keep] <= thr)
