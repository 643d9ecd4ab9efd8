"""CPU emulation of the lower-bound scan's float32 arithmetic (no GPU): the fine table (entries
L * delta^2 rounded toward zero), the fine bound (16 terms in the kernel's summation tree) and
the bound of a run of consecutive leaf-order series taken from the run's symbol envelope (per
segment, the table entry at the query's symbol clamped into the run's [min, max] symbol range,
summed in the same tree). The fine bound must stay within (1 + gamma_15) of the oracle's float64
bound, so that the scan's threshold margin covers it; the run bound must never exceed the fine
bound of any member in float32, so that pruning a run drops no series the fine bound keeps."""
import numpy as np

import synth
from oracle import isax, lb_table, lower_bound_sq, paa
from oracle.reference import sorted_order

G15 = 15 * 2.0 ** -24 / (1 - 15 * 2.0 ** -24)
RUN = 32


def _round_toward_zero_f32(x):
    f = x.astype(np.float32)
    over = f.astype(np.float64) > x
    f[over] = np.nextafter(f[over], np.float32(0))
    return f


def _tree(t):
    part = [(t[:, 4 * k] + t[:, 4 * k + 1]) + (t[:, 4 * k + 2] + t[:, 4 * k + 3]) for k in range(4)]
    return (part[0] + part[1]) + (part[2] + part[3])


def _fine32(T8, S):
    return _tree(T8[np.arange(16)[None, :], S])          # [N] float32


def _run32(T8, S, qsym):
    n = S.shape[0]
    runs = (n + RUN - 1) // RUN
    pad = np.concatenate([S, np.repeat(S[-1:], runs * RUN - n, axis=0)]).reshape(runs, RUN, 16)
    lo, hi = pad.min(axis=1), pad.max(axis=1)             # the tail run's envelope is its members'
    c = np.minimum(np.maximum(qsym[None, :], lo), hi)
    return _tree(T8[np.arange(16)[None, :], c])           # [runs] float32


def test_fine_and_run_bounds_within_the_margin():
    X = synth.random_walks(40000, 256, seed=71)
    S0 = isax(paa(X)).astype(np.int64)
    perm, _ = sorted_order(S0.astype(np.uint8))
    S = S0[perm]                                          # leaf order, as the scan reads it
    Qn, _, _ = synth.noisy_queries(X, 6, seed=72, sigma=(0.01, 0.8))
    Q = np.concatenate([Qn, synth.fresh_walk_queries(3, 256, seed=73)])
    for q in Q:
        qp = paa(q)
        qsym = isax(qp[None, :])[0].astype(np.int64)
        T8 = _round_toward_zero_f32(lb_table(qp, 16))
        lb = lower_bound_sq(qp, S, 16)
        fine = _fine32(T8, S)
        run = _run32(T8, S, qsym)
        assert np.all(fine.astype(np.float64) <= lb * (1 + G15) + 1e-30)
        member_run = np.repeat(run, RUN)[:S.shape[0]]
        assert np.all(member_run <= fine)                 # exact, in float32
        # at any threshold, a series within it by a relative 1e-6 passes both bounds
        for thr in np.quantile(lb, [0.001, 0.05, 0.5]):
            keep = lb <= thr * (1 - 1e-6)
            assert np.all(member_run[keep] <= thr) and np.all(fine[keep] <= thr)
        # in leaf order the envelopes are tight enough to prune: most runs fall at a low threshold
        thr = np.quantile(lb, 0.001)
        assert np.mean(run > thr) > 0.5
