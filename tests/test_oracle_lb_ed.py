"""Pins for the oracle's lower bound (Section 3.3.1) and Euclidean distance (Section 2.1)."""
import numpy as np
import pytest

from oracle import (breakpoints, ed_sq, isax, lb_table, lower_bound_sq,
                    nn_bruteforce, paa)

Q3 = 0.6744897501960817  # upper quartile of N(0,1)


def test_hand_worked_example():
    """n = 8, w = 2 (L = 4), cardinality 4 with boundaries (-Q3, 0, Q3).

    x = [1]*4 + [-0.5]*4 -> PAA (1, -0.5) -> word (3, 1).
    q = [-1]*4 + [1]*4   -> PAA (-1, 1).
    Segment 0: q mean -1 is BELOW x's region [Q3, inf): delta = Q3 + 1.
    Segment 1: q mean 1 is ABOVE x's region [-Q3, 0): delta = 1 - 0.
    LB^2 = 4 * ((Q3 + 1)^2 + 1); ED^2 = 4*(2^2) + 4*(1.5^2) = 25.
    """
    x = np.array([1, 1, 1, 1, -0.5, -0.5, -0.5, -0.5], np.float32)
    q = np.array([-1, -1, -1, -1, 1, 1, 1, 1], np.float32)
    xp, qp = paa(x, 2), paa(q, 2)
    assert list(xp) == [1.0, -0.5] and list(qp) == [-1.0, 1.0]
    wx = isax(xp, bits=2)
    assert list(wx) == [3, 1]
    assert list(isax(qp, bits=2)) == [0, 3]
    lb2 = lower_bound_sq(qp, wx, 4, bits=2)
    expect = 4.0 * ((Q3 + 1.0) * (Q3 + 1.0) + 1.0)
    assert lb2 == pytest.approx(expect, rel=1e-15)
    assert lb2 == pytest.approx(15.215663694046944, rel=1e-14)
    assert ed_sq(q, x) == 25.0
    # PAA bound L * sum (qbar - xbar)^2 is tight for piecewise-constant series
    assert 4.0 * np.sum((qp - xp) ** 2) == 25.0


def test_lb_zero_for_own_word_and_equal_words():
    rng = np.random.default_rng(7)
    X = np.cumsum(rng.standard_normal((40, 256)), axis=1).astype(np.float32)
    P = paa(X)
    S = isax(P)
    lb_self = lower_bound_sq(P, S, 16)
    assert np.all(lb_self == 0.0)
    q = P[0]
    same = np.repeat(S[:1], 5, axis=0)
    v = lower_bound_sq(q[None, :] + 0.3, same, 16)
    assert np.all(v == v[0])


def test_lb_branches_individually():
    b = breakpoints()
    L = 16
    # one segment moved, the other 15 set IN their region
    sym = np.full((1, 16), 128, np.uint8)       # region [0, b[129])
    q = np.full(16, 0.5 * b[129])               # inside
    assert lower_bound_sq(q, sym, L)[0] == 0.0
    q2 = q.copy(); q2[3] = -0.25                # BELOW region [0, ..): delta = 0 - (-0.25)
    assert lower_bound_sq(q2, sym, L)[0] == L * 0.0625
    q3 = q.copy(); q3[9] = b[129] + 0.5         # ABOVE: delta = q - b[129]
    d = (b[129] + 0.5) - b[129]
    assert lower_bound_sq(q3, sym, L)[0] == L * d * d
    # end regions: symbol 0 is (-inf, b1), symbol 255 is [b255, inf)
    sym0 = np.zeros((1, 16), np.uint8)
    q4 = np.full(16, b[1] - 1.0)
    assert lower_bound_sq(q4, sym0, L)[0] == 0.0
    sym255 = np.full((1, 16), 255, np.uint8)
    assert lower_bound_sq(q4, sym255, L)[0] == pytest.approx(L * 16 * (b[255] - q4[0]) ** 2, rel=1e-15)


def _walks(rng, N, n):
    w = np.cumsum(rng.standard_normal((N, n)), axis=1)
    w = (w - w.mean(1, keepdims=True)) / w.std(1, keepdims=True)
    return w.astype(np.float32)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_lb_below_paa_bound_below_ed(n):
    rng = np.random.default_rng(8 + n)
    X = _walks(rng, 500, n)
    Q = _walks(rng, 20, n)
    L = n // 16
    P = paa(X)
    S = isax(P)
    for q in Q:
        qp = paa(q)
        lb = lower_bound_sq(qp, S, L)
        lbp = L * np.sum((qp[None, :] - P) ** 2, axis=1)
        ed = ed_sq(q, X)
        assert np.all(lb <= lbp * (1 + 1e-12) + 1e-12)
        assert np.all(lbp <= ed * (1 + 1e-12) + 1e-12)


def test_paa_bound_equals_ed_with_unit_segments():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((30, 16)).astype(np.float32)
    q = rng.standard_normal(16).astype(np.float32)
    lbp = np.sum((paa(q)[None, :] - paa(X)) ** 2, axis=1)
    assert np.allclose(lbp, ed_sq(q, X), rtol=1e-15, atol=0)


def test_tables_reassemble_the_bound():
    rng = np.random.default_rng(10)
    X = _walks(rng, 300, 256)
    q = _walks(rng, 1, 256)[0]
    qp = paa(q)
    S = isax(paa(X))
    T = lb_table(qp, 16)
    via_table = T[np.arange(16)[None, :], S.astype(np.int64)].sum(axis=1)
    assert np.allclose(via_table, lower_bound_sq(qp, S, 16), rtol=1e-13, atol=1e-13)
    # a region's entry is zero where it holds the query's value and grows away from it: the
    # property that lets the symbol range of a group of series bound every member
    qs = isax(qp[None, :])[0].astype(np.int64)
    for s in range(16):
        assert T[s][qs[s]] == 0
        assert np.all(np.diff(T[s][:qs[s] + 1]) <= 0) and np.all(np.diff(T[s][qs[s]:]) >= 0)


def test_ed_against_library_routines():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(11)
    X = _walks(rng, 200, 256)
    q = _walks(rng, 1, 256)[0]
    ours = ed_sq(q, X)
    ref = cdist(q[None, :].astype(np.float64), X.astype(np.float64), "sqeuclidean")[0]
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(ours, ((X.astype(np.float64) - q.astype(np.float64)) ** 2).sum(1),
                       rtol=1e-12, atol=1e-12)


def test_nn_matches_library_argmin_and_ties():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(12)
    X = _walks(rng, 1000, 128)
    Q = _walks(rng, 10, 128)
    for q in Q:
        i, d2, d = nn_bruteforce(q, X)
        ref = cdist(q[None, :].astype(np.float64), X.astype(np.float64), "sqeuclidean")[0]
        assert i == int(np.argmin(ref))
        assert d == pytest.approx(np.sqrt(ref[i]), rel=1e-12)
    # duplicated series: the lowest index wins
    X2 = X.copy()
    X2[700] = X2[35]
    X2[900] = X2[35]
    i, _, d = nn_bruteforce(X2[35], X2)
    assert i == 35 and d == 0.0
    q = X2[35] + np.float32(1e-3)
    assert nn_bruteforce(q, X2)[0] == 35


def test_block_bound_hand_worked_and_special_cases():
    """The run bound: one member reduces it to that member's bound; a query inside the run's
    symbol envelope in every segment gets 0; a hand-worked two-member run."""
    from oracle import block_lower_bound_sq
    b = breakpoints()
    rng = np.random.default_rng(31)
    L = 16
    for _ in range(20):
        sym = rng.integers(0, 256, 16).astype(np.uint8)
        qp = rng.standard_normal(16)
        assert block_lower_bound_sq(qp, sym[None, :], L) == lower_bound_sq(qp, sym[None, :], L)[0]
    lo_sym = np.full(16, 100, np.uint8)
    hi_sym = np.full(16, 140, np.uint8)
    run = np.stack([lo_sym, hi_sym])
    inside = np.full(16, 0.5 * (b[120] + b[121]))
    assert block_lower_bound_sq(inside, run, L) == 0.0
    # segment 0 below the envelope by 0.25, segment 1 above it by 0.5, the rest inside:
    # L * (0.25^2 + 0.5^2) by hand
    q = inside.copy()
    q[0] = b[100] - 0.25
    q[1] = b[141] + 0.5
    assert block_lower_bound_sq(q, run, L) == pytest.approx(L * (0.25 ** 2 + 0.5 ** 2), rel=1e-14)


@pytest.mark.parametrize("run", [2, 32, 256])
def test_block_bound_below_every_member(run):
    """Brute force over every member: the run bound never exceeds a member's bound or its
    squared Euclidean distance, and adding members never raises it."""
    from oracle import block_lower_bound_sq
    rng = np.random.default_rng(40 + run)
    n = 64
    X = _walks(rng, 4 * run, n)
    Q = _walks(rng, 10, n)
    L = n // 16
    S = isax(paa(X))
    for q in Q:
        qp = paa(q)
        for r0 in range(0, X.shape[0], run):
            members = S[r0:r0 + run]
            blb = block_lower_bound_sq(qp, members, L)
            assert np.all(blb <= lower_bound_sq(qp, members, L))
            assert np.all(blb <= ed_sq(q, X[r0:r0 + run]))
            assert block_lower_bound_sq(qp, members[: max(1, run // 2)], L) >= blb
