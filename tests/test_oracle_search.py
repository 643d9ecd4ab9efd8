"""Pins for the oracle's exact-search twin (Section 3.3.3) and its leaf/seed layout, plus the
bit-exact agreement of the two oracle implementations (numpy and C)."""
import numpy as np
import pytest

import synth
from oracle import (equal_count_bounds, exact_search, isax, k64, lower_bound_sq, nn_bruteforce,
                    paa, query_summary, root_key, root_offsets, seed_window, sorted_order)


def _collection(N, n, seed=0):
    X = synth.random_walks(N, n, seed=seed)
    return X


@pytest.mark.parametrize("n,mode", [(16, "root16"), (128, "root16"), (256, "equal_count"),
                                    (256, "root16")])
def test_twin_equals_bruteforce(n, mode):
    X = _collection(1500, n, seed=n)
    Q, src, _ = synth.noisy_queries(X, 6, seed=1, sigma=(0.05, 0.6))
    S = isax(paa(X))
    for q in Q:
        i_bf, d_bf, _ = nn_bruteforce(q, X)
        i, d, st = exact_search(q, X, S, mode=mode, seed_cap=64, n_leaves=32)
        assert (i, d) == (i_bf, d_bf)
        assert st.lb_survivors >= 1 and st.refined >= 1
        i2, d2, st2 = exact_search(q, X, S, use_seed=False)
        assert (i2, d2) == (i_bf, d_bf)
        assert st2.lb_survivors == 1500  # BSF = +inf prunes nothing


def test_twin_ties_and_degenerate():
    X = _collection(600, 64, seed=3)
    X[400] = X[17]
    X[550] = X[17]
    S = isax(paa(X))
    i, d, _ = exact_search(X[17], X, S, seed_cap=16)
    assert (i, d) == (17, 0.0)
    q = (X[17] + np.float32(0.01)).astype(np.float32)
    assert exact_search(q, X, S, seed_cap=16)[0] == nn_bruteforce(q, X)[0] == 17
    one = X[:1].copy()
    assert exact_search(q, one)[0] == 0


def test_sorted_order_and_offsets():
    X = _collection(3000, 256, seed=4)
    S = isax(paa(X))
    perm, ks = sorted_order(S)
    keys = k64(S)
    assert np.all(np.diff(ks.astype(np.float64)) >= 0) or np.all(ks[1:] >= ks[:-1])
    # stable: equal keys keep ascending positions
    same = ks[1:] == ks[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])
    assert np.array_equal(np.sort(perm), np.arange(3000))
    off = root_offsets(ks)
    assert off[0] == 0 and off[-1] == 3000 and np.all(np.diff(off) >= 0)
    r = root_key(S)
    counts = np.bincount(r, minlength=65536)
    assert np.array_equal(np.diff(off), counts)
    b = equal_count_bounds(3000, 7)
    assert b[0] == 0 and b[-1] == 3000 and np.all(np.diff(b) >= 428)


def test_seed_window_rules():
    X = _collection(5000, 256, seed=5)
    S = isax(paa(X))
    perm, ks = sorted_order(S)
    off = root_offsets(ks)
    Q, _, _ = synth.noisy_queries(X, 30, seed=2, sigma=0.5)
    for q in Q:
        qs = query_summary(q)
        a, b = seed_window(qs, ks, 16, "root16", seed_cap=32, off=off)
        assert 0 <= a < b <= 5000 and b - a <= 32
        r = int(ks[a] >> np.uint64(48))
        assert np.all((ks[a:b] >> np.uint64(48)) == r)      # one root subtree
        if off[qs.root + 1] > off[qs.root]:
            assert r == qs.root
        a2, b2 = seed_window(qs, ks, 16, "equal_count", n_leaves=64)
        bounds = equal_count_bounds(5000, 64)
        assert a2 in bounds and b2 in bounds and b2 > a2
        c = int(np.searchsorted(ks, np.uint64(qs.k64)))
        assert a2 <= min(c, 4999) < b2


def test_empty_bucket_picks_min_card2_bound():
    X = _collection(200, 256, seed=6)
    S = isax(paa(X))
    perm, ks = sorted_order(S)
    off = root_offsets(ks)
    q = -X[0]  # sign flip: usually lands in a subtree with no members
    qs = query_summary(q.astype(np.float32))
    a, b = seed_window(qs, ks, 16, "root16", seed_cap=2048, off=off)
    r = int(ks[a] >> np.uint64(48))
    nonempty = np.nonzero(np.diff(off) > 0)[0]
    bits = ((nonempty[:, None] >> (15 - np.arange(16))[None, :]) & 1)
    lb = lower_bound_sq(qs.paa[None, :], bits, 16, bits=1)
    assert lb[list(nonempty).index(r)] == lb.min()


def test_numpy_and_c_oracles_bit_exact(oracle_native):
    X = _collection(2000, 256, seed=7)
    Q, _, _ = synth.noisy_queries(X, 5, seed=3, sigma=0.3)
    p_np = paa(X)
    s_np = isax(p_np)
    p_c, s_c = oracle_native.summarise(X)
    assert np.array_equal(p_np.view(np.uint64), p_c.view(np.uint64))
    assert np.array_equal(s_np, s_c)
    for q in Q:
        from oracle import ed_sq
        assert np.array_equal(ed_sq(q, X).view(np.uint64), oracle_native.ed2(q, X).view(np.uint64))
        qp = paa(q)
        assert np.array_equal(lower_bound_sq(qp, s_np, 16).view(np.uint64),
                              oracle_native.lb2(qp, s_np, 16).view(np.uint64))
    idx, d2, _ = oracle_native.nn_many(Q, X, threads=3)
    for m, q in enumerate(Q):
        i, d, _ = nn_bruteforce(q, X)
        assert idx[m] == i and d2[m] == d
    sel = np.array([5, 1999, 0, 77])
    assert np.array_equal(oracle_native.ed2_at(Q[0], X, sel), oracle_native.ed2(Q[0], X)[sel])


def test_c_oracle_short_segments(oracle_native):
    # L = 3 (n = 48): division by a non-power of two must round identically
    rng = np.random.default_rng(13)
    X = rng.standard_normal((500, 48)).astype(np.float32)
    p_c, s_c = oracle_native.summarise(X)
    assert np.array_equal(paa(X).view(np.uint64), p_c.view(np.uint64))
    assert np.array_equal(isax(paa(X)), s_c)
