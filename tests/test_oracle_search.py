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


# ---- the approximate search (Section 3.3): the smallest real distance over the reached leaf ----
def test_approximate_seed_hand_worked():
    """q = 0 and constant rows c: ED^2 = 16 c^2. Members 4, 1, 3, 0 hold 2.5, -2, 2, 3, so the
    squared distances are 100, 64, 64, 144: the minimum 64 is tied between series 1 and 3 and
    goes to the lower index 1. Series 2 (0.5, distance^2 4) is closer but not a member."""
    from oracle import approximate_seed, approximate_seed_k
    vals = [3.0, -2.0, 0.5, 2.0, 2.5]
    X = np.stack([np.full(16, v, np.float32) for v in vals])
    q = np.zeros(16, np.float32)
    members = np.array([4, 1, 3, 0])
    assert approximate_seed(q, X, members) == (1, 64.0)
    assert approximate_seed(q, X, members[::-1].copy()) == (1, 64.0)
    idx, d2 = approximate_seed_k(q, X, members, 3)
    assert list(idx) == [1, 3, 4] and list(d2) == [64.0, 64.0, 100.0]
    assert approximate_seed(q, X, np.array([], np.int64)) == (-1, float("inf"))


def test_approximate_seed_is_the_window_minimum_by_brute_force():
    """Against scipy's distance matrix over the whole window (every member, not a sample)."""
    from scipy.spatial.distance import cdist
    from oracle import approximate_seed
    X = _collection(6000, 64, seed=8)
    S = isax(paa(X))
    perm, ks = sorted_order(S)
    off = root_offsets(ks)
    Q, _, _ = synth.noisy_queries(X, 12, seed=9, sigma=(0.2, 0.8))
    windows = [seed_window(query_summary(q), ks, 4, "root16", seed_cap=1500, off=off) for q in Q]
    windows += [seed_window(query_summary(q), ks, 4, "equal_count", n_leaves=4) for q in Q]
    for q, (a, b) in zip(list(Q) + list(Q), windows):
        members = perm[a:b]
        d = cdist(q[None, :].astype(np.float64), X[members].astype(np.float64), "sqeuclidean")[0]
        j = np.lexsort((members, d))[0]
        i, d2 = approximate_seed(q, X, members)
        assert i == members[j] and d2 == pytest.approx(d[j], rel=1e-12)
        # the seed bounds the exact answer from above
        assert d2 >= nn_bruteforce(q, X)[1]


def _knn_refined_closed_form(q, X, S, k, a, b, perm):
    """Refined rows of the k-NN twin, from its definition: candidates outside the window are
    taken in ascending (bound, index); the k-th best before candidate t is the k-th smallest of
    the window's distances and the FULL distances of every earlier candidate (a pruned or
    abandoned candidate is farther than the k-th best, so adding it never changes that order
    statistic); candidate t is refined iff its bound does not exceed that value."""
    import heapq
    from oracle import ed_sq
    n = X.shape[1]
    lb = lower_bound_sq(query_summary(q).paa[None, :], S, n // 16)
    d_all = ed_sq(q, X)
    window = set(int(m) for m in perm[a:b])
    heap = [-float(d_all[m]) for m in window]          # max-heap of the k smallest
    heapq.heapify(heap)
    while len(heap) > k:
        heapq.heappop(heap)
    refined = 0
    for i in np.lexsort((np.arange(X.shape[0]), lb)):
        i = int(i)
        if i in window:
            continue
        kth = -heap[0] if len(heap) >= k else np.inf
        if not (lb[i] > kth * (1.0 + 1e-9) + 1e-12):
            refined += 1
        heapq.heappush(heap, -float(d_all[i]))
        if len(heap) > k:
            heapq.heappop(heap)
    return refined


@pytest.mark.parametrize("k", [1, 4, 16])
def test_knn_twin_refined_count_closed_form(k):
    from oracle import exact_search_knn
    X = _collection(1200, 64, seed=10)
    S = isax(paa(X))
    perm, ks = sorted_order(S)
    off = root_offsets(ks)
    Q, _, _ = synth.noisy_queries(X, 4, seed=11, sigma=(0.1, 0.7))
    Q = np.concatenate([Q, synth.fresh_walk_queries(2, 64, seed=12)])
    for q in Q:
        a, b = seed_window(query_summary(q), ks, 4, "root16", seed_cap=32, off=off)
        _, _, refined = exact_search_knn(q, X, k, S, seed_cap=32)
        assert refined == _knn_refined_closed_form(q, X, S, k, a, b, perm)
        assert refined < X.shape[0] - (b - a)      # the bound prunes something


# ---- the C oracle's eight-queries-per-pass brute force and its serial exact-search twin ------
@pytest.mark.parametrize("M", [1, 3, 8, 9, 17])
def test_c_brute_force_blocked_is_bit_identical(oracle_native, M):
    X = _collection(1500, 128, seed=31)
    X[900] = X[33]                       # an exact tie: the lower index must win in both
    Q, _, _ = synth.noisy_queries(X, M, seed=M, sigma=(0.05, 0.6))
    Q[0] = X[33]
    a_i, a_d, _ = oracle_native.nn_many(Q, X, threads=2)
    b_i, b_d, _ = oracle_native.nn_many_blocked(Q, X, threads=2)
    assert np.array_equal(a_i, b_i) and np.array_equal(a_d.view(np.uint64), b_d.view(np.uint64))
    assert b_i[0] == 33 and b_d[0] == 0.0


@pytest.mark.parametrize("mode", ["root16", "equal_count"])
def test_c_exact_search_twin_equals_numpy_twin_and_brute_force(oracle_native, mode):
    """The serial C twin takes the same steps as the numpy twin: same answer, seed and counters
    (survivors, refined, abandoned, updates), and the brute-force answer."""
    X = _collection(3000, 256, seed=32)
    X[2500] = X[40]
    S = isax(paa(X))
    Q, _, _ = synth.noisy_queries(X, 10, seed=5, sigma=(0.05, 0.6))
    Q = np.concatenate([Q, synth.fresh_walk_queries(3, 256, seed=6), X[40:41]])
    ix = oracle_native.SearchIndex(X, S, mode=mode, seed_cap=256, n_leaves=16)
    for q in Q:
        i, d2, st = oracle_native.exact_search(q, ix)
        j, e2, ref = exact_search(q, X, S, mode=mode, seed_cap=256, n_leaves=16)
        assert (i, d2) == (j, e2) == nn_bruteforce(q, X)[:2]
        assert st == {"seed_index": ref.seed_index, "lb_survivors": ref.lb_survivors,
                      "refined": ref.refined, "abandoned": ref.abandoned,
                      "bsf_updates": ref.bsf_updates}
    # the tie at distance 0 goes to the lower index, and an empty leaf means no seed
    assert oracle_native.exact_search(X[40], ix)[:2] == (40, 0.0)
    none = (np.zeros(0, np.int64), paa(Q[0]))
    i, d2, st = oracle_native.exact_search(Q[0], ix, members=none)
    assert (i, d2) == nn_bruteforce(Q[0], X)[:2] and st["seed_index"] == -1
    assert st["lb_survivors"] == 3000
