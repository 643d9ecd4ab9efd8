"""Pins for the oracle's exact k-NN (the k nearest series, used by the paper's k-NN
classification experiment, Section 4): the definition against scipy's distance matrix and a
library sort; k = 1 against the 1-NN definition and the 1-NN twin; the serial k-NN twin (the
best-so-far is the k-th best) against the definition, with ties, k >= N and both leaf modes."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synth
from oracle import exact_search, exact_search_knn, isax, knn_bruteforce, nn_bruteforce, paa
from oracle.reference import lower_bound_sq, query_summary, seed_window, sorted_order


def test_definition_against_library():
    X = synth.random_walks(800, 64, seed=21)
    Q = synth.fresh_walk_queries(4, 64, seed=22)
    for q in Q:
        d = cdist(q[None, :].astype(np.float64), X.astype(np.float64), "sqeuclidean")[0]
        ref = np.lexsort((np.arange(len(d)), d))[:25]
        idx, d2 = knn_bruteforce(q, X, 25)
        assert np.array_equal(idx, ref)
        assert np.allclose(d2, d[ref], rtol=1e-12, atol=0)
        assert np.all(np.diff(d2) >= 0)
        i1, d1, _ = nn_bruteforce(q, X)
        assert (int(knn_bruteforce(q, X, 1)[0][0]), float(knn_bruteforce(q, X, 1)[1][0])) == (i1, d1)


@pytest.mark.parametrize("k,mode", [(1, "root16"), (3, "root16"), (10, "equal_count"), (40, "root16")])
def test_twin_equals_definition(k, mode):
    X = synth.random_walks(1500, 128, seed=23)
    S = isax(paa(X))
    Qn, _, _ = synth.noisy_queries(X, 4, seed=24, sigma=(0.05, 0.6))
    Q = np.concatenate([Qn, synth.fresh_walk_queries(2, 128, seed=25)])
    for q in Q:
        ri, rd = knn_bruteforce(q, X, k)
        idx, d2, refined = exact_search_knn(q, X, k, S, mode=mode, seed_cap=64, n_leaves=32)
        assert np.array_equal(idx, ri) and np.array_equal(d2, rd)
        assert refined <= X.shape[0]
        if k == 1:
            i1, dd1, _ = exact_search(q, X, S, mode=mode, seed_cap=64, n_leaves=32)
            assert (int(idx[0]), float(d2[0])) == (i1, dd1)


def test_ties_and_k_beyond_n():
    X = synth.random_walks(1500, 64, seed=26)
    X[700] = X[20]
    X[1400] = X[20]
    S = isax(paa(X))
    q = (X[20] + np.float32(0.001)).astype(np.float32)
    idx, d2, _ = exact_search_knn(q, X, 3, S, seed_cap=16)
    assert list(idx) == [20, 700, 1400] and d2[0] == d2[1] == d2[2]
    small = X[:7]
    idx, d2, _ = exact_search_knn(q, small, 12, isax(paa(small)), seed_cap=16)
    ri, rd = knn_bruteforce(q, small, 12)
    assert len(idx) == 7 and np.array_equal(idx, ri) and np.array_equal(d2, rd)


@pytest.mark.parametrize("k", [5, 20])
def test_twin_refines_between_its_pruning_bounds(k):
    """The twin's pruning against bounds computed without it: every series outside the seed window
    whose lower bound is at most the final k-th distance must be refined (the threshold never
    drops below it), and none whose bound exceeds the k-th distance among the window's members
    (the threshold never rises above it); on this workload the second bound is well below the
    series outside the window, so a twin that does not prune fails it."""
    X = synth.random_walks(3000, 128, seed=27)
    S = isax(paa(X))
    L = 128 // 16
    Qn, _, _ = synth.noisy_queries(X, 3, seed=28, sigma=0.2)
    perm, keys = sorted_order(S)
    for q in Qn:
        idx, d2, refined = exact_search_knn(q, X, k, S, mode="equal_count", seed_cap=64, n_leaves=32)
        ri, rd = knn_bruteforce(q, X, k)
        assert np.array_equal(idx, ri) and np.array_equal(d2, rd)
        qs = query_summary(q)
        a, b = seed_window(qs, keys, L, "equal_count", 64, 32)
        members = np.sort(perm[a:b])
        assert len(members) >= k
        outside = np.ones(len(X), bool)
        outside[members] = False
        lb = lower_bound_sq(qs.paa[None, :], S, L)
        first_kth = float(knn_bruteforce(q, X[members], k)[1][-1])
        lo = int(np.sum(outside & (lb <= float(rd[-1]))))
        hi = int(np.sum(outside & (lb <= first_kth * (1.0 + 1e-9) + 1e-12)))
        assert lo <= refined <= hi
        assert hi < int(outside.sum()) // 2
