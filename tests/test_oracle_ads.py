"""Pins for the oracle's ADS+ tree (Section 2.2: root subtrees, leaves that split by refining one
segment's cardinality by one bit, the most balanced segment chosen; the approximate search's
descent to the query's leaf, Section 3.3): a hand-worked five-series tree, structural invariants
and the balance rule checked by brute force on random walks, the descent against the set of
series sharing the query's prefix, and the exact search in the tree's leaf mode against brute
force."""
import numpy as np
import pytest

import synth
from oracle import ads_query_leaf, ads_tree, exact_search, isax, nn_bruteforce, paa, query_summary

ROOT_ALL_ONES = 65535


def _hand_words():
    """Five words, every segment's symbol 128 (first bit 1, next bits 0) except segments 0 and 1."""
    S = np.full((5, 16), 128, np.uint8)
    S[:, 0] = [0b11000000, 0b10000000, 0b11000000, 0b10000000, 0b11100000]
    S[:, 1] = [0b10000000, 0b11000000, 0b11000000, 0b10000000, 0b10000000]
    return S


def test_hand_worked_tree():
    """All five share root key 0xFFFF. Round 1 (node 65535, 5 > cap 2): the second bit of segment
    0 is 1 for series 0, 2, 4 (gap |2*3 - 5| = 1) and of segment 1 for series 1, 2 (gap 1); every
    other segment puts all five on one side (gap 5). Tie: segment 0. Bit-0 child 65536 = {3, 1}
    (leaf order: ascending 64-bit key, then index), bit-1 child 65537 = {0, 4, 2}. Round 2 (node
    65537, 3 > 2): segment 0's third bit is 1 for series 4 only (gap 1), segment 1's second bit
    for series 2 only (gap 1): segment 0 again. Children 65538 = {0, 2}, 65539 = {4}."""
    t = ads_tree(_hand_words(), cap=2)
    assert t.n_nodes == 65540
    assert (t.child0[ROOT_ALL_ONES], t.split[ROOT_ALL_ONES]) == (65536, 0)
    assert list(t.perm) == [3, 1, 0, 2, 4]
    assert (t.start[65536], t.end[65536], t.child0[65536]) == (0, 2, -1)
    assert (t.start[65537], t.end[65537], t.child0[65537], t.split[65537]) == (2, 5, 65538, 0)
    assert (t.start[65538], t.end[65538], t.start[65539], t.end[65539]) == (2, 4, 4, 5)
    assert list(t.card[65539][:3]) == [3, 1, 1] and list(t.card[65536][:2]) == [2, 1]
    for r in range(65535):
        assert t.start[r] == t.end[r] == 0 and t.child0[r] == -1


@pytest.mark.parametrize("s0,leaf", [(0b11100000, 65539), (0b11000000, 65538), (0b10100000, 65536)])
def test_hand_worked_descent(s0, leaf):
    t = ads_tree(_hand_words(), cap=2)
    q = np.full(16, 128, np.int64)
    q[0] = s0
    assert ads_query_leaf(t, q, np.full(16, 0.1), 16) == leaf


def test_descent_into_an_empty_child_takes_the_other():
    """Four series that differ only in segment 3's second bit: the first split refines segment 3
    (gap 0); a later split of {0b1100.., 0b1100..} on every segment gives an empty child; a query
    whose bit leads there is sent to the non-empty sibling."""
    S = np.full((4, 16), 128, np.uint8)
    S[:, 3] = [0b11000000, 0b11000000, 0b10000000, 0b10000000]
    t = ads_tree(S, cap=1)
    v = ROOT_ALL_ONES
    assert t.split[v] == 3
    q = np.full(16, 128, np.int64)
    q[3] = 0b11000000
    q[0] = 0b11000000          # segment 0 leads to empty children of the duplicates' subtree
    leaf = ads_query_leaf(t, q, np.full(16, 0.1), 16)
    assert t.end[leaf] > t.start[leaf]
    assert set(t.perm[t.start[leaf]:t.end[leaf]].tolist()) <= {0, 1}


@pytest.mark.parametrize("N,n,cap", [(20000, 256, 64), (6000, 64, 16)])
def test_tree_invariants_and_balance_rule(N, n, cap):
    X = synth.random_walks(N, n, seed=41)
    X[100:140] = X[7]          # 41 identical words: an unsplittable node beyond the capacity
    S = isax(paa(X))
    t = ads_tree(S, cap)
    assert np.array_equal(np.sort(t.perm), np.arange(N))
    inner = np.nonzero(t.child0 >= 0)[0]
    for v in inner:
        c0 = t.child0[v]
        a, b = t.start[v], t.end[v]
        assert (t.start[c0], t.end[c0 + 1]) == (a, b) and t.end[c0] == t.start[c0 + 1]
        s = t.split[v]
        cc = t.card[v].copy()
        cc[s] += 1
        assert np.array_equal(t.card[c0], cc) and np.array_equal(t.card[c0 + 1], cc)
        words = S[t.perm[a:b]].astype(np.int64)
        m = b - a
        assert m > cap
        # the split's segment gives the most even division, lowest segment on ties (brute force)
        gaps = [abs(2 * int(((words[:, k] >> (7 - t.card[v][k])) & 1).sum()) - m) if t.card[v][k] < 8
                else 1 << 40 for k in range(16)]
        assert s == int(np.argmin(gaps))
        bits = (words[:, s] >> (7 - t.card[v][s])) & 1
        assert np.all(bits[: t.end[c0] - a] == 0) and np.all(bits[t.end[c0] - a:] == 1)
    for v in t.leaves():
        a, b = t.start[v], t.end[v]
        assert b - a <= cap or np.all(t.card[v] == 8)
        if b > a:   # every member shares the node's prefix at its cardinalities
            w = S[t.perm[a:b]].astype(np.int64)
            top = w >> (8 - t.card[v])[None, :]
            assert np.all(top == top[0])
    # numbering: the children of one round's splits are consecutive, in the order of their parents
    assert np.all(np.diff(t.child0[inner]) > 0)
    # the duplicated words ended in one leaf with all 8 bits of every segment, or within capacity
    assert any(t.end[v] - t.start[v] >= 41 and np.all(t.card[v] == 8) for v in t.leaves()) or cap >= 41


def test_descent_reaches_the_leaf_of_the_query_prefix():
    """Without a detour (the child on the query's side never empty) the reached leaf holds exactly
    the series that share the query's symbol prefix at the leaf's cardinalities."""
    X = synth.random_walks(30000, 128, seed=42)
    S = isax(paa(X))
    t = ads_tree(S, 50)
    Q, _, _ = synth.noisy_queries(X, 40, seed=43, sigma=(0.05, 0.5))
    checked = 0
    for q in Q:
        qs = query_summary(q)
        v = ads_query_leaf(t, qs.sym, qs.paa, 8)
        card = t.card[v]
        qtop = qs.sym.astype(np.int64) >> (8 - card)
        match = np.nonzero(np.all((S.astype(np.int64) >> (8 - card)[None, :]) == qtop[None, :], axis=1))[0]
        members = np.sort(t.perm[t.start[v]:t.end[v]])
        if len(match):
            assert np.array_equal(members, match)
            checked += 1
    assert checked >= 30


@pytest.mark.parametrize("cap", [16, 200])
def test_exact_search_in_tree_mode_equals_brute_force(cap):
    X = synth.random_walks(3000, 256, seed=44)
    S = isax(paa(X))
    Q, _, _ = synth.noisy_queries(X, 6, seed=45, sigma=(0.05, 0.6))
    Q = np.concatenate([Q, synth.fresh_walk_queries(2, 256, seed=46)])
    for q in Q:
        i, d, st = exact_search(q, X, S, mode="ads", leaf_cap=cap)
        assert (i, d) == nn_bruteforce(q, X)[:2]
        assert st.seed_index >= 0
