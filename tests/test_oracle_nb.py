"""Pins for the oracle's nb-ParIS+ twin (Section 3.3: distance workers with private best-so-far
copies over contiguous blocks, the answer the minimum of the copies): the answer is brute
force's; each worker's refined count equals its closed form, where the copy at position i is
the minimum of the approximate answer and the distances at earlier positions of the block
(computed here without early abandoning); and a finer split into blocks never refines fewer
rows than a coarser one that it nests in."""
import numpy as np
import pytest

import synth
from oracle import ed_sq, exact_search, exact_search_nb, isax, lower_bound_sq, nn_bruteforce, paa, query_summary


def _closed_form_refined(q, X, S, workers, seed):
    N, n = X.shape
    lb = lower_bound_sq(query_summary(q).paa[None, :], S, n // 16)
    d = ed_sq(q, X)
    out = []
    edges = [w * N // workers for w in range(workers + 1)]
    for w in range(workers):
        best, r = seed, 0
        for i in range(edges[w], edges[w + 1]):
            if not lb[i] > best * (1.0 + 1e-9) + 1e-12:
                r += 1
            best = min(best, d[i])
        out.append(r)
    return out


@pytest.mark.parametrize("workers", [1, 2, 5, 12])
def test_nb_twin_answers_and_counts(workers):
    X = synth.random_walks(1500, 64, seed=11)
    X[1400] = X[20]                       # a duplicate in another block: ties go to index 20
    S = isax(paa(X))
    Q, _, _ = synth.noisy_queries(X, 4, seed=2, sigma=(0.1, 0.8))
    Q = np.concatenate([Q, X[20:21], synth.fresh_walk_queries(2, 64, seed=3)])
    for q in Q:
        i_bf, d_bf, _ = nn_bruteforce(q, X)
        i, d, refined = exact_search_nb(q, X, workers, S, seed_cap=64)
        assert (i, d) == (i_bf, d_bf)
        seed = exact_search(q, X, S, seed_cap=64)[2].seed_d2
        assert refined == _closed_form_refined(q, X, S, workers, seed)


def test_nb_finer_split_refines_more():
    X = synth.random_walks(1500, 64, seed=12)
    S = isax(paa(X))
    Q = synth.fresh_walk_queries(6, 64, seed=4)     # hard queries: many rows survive the bound
    strict = 0
    for q in Q:
        totals = [sum(exact_search_nb(q, X, w, S, seed_cap=16)[2]) for w in (1, 4, 12)]
        assert totals[0] <= totals[1] <= totals[2]
        strict += totals[2] > totals[0]
    assert strict >= 1
