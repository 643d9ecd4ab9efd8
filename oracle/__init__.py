"""Plain, slow CPU oracle for exact 1-NN search over iSAX summaries.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may call it.
It shares no code, headers, tables or constant generators with the GPU library: its Gaussian
breakpoints come from its own high-precision computation (``breakpoints.py``), its arithmetic
from ``reference.py`` (numpy, float64) and ``paris_oracle.c`` (plain C, float64, built with
``-ffp-contract=off``); the ADS+ tree and its leaf descent from ``ads.py``; the learned seed's network (forward, back-propagation, Adam, top
leaves, labels) from ``mlp.py`` (numpy, float64).

Parity pins: every function here is checked by ``tests/test_oracle_*.py`` against values that
do not come from the oracle itself (closed forms, the paper's printed word example, library
routines such as scipy's normal quantile and pairwise distances, brute force on tiny inputs,
and the lower-bound invariant). Functions with no such pin say "parity unpinned" below.
"""
from .breakpoints import breakpoints, breakpoints_at_cardinality  # noqa: F401
from .reference import (  # noqa: F401
    paa, isax, root_key, k64, lower_bound_sq, ed_sq, nn_bruteforce, sorted_order,
    root_offsets, equal_count_bounds, seed_window, exact_search, exact_search_nb, ExactStats, query_summary,
    knn_bruteforce, exact_search_knn,
    lb_table, approximate_seed, approximate_seed_k, block_lower_bound_sq, seed_members,
)
from .ads import AdsTree, ads_query_leaf, ads_tree, next_bit  # noqa: F401
