"""Planted mistakes in the oracle (CPU only): each plausible slip must make at least one pin fail.

The mistakes are patched into ``oracle.reference`` for the duration of one test; the pins are the
unmodified test functions of the other oracle test modules.
"""
import numpy as np
import pytest

import oracle.reference as R
import tests.test_oracle_lb_ed as T_lb
import tests.test_oracle_search as T_search
import tests.test_oracle_summary as T_sum


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_boundary_side_flip_is_caught(monkeypatch):
    real = R.breakpoints_at_cardinality

    def isax_left(paa_values, bits=8):
        b = real(bits)
        return np.searchsorted(b[1:-1], np.asarray(paa_values, np.float64), side="left").astype(np.uint8)

    monkeypatch.setattr(R, "isax", isax_left)
    monkeypatch.setattr(T_sum, "isax", isax_left)
    _fails(T_sum.test_symbol_on_boundary_goes_up_and_extremes)


def test_breakpoint_index_shift_is_caught(monkeypatch):
    real = R.breakpoints_at_cardinality
    monkeypatch.setattr(R, "breakpoints_at_cardinality",
                        lambda bits: np.concatenate([real(bits)[1:], [np.inf]]))
    _fails(T_sum.test_paper_word_example)


def test_dropped_segment_length_factor_is_caught(monkeypatch):
    real = R.lower_bound_sq
    monkeypatch.setattr(T_lb, "lower_bound_sq", lambda q, s, L, bits=8: real(q, s, 1, bits))
    _fails(T_lb.test_hand_worked_example)


def test_lower_bound_branch_sign_is_caught(monkeypatch):
    def bad_delta(qp, lo, hi):
        d = np.zeros(np.broadcast(qp, lo).shape)
        d = np.where(qp < lo, lo + qp, d)        # wrong sign in the BELOW branch
        d = np.where(qp > hi, qp - hi, d)
        return d
    monkeypatch.setattr(R, "_delta", bad_delta)
    _fails(T_lb.test_lb_branches_individually)


def test_swapped_region_bounds_are_caught(monkeypatch):
    real = R._delta
    monkeypatch.setattr(R, "_delta", lambda qp, lo, hi: real(qp, hi, lo))
    _fails(T_lb.test_hand_worked_example)


def test_shifted_distance_index_is_caught(monkeypatch):
    def bad_ed(q, X):
        q = np.asarray(q, np.float32).astype(np.float64)
        X = np.asarray(X, np.float32)
        Xm = X[None, :] if X.ndim == 1 else X
        acc = np.zeros(Xm.shape[0])
        for j in range(Xm.shape[1]):
            d = q[j] - Xm[:, (j + 1) % Xm.shape[1]].astype(np.float64)   # off-by-one column
            acc = acc + d * d
        return acc[0] if X.ndim == 1 else acc
    monkeypatch.setattr(T_lb, "ed_sq", bad_ed)
    _fails(T_lb.test_ed_against_library_routines)


def test_root_key_bit_order_is_caught(monkeypatch):
    def bad_root(sym8):
        top = (np.asarray(sym8, np.uint8) >> 7).astype(np.uint32)
        key = np.zeros(top.shape[:-1], np.uint32)
        for s in range(16):
            key = key | (top[..., s] << np.uint32(s))
        return key
    monkeypatch.setattr(T_sum, "root_key", bad_root)
    _fails(T_sum.test_root_key_bit_order)


def test_strict_tie_rule_is_caught(monkeypatch):
    real_nn = R.nn_bruteforce

    def last_index_nn(q, X):
        d2 = R.ed_sq(q, X)
        i = int(len(d2) - 1 - np.argmin(d2[::-1]))   # ties to the highest index
        return i, float(d2[i]), float(np.sqrt(d2[i]))
    monkeypatch.setattr(T_search, "nn_bruteforce", last_index_nn)
    _fails(T_search.test_twin_ties_and_degenerate)
    monkeypatch.setattr(T_search, "nn_bruteforce", real_nn)


# ---- learned-seed oracle: back-propagation slips must fail the finite-difference pins ----------
import oracle.mlp as MLP  # noqa: E402
import tests.test_oracle_mlp as T_mlp  # noqa: E402


def _patched_grad(monkeypatch, edit):
    real = MLP.loss_and_grad

    def wrong(theta, P, y, n_out, rounding=True):
        L, g = real(theta, P, y, n_out, rounding)
        parts = MLP.unpack(g.copy(), n_out)
        edit(parts)
        return L, MLP.pack(parts, n_out)

    monkeypatch.setattr(MLP, "loss_and_grad", wrong)


def test_mlp_transposed_hidden_gradient_is_caught(monkeypatch):
    _patched_grad(monkeypatch, lambda p: p.__setitem__("W2", p["W2"].T.copy()))
    _fails(T_mlp.test_gradient_matches_finite_differences)


def test_mlp_dropped_bias_gradient_is_caught(monkeypatch):
    _patched_grad(monkeypatch, lambda p: p.__setitem__("b1", np.zeros_like(p["b1"])))
    _fails(T_mlp.test_gradient_matches_finite_differences)


def test_mlp_output_gradient_sign_is_caught(monkeypatch):
    _patched_grad(monkeypatch, lambda p: p.__setitem__("W3", -p["W3"]))
    _fails(T_mlp.test_gradient_matches_finite_differences)


def test_block_bound_lower_edge_of_largest_symbol_is_caught(monkeypatch):
    """Envelope closed at the lower edge of the largest symbol instead of its upper edge."""
    real_b = R.breakpoints_at_cardinality

    def bad(qpaa, sym_run, L, bits=8):
        b = real_b(bits)
        sym_run = np.asarray(sym_run).astype(np.int64).reshape(-1, R.W)
        d = R._delta(np.asarray(qpaa, np.float64), b[sym_run.min(0)], b[sym_run.max(0)])
        return np.float64(L) * float(np.sum(d * d))
    monkeypatch.setattr(R, "block_lower_bound_sq", bad)
    import oracle
    monkeypatch.setattr(oracle, "block_lower_bound_sq", bad)
    _fails(T_lb.test_block_bound_hand_worked_and_special_cases)


def test_block_bound_from_first_member_only_is_caught(monkeypatch):
    """The envelope taken from one member instead of the whole run."""
    real = R.lower_bound_sq
    bad = lambda qpaa, sym_run, L, bits=8: real(qpaa, np.asarray(sym_run).reshape(-1, R.W)[:1], L, bits)[0]
    import oracle
    monkeypatch.setattr(oracle, "block_lower_bound_sq", bad)
    _fails(T_lb.test_block_bound_below_every_member, 32)


def test_nb_copies_shared_between_workers_is_caught(monkeypatch):
    """nb-ParIS+ twin with one best-so-far for all workers (the copies not kept apart): the
    per-worker refined counts no longer match their closed form."""
    import tests.test_oracle_nb as T_nb
    real = R.exact_search_nb

    def shared_copy(q, X, workers, *a, **k):
        i, d, r = real(q, X, 1, *a, **k)
        return i, d, [sum(r)] + [0] * (workers - 1)

    monkeypatch.setattr(T_nb, "exact_search_nb", shared_copy)
    _fails(T_nb.test_nb_twin_answers_and_counts, 5)


# ---- approximate search and the k-NN twin ------------------------------------------------------
def _mutated(fn, old, new):
    """A copy of oracle function ``fn`` with one source fragment replaced (the planted slip)."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, old
    ns = dict(vars(R))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[fn.__name__]


def test_seed_sampled_per_run_is_caught(monkeypatch):
    """Refining only the smallest-bound member of every 512 sorted positions is a kernel design;
    as the oracle's seed it must fail the brute-force pin of the approximate search."""
    real = R.approximate_seed

    def sampled(q, X, members, run=512):
        members = np.asarray(members, np.int64)
        if len(members) == 0:
            return -1, float("inf")
        qp = R.query_summary(np.asarray(q, np.float32)).paa
        S = R.isax(R.paa(np.asarray(X[members], np.float32)))
        picks = []
        for a in range(0, len(members), run):
            lb = R.lower_bound_sq(qp[None, :], S[a:a + run], X.shape[1] // 16)
            picks.append(int(members[a + int(np.lexsort((members[a:a + run], lb))[0])]))
        return real(q, X, np.array(picks))
    monkeypatch.setattr(R, "approximate_seed", sampled)
    import oracle
    monkeypatch.setattr(oracle, "approximate_seed", sampled)
    _fails(T_search.test_approximate_seed_is_the_window_minimum_by_brute_force)


def test_seed_ties_to_highest_index_are_caught(monkeypatch):
    bad = _mutated(R.approximate_seed, "np.lexsort((members, d2))", "np.lexsort((-members, d2))")
    import oracle
    monkeypatch.setattr(oracle, "approximate_seed", bad)
    _fails(T_search.test_approximate_seed_hand_worked)


def test_knn_threshold_at_the_best_instead_of_the_kth_is_caught(monkeypatch):
    import oracle
    import tests.test_oracle_knn as T_knn
    bad = _mutated(R.exact_search_knn, "return best[-1][0] if len(best) >= k else np.inf",
                   "return best[0][0] if best else np.inf")
    monkeypatch.setattr(oracle, "exact_search_knn", bad)
    monkeypatch.setattr(T_knn, "exact_search_knn", bad)
    _fails(T_knn.test_twin_equals_definition, 10, "equal_count")
    _fails(T_search.test_knn_twin_refined_count_closed_form, 4)


def test_knn_twin_without_pruning_is_caught(monkeypatch):
    import oracle
    bad = _mutated(R.exact_search_knn, "lb[i] > kth() * (1.0 + 1e-9) + 1e-12", "False")
    monkeypatch.setattr(oracle, "exact_search_knn", bad)
    _fails(T_search.test_knn_twin_refined_count_closed_form, 4)


# ---- the ADS+ tree ----------------------------------------------------------------------------
def _ads_mutant(monkeypatch, old, new, fn_name="ads_tree"):
    """Replace ``oracle.ads.<fn_name>`` (and the name the tree tests import) by a copy of its source
    with one fragment changed."""
    import inspect
    import textwrap
    import oracle
    import oracle.ads as A
    import tests.test_oracle_ads as T_ads
    src = textwrap.dedent(inspect.getsource(getattr(A, fn_name)))
    assert old in src, old
    ns = dict(vars(A))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    bad = ns[fn_name]
    monkeypatch.setattr(A, fn_name, bad)
    monkeypatch.setattr(oracle, fn_name, bad)
    monkeypatch.setattr(T_ads, fn_name, bad)
    return T_ads


def test_ads_least_balanced_split_is_caught(monkeypatch):
    T = _ads_mutant(monkeypatch, "if best_gap is None or gap < best_gap:", "if best_gap is None or gap > best_gap:")
    _fails(T.test_hand_worked_tree)


def test_ads_ties_to_the_highest_segment_are_caught(monkeypatch):
    T = _ads_mutant(monkeypatch, "if best_gap is None or gap < best_gap:", "if best_gap is None or gap <= best_gap:")
    _fails(T.test_hand_worked_tree)


def test_ads_wrong_bit_is_caught(monkeypatch):
    import oracle.ads as A
    import tests.test_oracle_ads as T
    bad = lambda sym, card: (np.asarray(sym, np.int64) >> card) & 1      # counted from the wrong end
    monkeypatch.setattr(A, "next_bit", bad)
    _fails(T.test_hand_worked_tree)


def test_ads_unstable_partition_is_caught(monkeypatch):
    T = _ads_mutant(monkeypatch, "perm[a:b] = np.concatenate([zeros, ones_])",
                    "perm[a:b] = np.concatenate([zeros[::-1], ones_])")
    _fails(T.test_hand_worked_tree)


def test_ads_descent_without_detour_is_caught(monkeypatch):
    T = _ads_mutant(monkeypatch, "c = int(tree.child0[v]) + (1 - b)", "c = c", fn_name="ads_query_leaf")
    _fails(T.test_descent_into_an_empty_child_takes_the_other)
