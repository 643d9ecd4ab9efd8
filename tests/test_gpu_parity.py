"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bar: iSAX words, keys, orders and indices bit-exact; distances within 1e-5 relative of the
float64 oracle (they are in fact computed with the same float64 operation order, so the test
also checks bit equality of the squared distance); lower bounds within float32 rounding.
"""
import math

import numpy as np
import pytest

import synth
from oracle import (equal_count_bounds, isax, k64, lb_table, lower_bound_sq,
                    nn_bruteforce, paa, query_summary, root_key, root_offsets, seed_window,
                    sorted_order)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-5


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def small(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(100_000, 256, seed=0)
    Q, src, sig = synth.noisy_queries(X, 100, seed=0, sigma=0.1)
    Xd = torch.from_numpy(X).cuda()
    index = paris.build(Xd)
    ref_i, ref_d2, _ = oracle_native.nn_many(Q, X, threads=16)
    _, sym = oracle_native.summarise(X)
    return dict(X=X, Q=Q, src=src, Xd=Xd, Qd=torch.from_numpy(Q).cuda(), index=index,
                ref_i=ref_i, ref_d2=ref_d2, sym=sym)


def _check_answer(i, d, ref_i, ref_d2):
    assert i == int(ref_i)
    ref = math.sqrt(ref_d2)
    assert abs(d - ref) <= REL * ref + 1e-12
    assert d == ref  # same float64 operation order and a correctly rounded sqrt


# ---------------------------------------------------------------------------------- build
def test_sax_words_bit_exact(small):
    sax = small["index"].sax().cpu().numpy()
    assert np.array_equal(sax, small["sym"])


def test_leaf_order_and_root_offsets(small):
    perm, ks = sorted_order(small["sym"])
    idx = small["index"]
    assert np.array_equal(idx.sorted_keys().cpu().numpy().view(np.uint64), ks)
    assert np.array_equal(idx.sorted_positions().cpu().numpy().astype(np.int64), perm)
    assert np.array_equal(idx.root_offsets().cpu().numpy().astype(np.int64), root_offsets(ks))


def _adversarial(n, rng):
    from oracle import breakpoints
    L = n // 16
    b = breakpoints()
    rows = []
    for k in range(1, 256, 3):
        f = np.float32(b[k])
        for v in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
            rows.append(np.full(n, v, np.float32))
    rows.append(np.zeros(n, np.float32))                       # mean exactly beta_128 = 0
    rows.append(np.full(n, 1e30, np.float32))                  # beyond the last boundary
    rows.append(np.full(n, -1e30, np.float32))
    rows.append(np.full(n, 1e-40, np.float32))                 # subnormal values
    r = rng.standard_normal((64, n)).astype(np.float32)
    r[:, ::2] *= np.float32(1e6)
    r[:, 1::2] = -r[:, ::2] + np.float32(1e-3)                 # cancellation inside segments
    rows.extend(list(r))
    mixed = rng.standard_normal((64, n)).astype(np.float32)
    mixed[:, : L] = np.float32(b[200])                          # one segment near a boundary
    rows.extend(list(mixed))
    return np.stack(rows)


@pytest.mark.parametrize("n", [16, 48, 256, 1024, 2048])
def test_summaries_adversarial_and_lengths(n, oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    rng = np.random.default_rng(n)
    A = _adversarial(n, rng)
    W = synth.random_walks(4097 - A.shape[0], n, seed=n)     # ragged count (not a tile multiple)
    X = np.ascontiguousarray(np.concatenate([A, W]))
    index = paris.build(torch.from_numpy(X).cuda())
    _, sym = oracle_native.summarise(X)
    assert np.array_equal(index.sax().cpu().numpy(), sym)
    perm, ks = sorted_order(sym)
    assert np.array_equal(index.sorted_keys().cpu().numpy().view(np.uint64), ks)
    assert np.array_equal(index.sorted_positions().cpu().numpy().astype(np.int64), perm)
    index.close()


# ---------------------------------------------------------------------------------- query prep
def test_query_summaries_tables_and_window(small):
    idx = small["index"]
    perm, ks = sorted_order(small["sym"])
    off = root_offsets(ks)
    Qx, _, _ = synth.noisy_queries(small["X"], 20, seed=9, sigma=(0.01, 1.0))
    for q in list(small["Q"][:10]) + list(Qx):
        qs = query_summary(q)
        info = idx.query_info(torch.from_numpy(q).cuda(), tables=True)
        assert np.array_equal(np.array(info["paa"]).view(np.uint64), qs.paa.view(np.uint64))
        assert np.array_equal(np.array(info["sym"], np.uint8), qs.sym)
        assert info["root"] == qs.root and info["k64"] == qs.k64
        a, b = seed_window(qs, ks, 16, "root16", seed_cap=16384, off=off)
        assert (info["win_lo"], info["win_hi"]) == (a, b)
        t8 = info["table"].cpu().numpy().astype(np.float64)
        ref = lb_table(qs.paa, 16)
        up = np.nextafter(info["table"].cpu().numpy(), np.float32(np.inf)).astype(np.float64)
        assert np.all(t8 <= ref) and np.all(up > ref)             # rounded toward zero
        # each row is zero at the query's symbol and grows away from it, in float32: the run
        # envelopes of the scan bound every member of a run only under this property
        t32 = info["table"].cpu().numpy()
        for s_ in range(16):
            c = int(qs.sym[s_])
            assert t32[s_][c] == 0
            assert np.all(np.diff(t32[s_][:c + 1]) <= 0) and np.all(np.diff(t32[s_][c:]) >= 0)


def test_window_equal_count_mode(small):
    import paper_2009_00166_amd as paris
    idx = paris.build(small["Xd"], leaf_mode=1, n_leaves=64)
    perm, ks = sorted_order(small["sym"])
    for q in small["Q"][:20]:
        qs = query_summary(q)
        info = idx.query_info(torch.from_numpy(q).cuda())
        assert (info["win_lo"], info["win_hi"]) == seed_window(qs, ks, 16, "equal_count", n_leaves=64)
    idx.close()


# ---------------------------------------------------------------------------------- LB scan
def test_lb_scan_survivor_sandwich(small):
    idx = small["index"]
    S = small["sym"]
    for m in (0, 7, 33):
        q = small["Q"][m]
        ref = lower_bound_sq(paa(q), S, 16)
        for frac in (1e-4, 3e-3, 5e-2):
            thr = float(np.quantile(ref, frac))
            I, Bd, cnt, st = idx.lb_scan(torch.from_numpy(q).cuda(), thr)
            got = I.cpu().numpy().astype(np.int64)
            assert len(np.unique(got)) == len(got) == cnt
            strict = set(np.nonzero(ref < thr * (1 - REL))[0].tolist())
            loose = set(np.nonzero(ref <= thr * (1 + REL))[0].tolist())
            gs = set(got.tolist())
            assert strict <= gs <= loose
            bd = Bd.cpu().numpy().astype(np.float64)
            assert np.all(np.abs(bd - ref[got]) <= REL * ref[got] + 1e-6)
            assert np.all(bd <= ref[got] * (1 + 2e-6) + 1e-30)   # table terms are rounded down


@pytest.mark.parametrize("N", [33, 129, 4095, 10_007])
def test_lb_scan_ragged_sizes(N, oracle_native):
    """The scan's runs of 32 and lines of 4 runs with a partial last run and a partial last
    line (and fewer lines than a full grid): the survivors are still every series whose bound
    is within the threshold, as a scan of every word gives."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(N, 256, seed=N)
    idx = paris.build(torch.from_numpy(X).cuda())
    _, S = oracle_native.summarise(X)
    Qn, _, _ = synth.noisy_queries(X, 3, seed=N + 1, sigma=0.3)
    for q in list(Qn) + list(synth.fresh_walk_queries(2, 256, seed=N + 2)):
        ref = lower_bound_sq(paa(q), S, 16)
        for frac in (0.0, 0.01, 0.3, 1.0):
            thr = float(np.quantile(ref, frac))
            I, Bd, cnt, st = idx.lb_scan(torch.from_numpy(q).cuda(), thr)
            got = I.cpu().numpy().astype(np.int64)
            assert len(np.unique(got)) == len(got) == cnt
            strict = set(np.nonzero(ref < thr * (1 - REL))[0].tolist())
            loose = set(np.nonzero(ref <= thr * (1 + REL))[0].tolist())
            assert strict <= set(got.tolist()) <= loose
    idx.close()


def test_lb_scan_overflow_reports_count(small):
    idx = small["index"]
    q = torch.from_numpy(small["Q"][1]).cuda()
    I, Bd, cnt, st = idx.lb_scan(q, 1e9, capacity=5)
    assert cnt == small["X"].shape[0] and st == -5 and I.shape[0] == 5


# ---------------------------------------------------------------------------------- exact search
def test_exact_100_queries(small):
    idx = small["index"]
    for m in range(small["Q"].shape[0]):
        i, d, st = idx.query(small["Qd"][m], with_stats=True)
        _check_answer(i, d, small["ref_i"][m], small["ref_d2"][m])
        assert st["lb_survivors"] >= 1 and st["refined"] >= 1 and st["resolved"] >= 1
        assert st["seed_lo"] <= st["seed_hi"]


def test_exact_uneven_difficulty_and_fresh_walks(small, oracle_native):
    idx = small["index"]
    X = small["X"]
    Q1, _, _ = synth.noisy_queries(X, 30, seed=3, sigma=(0.01, 0.5))
    Q2 = synth.fresh_walk_queries(10, 256, seed=4)
    Q = np.concatenate([Q1, Q2])
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Qd = torch.from_numpy(Q).cuda()
    for m in range(Q.shape[0]):
        i, d = idx.query(Qd[m])
        _check_answer(i, d, ri[m], rd[m])


def test_private_bsf_copies_give_same_answers(small, oracle_native):
    """nb-ParIS+'s design (Section 3.3, the library's default): every distance worker (a lane
    group of the refine kernel) prunes with its own best-so-far copy; ParIS+'s shared
    best-so-far on request. Answers equal the oracle's in both modes; hard queries refine
    about as many rows or more with private copies; also without a seed (the copies then
    start at +inf)."""
    import paper_2009_00166_amd as paris
    idx, X = small["index"], small["X"]
    Q1, _, _ = synth.noisy_queries(X, 20, seed=5, sigma=0.5)
    Q = np.concatenate([Q1, synth.fresh_walk_queries(10, 256, seed=6), small["Q"][:10]])
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Qd = torch.from_numpy(Q).cuda()
    no_seed = paris.build(small["Xd"], seed_cap=0)
    refined = {}
    try:
        for shared in (True, False):
            idx.set_bsf_sharing(shared)
            total = 0
            for m in range(Q.shape[0]):
                i, d, st = idx.query(Qd[m], with_stats=True)
                _check_answer(i, d, ri[m], rd[m])
                total += st["refined"] if m < 30 else 0
            refined[shared] = total
        no_seed.set_bsf_sharing(False)
        for m in range(0, Q.shape[0], 7):
            i, d = no_seed.query(Qd[m])
            _check_answer(i, d, ri[m], rd[m])
    finally:
        idx.set_bsf_sharing(False)      # the default
        no_seed.close()
    # Not a theorem on the GPU (when the shared best-so-far falls depends on scheduling), so
    # only a loose check: private copies do not prune much better than the shared value.
    assert refined[False] >= 0.95 * refined[True]
    print(f"[parity] refined rows over 30 hard queries: shared {refined[True]}, private "
          f"{refined[False]}", flush=True)
    from paper_2009_00166_amd import _binding as B
    assert paris.load_library().paris_set_bsf_sharing(idx._h, 2) == B.PARIS_EINVAL


def test_seed_disabled_and_equal_count_give_same_answers(small):
    import paper_2009_00166_amd as paris
    no_seed = paris.build(small["Xd"], seed_cap=0)
    eq = paris.build(small["Xd"], leaf_mode=1, n_leaves=256)
    for m in range(0, 100, 9):
        i0, d0, st0 = no_seed.query(small["Qd"][m], with_stats=True)
        _check_answer(i0, d0, small["ref_i"][m], small["ref_d2"][m])
        assert st0["seed_index"] == -1 and st0["lb_survivors"] == small["X"].shape[0]
        i1, d1, st1 = eq.query(small["Qd"][m], with_stats=True)
        _check_answer(i1, d1, small["ref_i"][m], small["ref_d2"][m])
        assert st1["seed_lo"] < st1["seed_hi"]
    no_seed.close()
    eq.close()


def test_seed_is_a_true_distance_in_its_window(small):
    """Whatever members of the window the kernel refines (it samples the smallest-bound member of
    every 512 sorted positions), a valid seed is the true distance of a member of the window the
    oracle's approximate search reaches, never below the oracle's seed (the smallest distance over
    every member of that window, Section 3.3), and leaves the answer unchanged."""
    idx = small["index"]
    perm, ks = sorted_order(small["sym"])
    off = root_offsets(ks)
    from oracle import approximate_seed, ed_sq
    for m in range(0, 100, 11):
        q = small["Q"][m]
        i, d, st = idx.query(small["Qd"][m], with_stats=True)
        a, b = seed_window(query_summary(q), ks, 16, "root16", seed_cap=16384, off=off)
        assert (st["seed_lo"], st["seed_hi"]) == (a, b)
        members = perm[a:b]
        assert st["seed_index"] in set(members.tolist())
        own = math.sqrt(float(ed_sq(q, small["X"][st["seed_index"]])))
        assert abs(st["seed_dist"] - own) <= 1e-5 * own + 1e-6       # a true distance
        _, ref_d2 = approximate_seed(q, small["X"], members)
        assert st["seed_dist"] >= math.sqrt(ref_d2) * (1 - 1e-5) and st["seed_dist"] >= d * (1 - 1e-5)
        _check_answer(i, d, small["ref_i"][m], small["ref_d2"][m])


def test_ties_duplicates_and_degenerate_sizes(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(5000, 128, seed=11)
    for dst in (4000, 4999, 2500):
        X[dst] = X[123]
    X[77] = X[4500]
    Xd = torch.from_numpy(X).cuda()
    idx = paris.build(Xd, seed_cap=64)
    qs = [X[123].copy(), X[4500].copy(), (X[123] + np.float32(1e-3)).astype(np.float32), X[4999].copy()]
    for q in qs:
        i, d = idx.query(torch.from_numpy(q).cuda())
        ri, _, rdist = nn_bruteforce(q, X)
        assert i == ri and d == rdist
    assert idx.query(torch.from_numpy(X[4500].copy()).cuda())[0] == 77
    idx.close()
    for N in (1, 2, 17, 4097):
        Xs = synth.random_walks(N, 64, seed=N)
        ids = paris.build(torch.from_numpy(Xs).cuda())
        Qs, _, _ = synth.noisy_queries(Xs, 3, seed=1, sigma=0.3)
        for q in Qs:
            i, d = ids.query(torch.from_numpy(q).cuda())
            ri, _, rdist = nn_bruteforce(q, Xs)
            assert i == ri and d == rdist
        ids.close()


@pytest.mark.parametrize("n", [16, 48, 128, 512, 1024])
def test_exact_other_lengths(n, oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(6000, n, seed=n + 1)
    Q, _, _ = synth.noisy_queries(X, 10, seed=2, sigma=(0.05, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    idx = paris.build(torch.from_numpy(X).cuda())
    Qd = torch.from_numpy(Q).cuda()
    for m in range(10):
        i, d = idx.query(Qd[m])
        _check_answer(i, d, ri[m], rd[m])
    I, D = idx.query_batch(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    idx.close()


def test_batch_equals_reference(small):
    idx = small["index"]
    I, D, st = idx.query_batch(small["Qd"], with_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), small["ref_i"])
    ref = np.sqrt(small["ref_d2"])
    assert np.all(np.abs(D.cpu().numpy() - ref) <= REL * ref + 1e-12)
    assert st["lb_survivors"] >= 100


@pytest.mark.parametrize("mode", ["all", "scan", "sampled"])
def test_timing_modes_count_and_keep_answers(small, mode):
    """Event timing (all phases, the scan of every query, the scan of every 8th query) changes
    no answer and counts the calls it timed."""
    idx = small["index"]
    idx.set_timing(True, scan_only=(mode != "all"), sampled=(mode == "sampled"))
    for m in range(40):
        i, d = idx.query(small["Qd"][m])
        _check_answer(i, d, small["ref_i"][m], small["ref_d2"][m])
    ms, n = idx.timing()
    idx.set_timing(False)
    assert n == (5 if mode == "sampled" else 40)
    assert ms[1] > 0.0
    assert (ms[0] > 0.0) == (mode == "all")


# ---------------------------------------------------------------------------------- errors
def test_nonfinite_inputs_are_rejected():
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(3000, 64, seed=5)
    bad = X.copy()
    bad[1234, 17] = np.nan
    with pytest.raises(paris.ParisError) as e:
        paris.build(torch.from_numpy(bad).cuda())
    assert e.value.status == -1
    bad[1234, 17] = np.inf
    with pytest.raises(paris.ParisError):
        paris.build(torch.from_numpy(bad).cuda())
    idx = paris.build(torch.from_numpy(X).cuda())
    q = X[5].copy()
    q[3] = np.nan
    with pytest.raises(paris.ParisError) as e:
        idx.query(torch.from_numpy(q).cuda())
    assert e.value.status == -1
    Qb = np.stack([X[1], q, X[2]]).astype(np.float32)
    I, D = idx.query_batch(torch.from_numpy(Qb).cuda())
    torch.cuda.synchronize()
    I = I.cpu().numpy()
    assert I[0] == 1 and I[1] == -1 and I[2] == 2 and np.isnan(D.cpu().numpy()[1])
    # the handle stays valid after an error
    assert idx.query(torch.from_numpy(X[7].copy()).cuda())[0] == 7
    idx.close()
    idx.close()
