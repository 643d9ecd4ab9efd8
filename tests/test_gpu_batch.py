"""GPU parity of the batched pipeline (bfloat16 MFMA screen + float32 re-score + float64 resolve)
against the oracle, and the screen's certified error bound."""
import math

import numpy as np
import pytest

import synth
from oracle import nn_bruteforce

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gamma(k, u):
    return k * u / (1 - k * u)


def _screen_margin(n, np_):
    """The bound of the screen as documented: |d~^2 - d^2| <= c (qn + xn)."""
    ub = 2.0 ** -8
    c = (2 * ub + ub * ub) + 6 * _gamma(np_ + 48, 2.0 ** -23) * (1 + ub) ** 2 + 2 * _gamma(n, 2.0 ** -24) \
        + 16 * 2.0 ** -24
    return 1.05 * c + 32 * 2.0 ** -24


@pytest.fixture(scope="module")
def coll(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(100_000, 256, seed=0)
    Xd = torch.from_numpy(X).cuda()
    index = paris.build(Xd)
    index.attach_batch(max_batch=512)
    return dict(X=X, Xd=Xd, index=index)


def test_screen_dot_error_bound_1e7_pairs(coll):
    """Certified bound of the bfloat16 screen on >= 10^7 (query, series) pairs, plus
    adversarial pairs (identical, opposite and scaled rows)."""
    X = coll["X"]
    idx = coll["index"]
    rng = np.random.default_rng(0)
    Q, _, _ = synth.noisy_queries(X, 400, seed=5, sigma=(0.0, 1.0))
    adv = np.stack([X[0], -X[1], X[2] * np.float32(3.0), X[3], np.zeros(256, np.float32) + np.float32(1e-3)])
    Qa = np.ascontiguousarray(np.concatenate([Q, adv, rng.standard_normal((107, 256)).astype(np.float32)]))
    dots = idx.screen_dots(torch.from_numpy(Qa).cuda()).cpu().numpy().astype(np.float64)
    assert dots.shape == (512, 100_000)
    Xf = X.astype(np.float64)
    Qf = Qa.astype(np.float64)
    exact = Qf @ Xf.T
    absum = np.abs(Qf) @ np.abs(Xf).T
    ub = 2.0 ** -8
    bound = (2 * ub + ub * ub) * absum + _gamma(256 + 16, 2.0 ** -23) * (1 + ub) ** 2 * absum + 1e-30
    err = np.abs(dots - exact)
    assert np.all(err <= bound), float((err / np.maximum(bound, 1e-300)).max())
    # the squared-distance margin used by the screen
    qn = (Qf ** 2).sum(1)[:, None]
    xn = (Xf ** 2).sum(1)[None, :]
    d2 = qn + xn - 2 * exact
    d2_screen = qn + xn - 2 * dots
    c = _screen_margin(256, 256)
    assert np.all(np.abs(d2_screen - d2) <= c * (qn + xn))
    # the bound is not vacuous: bfloat16 errors are a visible fraction of it
    assert np.max(err / np.maximum(bound, 1e-300)) > 0.01


def test_batch_answers_match_oracle(coll, oracle_native):
    X, idx = coll["X"], coll["index"]
    Q1, _, _ = synth.noisy_queries(X, 400, seed=1, sigma=(0.01, 0.5))
    Q2 = synth.fresh_walk_queries(112, 256, seed=2)
    Q = np.ascontiguousarray(np.concatenate([Q1, Q2]))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    I, D, st = idx.query_batch(torch.from_numpy(Q).cuda(), with_stats=True)
    torch.cuda.synchronize()
    I = I.cpu().numpy()
    D = D.cpu().numpy()
    assert np.array_equal(I, ri)
    ref = np.sqrt(rd)
    assert np.all(np.abs(D - ref) <= 1e-5 * ref + 1e-12)
    assert np.array_equal(D, ref)  # same float64 operation order, correctly rounded sqrt
    assert st["lb_survivors"] >= Q.shape[0]


def test_batch_chunks_and_partial_chunk(coll, oracle_native):
    """1,100 queries with max_batch 512: two graph-launched chunks and a partial one."""
    X, idx = coll["X"], coll["index"]
    Q, _, _ = synth.noisy_queries(X, 1100, seed=3, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    I, D = idx.query_batch(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)


def test_batch_ties_fallback_nan_and_equal_count(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(20_000, 256, seed=7)
    for dst in (500, 900, 1200, 5000, 7000, 9000, 11000, 19999):
        X[dst] = X[321]                       # nine identical rows: the band list overflows
    X[77] = X[4500]
    Xd = torch.from_numpy(X).cuda()
    Q = np.stack([X[321], X[5000], X[4500], (X[321] + np.float32(1e-3)).astype(np.float32), X[10]]).astype(np.float32)
    bad = X[11].copy()
    bad[7] = np.nan
    Qn = np.ascontiguousarray(np.concatenate([Q, bad[None, :], X[12:13]]))
    for kw in ({}, {"leaf_mode": 1, "n_leaves": 64}):
        idx = paris.build(Xd, **kw)
        idx.attach_batch(max_batch=64)
        I, D, st = idx.query_batch(torch.from_numpy(Qn).cuda(), with_stats=True)
        torch.cuda.synchronize()
        I = I.cpu().numpy()
        D = D.cpu().numpy()
        for m in range(5):
            ri, _, rdist = nn_bruteforce(Q[m], X)
            assert I[m] == ri and D[m] == rdist
        assert I[0] == 321 and I[1] == 321 and I[2] == 77
        assert I[5] == -1 and np.isnan(D[5]) and I[6] == 12
        assert st["resolved"] >= 2            # the tied queries went to the per-query path
        idx.close()


@pytest.mark.parametrize("n", [64, 128])
def test_batch_other_lengths(n, oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(30_000, n, seed=n)
    Q, _, _ = synth.noisy_queries(X, 200, seed=4, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=256)
    I, D = idx.query_batch(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    assert np.all(np.abs(D.cpu().numpy() - np.sqrt(rd)) <= 1e-5 * np.sqrt(rd) + 1e-12)
    idx.close()


@pytest.mark.parametrize("n", [272, 512, 1024, 2048])
def test_long_series_screened_on_segment_means(n, oracle_native):
    """Series longer than 256 points are screened on segment means (a lower bound of the
    distance); answers stay exact and the screen still prunes."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    N = 6000 if n < 2048 else 3000
    X = synth.random_walks(N, n, seed=9)
    Q, _, _ = synth.noisy_queries(X, 40, seed=4, sigma=(0.05, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=32)
    I, D, st = idx.query_batch(torch.from_numpy(Q).cuda(), with_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    assert np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    assert st["lb_survivors"] < 0.2 * N * len(Q)      # the projected screen prunes most pairs
    assert st["refined"] <= st["lb_survivors"]
    print(f"n={n}: screen survivors {st['lb_survivors']}, rows re-scored {st['refined']}", flush=True)
    idx.close()


def test_projected_screen_bound_and_lower_bound():
    """n = 2048 is screened on means of 4-point segments: the bfloat16 dot products obey the
    screen's bound for the projected vectors, and 4 |p_q - p_x|^2 <= |q - x|^2."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    n, P = 2048, 4
    X = synth.random_walks(3000, n, seed=13)
    Q, _, _ = synth.noisy_queries(X, 64, seed=14, sigma=(0.0, 1.0))
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=64)
    dots = idx.screen_dots(torch.from_numpy(Q).cuda()).cpu().numpy().astype(np.float64)
    px = X.astype(np.float64).reshape(3000, n // P, P).mean(axis=2)
    pq = Q.astype(np.float64).reshape(64, n // P, P).mean(axis=2)
    exact = pq @ px.T
    qn = (pq ** 2).sum(1)[:, None]
    xn = (px ** 2).sum(1)[None, :]
    c = _screen_margin(n // P, n // P)
    assert np.all(np.abs((qn + xn - 2 * dots) - (qn + xn - 2 * exact)) <= c * (qn + xn))
    d2 = ((Q.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :]) ** 2).sum(-1)
    assert np.all(P * (qn + xn - 2 * exact) <= d2 * (1 + 1e-12) + 1e-9)
    idx.close()


@pytest.mark.parametrize("n", [96, 160, 272, 400, 512])
def test_screen_dot_error_bound_row_widths(n):
    """The 32-wide screen's rows of np = roundup(n, 32) dimensions (np / 8 = 12, 20, 36, 52 or
    64 chunks of 16 bytes, swizzled in LDS): the bound on every (query, series) pair."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(4000, n, seed=15)
    Q, _, _ = synth.noisy_queries(X, 64, seed=16, sigma=(0.0, 1.0))
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=64)
    dots = idx.screen_dots(torch.from_numpy(Q).cuda()).cpu().numpy().astype(np.float64)
    Xf, Qf = X.astype(np.float64), Q.astype(np.float64)
    exact = Qf @ Xf.T
    qn = (Qf ** 2).sum(1)[:, None]
    xn = (Xf ** 2).sum(1)[None, :]
    np_ = (n + 31) // 32 * 32
    c = _screen_margin(n, np_)
    assert np.all(np.abs(2 * dots - 2 * exact) <= c * (qn + xn))
    idx.close()


def test_query_batch_multi_mixed_lengths(oracle_native):
    """Three collections of lengths 128, 512 and 1024 in one call, each with its own tuned
    screen; answers identical to the oracle."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    specs = [(30_000, 128, 1), (8_000, 512, 2), (4_000, 1024, 3)]
    idxs, Qs, refs = [], [], []
    for N, n, seed in specs:
        X = synth.random_walks(N, n, seed=seed)
        m = {128: 120, 512: 80, 1024: 56}[n]
        Q, _, _ = synth.noisy_queries(X, m, seed=seed + 10, sigma=(0.05, 0.5))
        ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
        ix = paris.build(torch.from_numpy(X).cuda())
        ix.attach_batch(max_batch=64)     # chunks of 64 plus a partial chunk per collection
        idxs.append(ix)
        Qs.append(torch.from_numpy(Q).cuda())
        refs.append((ri, np.sqrt(rd)))
    outs, st = paris.query_batch_multi(idxs, Qs, with_stats=True)
    torch.cuda.synchronize()
    for (I, D), (ri, rdist) in zip(outs, refs):
        assert np.array_equal(I.cpu().numpy(), ri)
        assert np.array_equal(D.cpu().numpy(), rdist)
    assert st["lb_survivors"] > 0
    for ix in idxs:
        ix.close()


SCREEN_SHAPES = ["32,2,16", "64,2,16", "32,4,16", "64,4,16", "32,2,32", "64,1,32", "32,1,32", "64,2,32"]


def test_every_screen_shape_gives_exact_answers(oracle_native, monkeypatch):
    """Every launch shape the screen tuner may choose (both MFMA forms) answers exactly."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(30_000, 256, seed=17)
    Q, _, _ = synth.noisy_queries(X, 150, seed=18, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    idx = paris.build(Xd)
    for shape in SCREEN_SHAPES:
        monkeypatch.setenv("PARIS_SCREEN_SHAPE", shape)
        idx.attach_batch(max_batch=128)      # a full chunk (graph) and a partial one
        I, D = idx.query_batch(Qd)
        torch.cuda.synchronize()
        assert np.array_equal(I.cpu().numpy(), ri), shape
        assert np.array_equal(D.cpu().numpy(), np.sqrt(rd)), shape
    idx.close()


def test_block_bound_prunes_and_changes_no_answer(oracle_native, monkeypatch):
    """The block bound (iSAX lower bound of each query against the symbol envelope of runs of
    consecutive series in leaf order, Section 3.3.1) keeps the screen away from most
    (query, run) pairs, and every answer stays the oracle's: the same with the bound off."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(200_000, 256, seed=21)
    Q, _, _ = synth.noisy_queries(X, 300, seed=22, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    idx = paris.build(Xd)
    monkeypatch.setenv("PARIS_SCREEN_SHAPE", "32,2,32")   # the same work items either way
    res = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("PARIS_BLOCK_LB", flag)
        idx.attach_batch(max_batch=256)
        I, D = idx.query_batch(Qd)
        torch.cuda.synchronize()
        res[flag] = (I.cpu().numpy(), D.cpu().numpy(), idx.screen_tiles(reset=True))
    for flag, (I, D, _) in res.items():
        assert np.array_equal(I, ri), flag
        assert np.array_equal(D, np.sqrt(rd)), flag
    run0, dense0 = res["0"][2]
    run1, dense1 = res["1"][2]
    assert run0 == dense0 > 0
    assert dense1 == dense0
    print(f"screen tiles with the block bound: {run1} of {dense1} ({run1 / dense1:.3f})")
    assert run1 < 0.75 * dense1
    idx.close()


@pytest.mark.parametrize("shape", ["32,2,32", "64,1,32"])
def test_block_bound_over_several_query_groups(shape, oracle_native, monkeypatch):
    """A chunk of 4,500 queries: the 32-wide screen walks its alive lists in groups (4,096 or
    2,048 queries), with a ragged last group and series tail."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(8_000, 256, seed=25)
    Q, _, _ = synth.noisy_queries(X, 4500, seed=26, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    idx = paris.build(Xd)
    monkeypatch.setenv("PARIS_SCREEN_SHAPE", shape)
    idx.attach_batch(max_batch=4500)
    I, D = idx.query_batch(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    assert np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    run, dense = idx.screen_tiles()
    assert 0 < run < dense
    idx.close()


@pytest.mark.parametrize("item_series", [128, 256])
def test_block_bound_bits_match_oracle(item_series, oracle_native):
    """The block bound's alive bits against the oracle's run bound (block_lower_bound_sq over the
    oracle's own leaf order, runs of 128 or 256 sorted positions with a ragged last run): every
    pair clearly within its threshold is kept, every pair clearly beyond it is dropped; only
    pairs within the kernel's margins (below 1e-4 relative) of the threshold may go either way.
    Thresholds: 1.3 times each query's exact nearest squared distance."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    from oracle import reference as R
    N, n, M = 20_000, 256, 100
    X = synth.random_walks(N, n, seed=27)
    Q, _, _ = synth.noisy_queries(X, M, seed=28, sigma=(0.01, 0.5))
    _, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    U = (rd * 1.3).astype(np.float32)
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=128)
    bits = idx.block_bound_bits(torch.from_numpy(Q).cuda(), torch.from_numpy(U).cuda(), item_series)
    bits = bits.cpu().numpy().view(np.uint64)
    n_items = (N + item_series - 1) // item_series
    assert bits.shape == (n_items, 2)
    perm, _ = R.sorted_order(R.isax(R.paa(X)))
    syms = R.isax(R.paa(X))[perm]
    L = n // 16
    decided = kept = 0
    for q in range(M):
        qp = R.paa(Q[q])
        for it in range(n_items):
            lb = R.block_lower_bound_sq(qp, syms[it * item_series:(it + 1) * item_series], L)
            g = int((int(bits[it, q >> 6]) >> (q & 63)) & 1)
            if lb <= float(U[q]) * (1 - 1e-4):
                assert g == 1, (q, it, lb, float(U[q]))
                decided += 1
                kept += 1
            elif lb > float(U[q]) * (1 + 1e-3):
                assert g == 0, (q, it, lb, float(U[q]))
                decided += 1
    assert decided >= 0.99 * M * n_items
    assert 0 < kept < M * n_items            # the bound keeps some runs and drops others
    assert np.all((bits[:, 1] >> np.uint64(M - 64)) == 0)   # no bits past the last query
    idx.close()


@pytest.mark.parametrize("N", [1, 5, 31, 33, 127, 129, 300, 1000])
def test_batch_tiny_and_ragged_collections(N, oracle_native):
    """Collections smaller than one symbol-envelope run, one work item or one tile, and sizes
    just past those boundaries: the block bound's partial runs and items, the screen's partial
    series tiles and the batched answers against the oracle."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(N, 256, seed=40 + N)
    Q, _, _ = synth.noisy_queries(X, 37, seed=41, sigma=(0.01, 0.5))
    Q = np.ascontiguousarray(np.concatenate([Q, synth.fresh_walk_queries(3, 256, seed=42)]))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=32)            # a full chunk and a partial one
    I, D = idx.query_batch(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    assert np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    idx.close()


def test_rescore_skips_candidates_beyond_the_screened_upper_bound(oracle_native):
    """The re-score skips screen survivors whose screened lower bound exceeds the query's
    certified upper bound from the other survivors (reported as refined < screen survivors),
    and every answer stays the oracle's, hard queries and near-ties included."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(200_000, 256, seed=31)
    for dst in (1000, 2000, 3000):
        X[dst] = X[55]                                   # exact ties
    Q1, _, _ = synth.noisy_queries(X, 300, seed=32, sigma=(0.2, 0.5))
    Q = np.ascontiguousarray(np.concatenate([Q1, X[55:56], (X[55] + np.float32(1e-4)).astype(np.float32)[None, :]]))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    idx = paris.build(torch.from_numpy(X).cuda())
    idx.attach_batch(max_batch=512)
    I, D, st = idx.query_batch(torch.from_numpy(Q).cuda(), with_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    assert np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    print(f"screen survivors {st['lb_survivors']}, re-scored {st['refined']}")
    assert 0 < st["refined"] < st["lb_survivors"]
    idx.close()
