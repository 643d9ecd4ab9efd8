"""GPU parity at the full collection size the benchmark times (10,000,000 x 256, launch
configuration of the plain query path): sampled iSAX words, order properties of the whole leaf
order, and exact answers for a sample of queries checked by the brute-force C oracle."""
import math
import time

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_FULL, LEN = 10_000_000, 256


@pytest.fixture(scope="module")
def full(oracle_native):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_00166_amd as paris
    t0 = time.time()
    X = synth.random_walks(N_FULL, LEN, seed=0, threads=16)
    print(f"[scale] generated {N_FULL}x{LEN} in {time.time() - t0:.1f}s", flush=True)
    Xd = torch.from_numpy(X).cuda()
    index = paris.build(Xd)
    torch.cuda.synchronize()
    print(f"[scale] built index at {time.time() - t0:.1f}s", flush=True)
    yield dict(X=X, Xd=Xd, index=index)
    index.close()


def test_sampled_words_and_order(full, oracle_native):
    X, index = full["X"], full["index"]
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(N_FULL, 200_000, replace=False))
    _, sym = oracle_native.summarise(X[rows])
    sax = index.sax()
    got = sax[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.array_equal(got, sym)
    keys = index.sorted_keys()
    ku = keys.cpu().numpy().view(np.uint64)
    assert np.all(ku[1:] >= ku[:-1])
    perm = index.sorted_positions().cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(N_FULL))
    same = ku[1:] == ku[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])          # stable: ties keep position order
    from oracle import k64
    sample = rng.choice(N_FULL, 50_000, replace=False)
    _, s2 = oracle_native.summarise(X[perm[sample]])
    assert np.array_equal(k64(s2), ku[sample])
    roff = index.root_offsets().cpu().numpy().astype(np.int64)
    assert roff[0] == 0 and roff[-1] == N_FULL and np.all(np.diff(roff) >= 0)
    r = (ku >> np.uint64(48)).astype(np.int64)
    assert np.array_equal(np.bincount(r, minlength=65536), np.diff(roff))


def test_sampled_exact_answers(full, oracle_native):
    X, index = full["X"], full["index"]
    Q1, _, _ = synth.noisy_queries(X, 12, seed=0, sigma=0.1)
    Q2, _, _ = synth.noisy_queries(X, 4, seed=1, sigma=(0.01, 0.5))
    Q = np.concatenate([Q1, Q2])
    t0 = time.time()
    ri, rd, used = oracle_native.nn_many(Q, X, threads=16)
    print(f"[scale] oracle brute force {Q.shape[0]} queries in {time.time() - t0:.1f}s on {used} threads",
          flush=True)
    Qd = torch.from_numpy(Q).cuda()
    for m in range(Q.shape[0]):
        i, d = index.query(Qd[m])
        ref = math.sqrt(rd[m])
        assert i == int(ri[m]), (m, i, int(ri[m]))
        assert abs(d - ref) <= 1e-5 * ref
    I, D = index.query_batch(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)


def test_batched_pipeline_at_scale(full, oracle_native):
    """The batched pipeline (bfloat16 MFMA screen) at 10M x 256, in the launch configuration the
    benchmark times (chunks of 4096), on a sample of uneven-difficulty queries."""
    X, index = full["X"], full["index"]
    index.attach_batch(max_batch=4096)
    Q, _, _ = synth.noisy_queries(X, 48, seed=2, sigma=(0.01, 0.5))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    I, D, st = index.query_batch(torch.from_numpy(Q).cuda(), with_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri)
    ref = np.sqrt(rd)
    assert np.all(np.abs(D.cpu().numpy() - ref) <= 1e-5 * ref)
    print(f"[scale] batched: {st['lb_survivors']} screen survivors, {st['resolved']} fallbacks", flush=True)


def _oracle_sample(sig, count, hardest, seed):
    """Indices of the queries checked by brute force: the ``hardest`` with the largest noise and
    ``count - hardest`` others at random, ascending."""
    order = np.argsort(-np.asarray(sig), kind="stable")
    top = order[:hardest]
    rest = np.random.default_rng(seed).choice(order[hardest:], count - hardest, replace=False)
    return np.sort(np.concatenate([top, rest]))


def test_full_batch_at_scale(full, oracle_native):
    """One whole batch of 4096 uneven-difficulty queries at 10M x 256, the batch size and tuned
    launch shape the benchmark times: the brute-force oracle's answers on 256 of its queries
    (the 64 with the largest noise, the hardest to prune, and 192 drawn at random); for every
    query, the returned distance is bit-identical to the oracle's float64 distance to the
    returned series and no larger than the distance to the series the query was made from."""
    X, index = full["X"], full["index"]
    index.attach_batch(max_batch=4096)
    M = 4096
    Q, src, sig = synth.noisy_queries(X, M, seed=3, sigma=(0.01, 0.5))
    I, D, st = index.query_batch(torch.from_numpy(Q).cuda(), with_stats=True)
    torch.cuda.synchronize()
    I, D = I.cpu().numpy(), D.cpu().numpy()
    pick = _oracle_sample(sig, 256, 64, seed=3)
    t0 = time.time()
    ri, rd, _ = oracle_native.nn_many_blocked(Q[pick], X, threads=16)
    print(f"[scale] oracle: {len(pick)} of the batch's queries in {time.time() - t0:.1f}s", flush=True)
    assert np.array_equal(I[pick], ri)
    assert np.array_equal(D[pick], np.sqrt(rd))
    assert np.all((I >= 0) & (I < N_FULL))
    for m in range(M):
        d_ret, d_src = oracle_native.ed2_at(Q[m], X, [I[m], src[m]])
        assert D[m] == math.sqrt(d_ret), m
        assert d_ret <= d_src, m
    print(f"[scale] full batch: {st['lb_survivors']} screen survivors, {st['refined']} re-scored, "
          f"{st['resolved']} fallbacks", flush=True)


def test_shared_and_private_best_so_far_at_scale(full, oracle_native):
    """Both best-so-far modes of the refine kernel (private copies per lane group, the default,
    and ParIS+'s shared value) at 10M x 256 on hard and new-walk queries: identical answers,
    equal to the brute-force oracle's."""
    X, index = full["X"], full["index"]
    Qh, _, _ = synth.noisy_queries(X, 8, seed=5, sigma=0.5)
    Q = np.ascontiguousarray(np.concatenate([Qh, synth.fresh_walk_queries(4, LEN, seed=6)]))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Qd = torch.from_numpy(Q).cuda()
    try:
        for shared in (True, False):
            index.set_bsf_sharing(shared)
            for m in range(Q.shape[0]):
                i, d = index.query(Qd[m])
                ref = math.sqrt(rd[m])
                assert i == int(ri[m]), (shared, m, i, int(ri[m]))
                assert abs(d - ref) <= 1e-5 * ref
    finally:
        index.set_bsf_sharing(False)


def test_knn_at_scale(full, oracle_native):
    """Exact k-NN (k = 10 and 64) at 10M x 256 on easy, hard and new-walk queries against the
    k-NN by definition: the C oracle's float64 distances to every series, ordered by (distance,
    index)."""
    from concurrent.futures import ThreadPoolExecutor
    X, index = full["X"], full["index"]
    Qe, _, _ = synth.noisy_queries(X, 3, seed=11, sigma=0.1)
    Qh, _, _ = synth.noisy_queries(X, 2, seed=12, sigma=0.5)
    Q = np.ascontiguousarray(np.concatenate([Qe, Qh, synth.fresh_walk_queries(1, LEN, seed=13)]))
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=Q.shape[0]) as ex:
        d2s = list(ex.map(lambda q: oracle_native.ed2(q, X), Q))
    print(f"[scale] k-NN oracle distances for {Q.shape[0]} queries in {time.time() - t0:.1f}s", flush=True)
    Qd = torch.from_numpy(Q).cuda()
    for m in range(Q.shape[0]):
        order = np.lexsort((np.arange(N_FULL), d2s[m]))[:64]
        for k in (10, 64):
            idx, dist, st = index.query_knn(Qd[m], k, with_stats=True)
            assert np.array_equal(idx, order[:k]), (m, k)
            assert np.array_equal(dist, np.sqrt(d2s[m][order[:k]])), (m, k)
        print(f"[scale] k-NN query {m}: {st['lb_survivors']} LB survivors, {st['refined']} refined", flush=True)
