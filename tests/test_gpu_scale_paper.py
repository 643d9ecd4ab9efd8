"""GPU parity at the paper's own scale and query workload: 100,000,000 random walks of length
256 (102.4 GB of float32, inside the 50-250 GB range of the paper's query experiments, Section
4), queried with new random walks as the paper's query sets are (Section 4, datasets), plus a
few dataset-series-plus-noise queries. The per-query path (paris_query_exact) and one batch
through paris_query_batch are checked against the brute-force C oracle; at this size the iSAX
array (1.6 GB) no longer fits the chip's last-level cache, so the scan streams from HBM."""
import math
import time

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_FULL, LEN = 100_000_000, 256


@pytest.fixture(scope="module")
def paper_full(oracle_native):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_00166_amd as paris
    torch.cuda.empty_cache()
    t0 = time.time()
    X = synth.random_walks(N_FULL, LEN, seed=0, threads=16)
    print(f"[scale100] generated {N_FULL}x{LEN} in {time.time() - t0:.1f}s", flush=True)
    Xd = torch.from_numpy(X).cuda()
    index = paris.build(Xd)
    torch.cuda.synchronize()
    print(f"[scale100] built index at {time.time() - t0:.1f}s", flush=True)
    Qf = synth.fresh_walk_queries(48, LEN, seed=7)
    Qn, _, _ = synth.noisy_queries(X, 16, seed=8, sigma=(0.05, 0.5))
    Q = np.ascontiguousarray(np.concatenate([Qf, Qn]))
    t1 = time.time()
    ri, rd, used = oracle_native.nn_many_blocked(Q, X, threads=16)
    print(f"[scale100] oracle brute force {Q.shape[0]} queries in {time.time() - t1:.1f}s on {used} "
          "threads", flush=True)
    yield dict(X=X, Xd=Xd, index=index, Q=Q, ri=ri, rd=rd)
    index.close()
    del Xd
    torch.cuda.empty_cache()


def test_sampled_words_and_leaf_order_at_100m(paper_full, oracle_native):
    X, index = paper_full["X"], paper_full["index"]
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(N_FULL, 100_000, replace=False))
    _, sym = oracle_native.summarise(X[rows])
    got = index.sax()[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.array_equal(got, sym)
    ku = index.sorted_keys().cpu().numpy().view(np.uint64)
    assert np.all(ku[1:] >= ku[:-1])
    perm = index.sorted_positions().cpu().numpy()
    assert np.all(np.bincount(perm.astype(np.int64), minlength=N_FULL) == 1)   # a permutation
    roff = index.root_offsets().cpu().numpy().astype(np.int64)
    assert roff[0] == 0 and roff[-1] == N_FULL and np.all(np.diff(roff) >= 0)


def test_exact_answers_fresh_walk_queries_at_100m(paper_full):
    index, Q, ri, rd = paper_full["index"], paper_full["Q"], paper_full["ri"], paper_full["rd"]
    Qd = torch.from_numpy(Q).cuda()
    for m in range(Q.shape[0]):
        t0 = time.time()
        i, d, st = index.query(Qd[m], with_stats=True)
        ref = math.sqrt(rd[m])
        print(f"[scale100] query {m}: {(time.time() - t0) * 1e3:.1f} ms, {st['lb_survivors']} LB "
              f"survivors, {st['refined']} refined", flush=True)
        assert i == int(ri[m]), (m, i, int(ri[m]))
        assert abs(d - ref) <= 1e-5 * ref


def test_batched_fresh_walk_queries_at_100m(paper_full, oracle_native):
    X, index, Q, ri, rd = (paper_full[k] for k in ("X", "index", "Q", "ri", "rd"))
    M = 512
    extra = synth.fresh_walk_queries(M - Q.shape[0], LEN, seed=9)
    Qb = np.ascontiguousarray(np.concatenate([Q, extra]))
    index.attach_batch(max_batch=M)
    I, D, st = index.query_batch(torch.from_numpy(Qb).cuda(), with_stats=True)
    torch.cuda.synchronize()
    I, D = I.cpu().numpy(), D.cpu().numpy()
    k = Q.shape[0]
    assert np.array_equal(I[:k], ri)
    assert np.all(np.abs(D[:k] - np.sqrt(rd)) <= 1e-5 * np.sqrt(rd))
    assert np.all((I >= 0) & (I < N_FULL))
    for m in range(M):          # every answer's distance is the float64 distance to its series
        assert D[m] == math.sqrt(oracle_native.ed2_at(Qb[m], X, [I[m]])[0]), m
    print(f"[scale100] batch of {M}: {st['lb_survivors']} screen survivors, {st['refined']} "
          f"re-scored, {st['resolved']} fallbacks", flush=True)
