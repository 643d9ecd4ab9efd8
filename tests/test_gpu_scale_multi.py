"""GPU parity of the mixed-length workload at its full sizes: three collections resident together
(100,000,000 x 128, 20,000,000 x 512 and 5,000,000 x 1024 random walks) and one mixed batch of
2048 queries (collection drawn uniformly, noise sigma ~ U[0.05, 0.5]) through
paris_query_batch_multi, in the launch configuration the benchmark's mixed-length section times
(one index per collection, batch workspaces of 2048, tuned screen per length). 64 queries of every
collection (its 16 noisiest, 48 at random) are checked by the brute-force C oracle; every answer's distance equals the
oracle's float64 distance to the returned series and is no larger than the distance to the
series the query was made from. The per-query path over the 100M collection (whose 1.6 GB iSAX
array no cache holds) is checked on a few queries too."""
import math
import time

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SPECS = [(100_000_000, 128, 0), (20_000_000, 512, 1), (5_000_000, 1024, 2)]
BATCH = 2048


@pytest.fixture(scope="module")
def mixed(oracle_native):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_00166_amd as paris
    t0 = time.time()
    Xs, idxs = [], []
    for N, n, seed in SPECS:
        X = synth.random_walks(N, n, seed=seed, threads=16)
        ix = paris.build(torch.from_numpy(X).cuda())
        ix.attach_batch(max_batch=BATCH)
        Xs.append(X)
        idxs.append(ix)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(7)))
    which = rng.integers(0, 3, size=BATCH)
    Qs, srcs, sigs = [], [], []
    for c, X in enumerate(Xs):
        Q, src, sig = synth.noisy_queries(X, int((which == c).sum()), seed=10 + c, sigma=(0.05, 0.5))
        Qs.append(Q)
        srcs.append(src)
        sigs.append(sig)
    print(f"[multi] three collections generated, built and attached in {time.time() - t0:.1f}s", flush=True)
    yield dict(Xs=Xs, idxs=idxs, Qs=Qs, srcs=srcs, sigs=sigs)
    for ix in idxs:
        ix.close()


def test_mixed_batch_at_full_size(mixed, oracle_native):
    import paper_2009_00166_amd as paris
    Xs, idxs, Qs, srcs = mixed["Xs"], mixed["idxs"], mixed["Qs"], mixed["srcs"]
    outs, st = paris.query_batch_multi(idxs, [torch.from_numpy(Q).cuda() for Q in Qs], with_stats=True)
    torch.cuda.synchronize()
    for c, (I, D) in enumerate(outs):
        X, Q, src = Xs[c], Qs[c], srcs[c]
        I, D = I.cpu().numpy(), D.cpu().numpy()
        assert np.all((I >= 0) & (I < X.shape[0]))
        # 64 of the collection's queries by brute force: the 16 with the largest noise, 48 at random
        order = np.argsort(-mixed["sigs"][c], kind="stable")
        pick = np.sort(np.concatenate([order[:16], np.random.default_rng(c).choice(order[16:], 48, replace=False)]))
        t0 = time.time()
        ri, rd, _ = oracle_native.nn_many_blocked(Q[pick], X, threads=16)
        print(f"[multi] oracle: {len(pick)} queries of {X.shape[0]} x {X.shape[1]} in {time.time() - t0:.1f}s",
              flush=True)
        assert np.array_equal(I[pick], ri), c
        assert np.array_equal(D[pick], np.sqrt(rd)), c
        for m in range(Q.shape[0]):
            d_ret, d_src = oracle_native.ed2_at(Q[m], X, [I[m], src[m]])
            assert D[m] == math.sqrt(d_ret), (c, m)
            assert d_ret <= d_src, (c, m)
    print(f"[multi] {st['lb_survivors']} screen survivors, {st['refined']} re-scored, "
          f"{st['resolved']} fallbacks", flush=True)


def test_per_query_path_over_100m(mixed, oracle_native):
    X, ix, Q = mixed["Xs"][0], mixed["idxs"][0], mixed["Qs"][0]
    k = 3
    ri, rd, _ = oracle_native.nn_many(Q[-k:], X, threads=16)
    Qd = torch.from_numpy(Q[-k:]).cuda()
    for m in range(k):
        i, d = ix.query(Qd[m])
        assert i == int(ri[m]), (m, i, int(ri[m]))
        assert d == math.sqrt(rd[m])
