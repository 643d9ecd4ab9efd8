"""GPU parity of the exact k-NN (paris_query_knn, through the C ABI) against the oracle's k-NN by
definition (knn_bruteforce: the k smallest (float64 squared distance, index) pairs in that
order): indices bit-exact and in order, distances bit-identical (same float64 operation order,
correctly rounded sqrt), for k = 1, 10 and 64 on every query of the 100,000 x 256 workload
(noisy, hard and new-walk queries), both leaf modes and the seed disabled; a three-way exact tie;
k beyond the collection size; k = 1 against the 1-NN entry point."""
import math

import numpy as np
import pytest

import synth
from oracle import knn_bruteforce

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def coll():
    _need_gpu()
    X = synth.random_walks(100_000, 256, seed=0)
    Qn, _, _ = synth.noisy_queries(X, 100, seed=0, sigma=0.1)
    Qh, _, _ = synth.noisy_queries(X, 12, seed=1, sigma=0.5)
    Q = np.ascontiguousarray(np.concatenate([Qn, Qh, synth.fresh_walk_queries(8, 256, seed=2)]))
    refs = {}
    for m, q in enumerate(Q):
        refs[m] = knn_bruteforce(q, X, 64)          # the first k of the 64 are the k-NN
    return dict(X=X, Xd=torch.from_numpy(X).cuda(), Q=Q, Qd=torch.from_numpy(Q).cuda(), refs=refs)


def _check(idx, dist, ref_i, ref_d2, k):
    kk = min(k, len(ref_i))
    assert len(idx) == kk
    assert np.array_equal(idx, ref_i[:kk])
    assert np.array_equal(dist, np.sqrt(ref_d2[:kk]))


@pytest.mark.parametrize("cfg", [dict(), dict(leaf_mode=1, n_leaves=64), dict(seed_cap=0)],
                         ids=["root16", "equal_count", "no_seed"])
def test_knn_every_query(coll, cfg):
    import paper_2009_00166_amd as paris
    index = paris.build(coll["Xd"], **cfg)
    for m in range(coll["Q"].shape[0]):
        ri, rd = coll["refs"][m]
        for k in (1, 10, 64):
            idx, dist, st = index.query_knn(coll["Qd"][m], k, with_stats=True)
            _check(idx, dist, ri, rd, k)
            assert st["resolved"] >= k
        if m % 10 == 0:
            print(f"knn: query {m} ok ({cfg})", flush=True)
    index.close()


def test_knn_one_equals_exact_and_seed_counts(coll):
    import paper_2009_00166_amd as paris
    index = paris.build(coll["Xd"])
    for m in range(0, coll["Q"].shape[0], 7):
        i, d = index.query(coll["Qd"][m])
        idx, dist = index.query_knn(coll["Qd"][m], 1)
        assert (int(idx[0]), float(dist[0])) == (i, d)
    index.close()


def test_knn_ties_and_k_beyond_n():
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(5000, 64, seed=26)
    X[700] = X[20]
    X[4400] = X[20]
    q = (X[20] + np.float32(0.001)).astype(np.float32)
    index = paris.build(torch.from_numpy(X).cuda())
    for k in (3, 5):
        idx, dist = index.query_knn(torch.from_numpy(q).cuda(), k)
        ri, rd = knn_bruteforce(q, X, k)
        assert list(idx[:3]) == [20, 700, 4400] and dist[0] == dist[1] == dist[2]
        _check(idx, dist, ri, rd, k)
    index.close()
    small = np.ascontiguousarray(X[:40])
    sx = paris.build(torch.from_numpy(small).cuda())
    idx, dist = sx.query_knn(torch.from_numpy(q).cuda(), 64)
    ri, rd = knn_bruteforce(q, small, 64)
    assert len(idx) == 40
    _check(idx, dist, ri, rd, 64)
    with pytest.raises(paris.ParisError):
        sx.query_knn(torch.from_numpy(q).cuda(), 65)
    with pytest.raises(paris.ParisError):
        sx.query_knn(torch.from_numpy(q).cuda(), 0)
    sx.close()
