"""GPU parity of the ADS+ tree leaf mode (PARIS_LEAF_ADS), through the C ABI: the tree the GPU
bulk-loads (nodes, split segments, cardinalities, ranges, leaf order) equals the oracle's
``ads_tree`` node for node and position for position; the approximate search reaches the
oracle's leaf; exact 1-NN answers (per query and batched) and exact k-NN answers equal brute
force."""
import math

import numpy as np
import pytest

import synth
from oracle import (ads_query_leaf, ads_tree, approximate_seed, ed_sq, isax, k64, knn_bruteforce, paa,
                    query_summary)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _collection(N, n, seed, dups=0):
    X = synth.random_walks(N, n, seed=seed)
    if dups:
        X[100:100 + dups] = X[7]       # a group of identical words larger than the capacity
    return X


@pytest.mark.parametrize("N,n,cap,dups", [(100_000, 256, 2048, 0), (100_000, 256, 64, 0), (20_000, 64, 16, 41),
                                          (1, 256, 4, 0), (17, 128, 1, 3)])
def test_tree_equals_oracle(oracle_native, N, n, cap, dups):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = _collection(N, n, seed=N + cap, dups=dups)
    _, S = oracle_native.summarise(X)
    ref = ads_tree(S, cap)
    index = paris.build(torch.from_numpy(X).cuda(), leaf_mode=paris.LEAF_ADS, leaf_cap=cap)
    t = index.tree_nodes()
    assert len(t["start"]) == ref.n_nodes
    for f in ("start", "end", "child0", "split"):
        assert np.array_equal(t[f], getattr(ref, f)), f
    assert np.array_equal(t["card"], ref.card)
    perm = index.sorted_positions().cpu().numpy().astype(np.int64)
    assert np.array_equal(perm, ref.perm)
    leaves = ref.leaves()
    assert t["max_leaf"] == int(np.max(ref.end[leaves] - ref.start[leaves]))
    keys = index.sorted_keys().cpu().numpy().view(np.uint64)
    assert np.array_equal(keys, k64(S[perm]))
    print(f"tree N={N} cap={cap}: {ref.n_nodes - 65536} split nodes, largest leaf {t['max_leaf']}", flush=True)
    index.close()


@pytest.fixture(scope="module")
def tree_coll(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(100_000, 256, seed=5)
    Qn, _, _ = synth.noisy_queries(X, 60, seed=6, sigma=0.1)
    Qh, _, _ = synth.noisy_queries(X, 20, seed=7, sigma=0.5)
    Q = np.ascontiguousarray(np.concatenate([Qn, Qh, synth.fresh_walk_queries(20, 256, seed=8)]))
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    _, S = oracle_native.summarise(X)
    index = paris.build(torch.from_numpy(X).cuda(), leaf_mode=paris.LEAF_ADS, leaf_cap=512)
    yield dict(X=X, S=S, Q=Q, Qd=torch.from_numpy(Q).cuda(), ri=ri, rd=rd, index=index, tree=ads_tree(S, 512))
    index.close()


def test_tree_mode_answers_and_leaf(tree_coll):
    X, Q, index, tree = tree_coll["X"], tree_coll["Q"], tree_coll["index"], tree_coll["tree"]
    for m in range(Q.shape[0]):
        i, d, st = index.query(tree_coll["Qd"][m], with_stats=True)
        assert i == int(tree_coll["ri"][m]) and d == math.sqrt(tree_coll["rd"][m])
        qs = query_summary(Q[m])
        v = ads_query_leaf(tree, qs.sym, qs.paa, 16)
        a, b = int(tree.start[v]), int(tree.end[v])
        assert (st["seed_lo"], st["seed_hi"]) == (a, min(b, a + 16384))
        members = tree.perm[a:b]
        assert st["seed_index"] in set(members.tolist())
        _, ref_seed = approximate_seed(Q[m], X, members)      # the paper's approximate search
        own = float(ed_sq(Q[m], X[st["seed_index"]]))
        assert abs(st["seed_dist"] ** 2 - own) <= 1e-4 * own + 1e-9      # a true distance
        assert st["seed_dist"] >= math.sqrt(ref_seed) * (1 - 1e-5)


def test_tree_mode_batched_and_knn(tree_coll):
    X, Q, index = tree_coll["X"], tree_coll["Q"], tree_coll["index"]
    I, D = index.query_batch(tree_coll["Qd"])          # per-query kernels, no batch workspace
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), tree_coll["ri"])
    index.attach_batch(max_batch=64)                    # the batched pipeline, chunks of 64
    I, D = index.query_batch(tree_coll["Qd"])
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), tree_coll["ri"])
    assert np.array_equal(D.cpu().numpy(), np.sqrt(tree_coll["rd"]))
    for m in range(0, Q.shape[0], 9):
        ri, rd = knn_bruteforce(Q[m], X, 10)
        idx, dist = index.query_knn(tree_coll["Qd"][m], 10)
        assert np.array_equal(idx, ri) and np.array_equal(dist, np.sqrt(rd))


def test_tree_config_errors():
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = torch.from_numpy(synth.random_walks(100, 64, seed=1)).cuda()
    for cap in (0, (1 << 20) + 1):
        with pytest.raises((paris.ParisError, ValueError)):
            paris.build(X, leaf_mode=paris.LEAF_ADS, leaf_cap=cap)
