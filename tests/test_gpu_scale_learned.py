"""GPU parity of the learned best-so-far seed at its full collection size (50,000,000 x 256,
4096 equal-count leaves, network 16-256-256-4096), in the launch configurations the benchmark's
learned section times: hard queries (noise 0.5) one at a time with the learned and the plain
seed, checked by the brute-force C oracle, and one whole batch of 4096 queries through the
batched pipeline with the learned seed (128 of its queries checked by the oracle, every answer's distance
checked against the oracle's float64 distance to the returned series). The network is trained
briefly: its quality changes only the speed, never an answer."""
import math
import time

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_FULL, LEN, LEAVES = 50_000_000, 256, 4096


@pytest.fixture(scope="module")
def learned_full(oracle_native):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_00166_amd as paris
    t0 = time.time()
    X = synth.random_walks(N_FULL, LEN, seed=0, threads=16)
    Xd = torch.from_numpy(X).cuda()
    idx = paris.build(Xd, leaf_mode=1, n_leaves=LEAVES)
    idx.attach_batch(max_batch=4096)
    Qt, _, _ = synth.training_queries(X, 20_000, seed=0)
    F, y, _ = paris.learned.exact_labels(idx, torch.from_numpy(Qt).cuda())
    net = paris.SeedModel(LEAVES, max_rows=1024, params=paris.init_params(LEAVES, seed=0))
    hist = paris.train_seed_model(net, F, y, epochs=2, batch=1024, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    print(f"[scale50] generated, built, labelled and trained in {time.time() - t0:.1f}s "
          f"(loss {hist[0]:.3f} -> {hist[-1]:.3f})", flush=True)
    yield dict(X=X, idx=idx, net=net)
    idx.set_seed_model(None, False)
    net.close()
    idx.close()


def test_learned_seed_per_query_at_50m(learned_full, oracle_native):
    X, idx, net = learned_full["X"], learned_full["idx"], learned_full["net"]
    Q, _, _ = synth.noisy_queries(X, 10, seed=2, sigma=0.5)
    t0 = time.time()
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    print(f"[scale50] oracle brute force {Q.shape[0]} queries in {time.time() - t0:.1f}s", flush=True)
    Qd = torch.from_numpy(Q).cuda()
    for enabled in (True, False):
        idx.set_seed_model(net, enabled)
        for m in range(Q.shape[0]):
            i, d, st = idx.query(Qd[m], with_stats=True)
            assert i == int(ri[m]), (enabled, m, i, int(ri[m]))
            assert d == math.sqrt(rd[m])
            assert st["seed_dist"] >= d * (1 - 1e-5)      # the seed is a true distance
    idx.set_seed_model(None, False)


def test_learned_seed_full_batch_at_50m(learned_full, oracle_native):
    X, idx, net = learned_full["X"], learned_full["idx"], learned_full["net"]
    M = 4096
    Q, src, sig = synth.noisy_queries(X, M, seed=1, sigma=(0.01, 0.5))
    Qd = torch.from_numpy(Q).cuda()
    idx.set_seed_model(net, True)
    I, D, st = idx.query_batch(Qd, with_stats=True)
    torch.cuda.synchronize()
    idx.set_seed_model(None, False)
    I, D = I.cpu().numpy(), D.cpu().numpy()
    # 128 queries checked by brute force: the 32 with the largest noise and 96 at random
    order = np.argsort(-sig, kind="stable")
    pick = np.sort(np.concatenate([order[:32], np.random.default_rng(4).choice(order[32:], 96, replace=False)]))
    t0 = time.time()
    ri, rd, _ = oracle_native.nn_many_blocked(Q[pick], X, threads=16)
    print(f"[scale50] oracle: {len(pick)} of the batch's queries in {time.time() - t0:.1f}s", flush=True)
    assert np.array_equal(I[pick], ri)
    assert np.array_equal(D[pick], np.sqrt(rd))
    assert np.all((I >= 0) & (I < N_FULL))
    for m in range(M):
        d_ret, d_src = oracle_native.ed2_at(Q[m], X, [I[m], src[m]])
        assert D[m] == math.sqrt(d_ret), m
        assert d_ret <= d_src, m
    print(f"[scale50] learned batch: {st['lb_survivors']} screen survivors, {st['refined']} re-scored, "
          f"{st['resolved']} fallbacks", flush=True)
