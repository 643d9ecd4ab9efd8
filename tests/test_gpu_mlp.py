"""GPU parity of the learned seed against the float64 oracle (oracle/mlp.py): features, forward
logits, top leaves, gradients (relative error <= 1e-2 per parameter tensor), Adam, training, the
leaf labels, and the seed's effect on the exact search (answers identical to the oracle)."""
import numpy as np
import pytest

import oracle.mlp as M
import synth
from oracle import isax, paa, sorted_order

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_OUT = 256


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _paris():
    _need_gpu()
    import paper_2009_00166_amd as paris
    return paris


def _gamma(k, u=2.0 ** -24):
    return k * u / (1 - k * u)


def _theta(seed, n_out=N_OUT):
    import paper_2009_00166_amd as paris
    th = paris.init_params(n_out, seed=seed)
    # non-zero biases so that every term of the forward pass is exercised
    parts = M.unpack(th.astype(np.float64), n_out)
    rng = np.random.default_rng(seed + 100)
    for b in ("b1", "b2", "b3"):
        parts[b][:] = rng.standard_normal(parts[b].shape) * 0.1
    return M.pack(parts, n_out).astype(np.float32)


def _features(rows, seed):
    X = synth.random_walks(rows, 256, seed=seed)
    return M.features(X), X


def test_features_are_bit_exact():
    paris = _paris()
    Q = synth.fresh_walk_queries(333, 256, seed=5)
    F = paris.query_features(torch.from_numpy(Q).cuda()).cpu().numpy()
    assert np.array_equal(F, M.features(Q))
    Q2 = synth.fresh_walk_queries(17, 1024, seed=6)
    assert np.array_equal(paris.query_features(torch.from_numpy(Q2).cuda()).cpu().numpy(), M.features(Q2))


def _logit_bounds(f, th32):
    """Per-logit tolerance. Tight: float32 accumulation of the same bfloat16 operands,
    gamma_{K+2} times the absolute products. Loose: additionally a hidden activation may round
    to the neighbouring bfloat16 value (its float32 and float64 values straddle a rounding
    boundary), moving a logit by at most 2^-7 of the absolute products."""
    abs_terms = np.abs(f["H2r"]) @ np.abs(f["W3"]).T + np.abs(M.unpack(th32.astype(np.float64), N_OUT)["b3"])
    tight = 2 * _gamma(258) * abs_terms + 1e-30
    loose = 2.0 ** -7 * abs_terms + 1e-6
    return tight, loose


def test_forward_logits_and_top_leaves_match_oracle():
    paris = _paris()
    th = _theta(1)
    F, _ = _features(200, seed=11)       # 200 rows: a ragged last tile of 64
    net = paris.SeedModel(N_OUT, max_rows=128, params=th)   # two pieces of at most 128 rows
    Fd = torch.from_numpy(F).cuda()
    Z = net.forward(Fd).cpu().numpy().astype(np.float64)
    f = M.forward(th.astype(np.float64), F, N_OUT, rounding=True)
    tight, loose = _logit_bounds(f, th)
    err = np.abs(Z - f["Z"])
    assert np.all(err <= loose), float(np.max(err / loose))
    assert np.mean(err <= tight) >= 0.9
    # top leaves: exactly the top 8 of the GPU's own logits (value desc, id asc) ...
    T = net.top_leaves(Fd).cpu().numpy()
    assert np.array_equal(T, M.top_leaves(Z, 8))
    # ... and the oracle's where its 8th and 9th logits are separated by more than the tolerance
    To = M.top_leaves(f["Z"], 8)
    clear = 0
    for b in range(F.shape[0]):
        z, tol = f["Z"][b], loose[b]
        inside = np.zeros(N_OUT, bool)
        inside[To[b]] = True
        # every oracle top-8 logit stays above every other logit within the tolerances
        if np.min(z[inside] - tol[inside]) > np.max(z[~inside] + tol[~inside]):
            clear += 1
            assert set(T[b]) == set(To[b])
    assert clear >= 20
    net.close()


def test_gradient_matches_oracle_within_1e_2():
    paris = _paris()
    th = _theta(2)
    F, _ = _features(300, seed=12)
    rng = np.random.default_rng(3)
    y = rng.integers(0, N_OUT, size=300).astype(np.int32)
    sel = rng.permutation(300)[:190].astype(np.int32)   # a shuffled subset: ragged, indirect rows
    net = paris.SeedModel(N_OUT, max_rows=256, params=th)
    for s in (None, sel):
        rows = np.arange(300) if s is None else s
        if s is None:
            rows = rows[:256]
            g, loss = net.grad(torch.from_numpy(F[:256]).cuda(), torch.from_numpy(y[:256]).cuda())
        else:
            g, loss = net.grad(torch.from_numpy(F).cuda(), torch.from_numpy(y).cuda(),
                               sel=torch.from_numpy(s).cuda())
        L, gref = M.loss_and_grad(th.astype(np.float64), F[rows], y[rows], N_OUT, rounding=True)
        assert abs(float(loss.item()) - L) <= 1e-4 * abs(L)
        gp = M.unpack(g.cpu().numpy().astype(np.float64), N_OUT)
        gr = M.unpack(gref, N_OUT)
        for name in gr:
            rel = np.linalg.norm(gp[name] - gr[name]) / np.linalg.norm(gr[name])
            assert rel <= 1e-2, (name, rel)
    net.close()


def test_adam_apply_matches_oracle():
    paris = _paris()
    th = _theta(4)
    net = paris.SeedModel(N_OUT, max_rows=64, params=th)
    rng = np.random.default_rng(8)
    ref, m, v = th.astype(np.float64), np.zeros(th.shape[0]), np.zeros(th.shape[0])
    for t in range(1, 4):
        g = (rng.standard_normal(th.shape[0]) * 10.0 ** rng.uniform(-6, 0, th.shape[0])).astype(np.float32)
        net.apply(torch.from_numpy(g).cuda(), lr=1e-3)
        ref, m, v = M.adam_step(ref, g.astype(np.float64), m, v, t, 1e-3)
    got = net.params().cpu().numpy().astype(np.float64)
    # float32 state: a few ulps of the parameter plus a relative 1e-4 of the step size per step
    assert np.all(np.abs(got - ref) <= 4 * 2.0 ** -24 * np.abs(ref) + 3 * 1e-3 * 1e-4), \
        float(np.max(np.abs(got - ref)))
    net.close()


def test_leaf_labels_match_oracle():
    paris = _paris()
    X = synth.random_walks(30_011, 256, seed=21)
    idx = paris.build(torch.from_numpy(X).cuda(), leaf_mode=1, n_leaves=64)
    perm, _ = sorted_order(isax(paa(X), 8))
    series = np.concatenate([np.arange(0, 30_011, 7), [0, 30_010, -1, 30_011]]).astype(np.int64)
    got = idx.leaf_of(torch.from_numpy(series).cuda()).cpu().numpy()
    valid = (series >= 0) & (series < 30_011)
    assert np.array_equal(got[valid], M.leaf_of_index(perm, 64, series[valid]))
    assert np.all(got[~valid] == -1)
    idx.close()


def test_training_lowers_the_loss():
    paris = _paris()
    X = synth.random_walks(40_000, 256, seed=31)
    Xd = torch.from_numpy(X).cuda()
    idx = paris.build(Xd, leaf_mode=1, n_leaves=64)
    idx.attach_batch(max_batch=1024)
    Q, _, _ = synth.training_queries(X, 3000, seed=31)
    F, y, _ = paris.learned.exact_labels(idx, torch.from_numpy(Q).cuda())
    net = paris.SeedModel(64, max_rows=512, params=paris.init_params(64, seed=0))
    hist = paris.train_seed_model(net, F, y, epochs=8, batch=256, lr=2e-3, seed=0)
    assert hist[-1] < 0.6 * hist[0], hist
    assert all(np.isfinite(hist))
    net.close()
    idx.close()


@pytest.fixture(scope="module")
def learned_setup(oracle_native):
    """200,000 x 256 walks, 256 equal-count leaves, a network trained on 20,000 exact labels."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    X = synth.random_walks(200_000, 256, seed=41)
    Xd = torch.from_numpy(X).cuda()
    idx = paris.build(Xd, leaf_mode=1, n_leaves=256)
    idx.attach_batch(max_batch=2048)
    Qt, _, _ = synth.training_queries(X, 20_000, seed=41)
    F, y, _ = paris.learned.exact_labels(idx, torch.from_numpy(Qt).cuda())
    net = paris.SeedModel(256, max_rows=1024, params=paris.init_params(256, seed=1))
    hist = paris.train_seed_model(net, F, y, epochs=12, batch=512, lr=2e-3, seed=1)
    Qe, _, _ = synth.noisy_queries(X, 300, seed=42, sigma=0.5)
    ri, rd, _ = oracle_native.nn_many(Qe, X, threads=16)
    return dict(X=X, Xd=Xd, idx=idx, net=net, hist=hist, Qe=Qe, ri=ri, rd=rd)


def test_learned_seed_keeps_answers_exact_and_prunes_more(learned_setup):
    s = learned_setup
    idx, net, Qe = s["idx"], s["net"], s["Qe"]
    Qd = torch.from_numpy(Qe).cuda()
    plain, learned = [], []
    I0 = np.empty(len(Qe), np.int64)
    I1 = np.empty(len(Qe), np.int64)
    D1 = np.empty(len(Qe))
    for m in range(len(Qe)):
        i, _, st = idx.query(Qd[m], with_stats=True)
        I0[m] = i
        plain.append(st)
    idx.set_seed_model(net, True)
    for m in range(len(Qe)):
        i, d, st = idx.query(Qd[m], with_stats=True)
        I1[m], D1[m] = i, d
        learned.append(st)
    assert np.array_equal(I0, s["ri"]) and np.array_equal(I1, s["ri"])
    assert np.array_equal(D1, np.sqrt(s["rd"]))
    # the seed is a true distance of a series in one of the query's 8 best-scoring leaves
    import paper_2009_00166_amd as paris
    T = net.top_leaves(paris.query_features(Qd)).cpu().numpy()
    leaf = idx.leaf_of(torch.tensor([st["seed_index"] for st in learned], dtype=torch.int64).cuda()).cpu().numpy()
    X = s["X"]
    # the per-query kernel accumulates the logits in another order than the batched MFMA pass,
    # so a near-tie at the 8th place may pick a different leaf there
    assert np.mean([leaf[m] in set(T[m]) for m in range(len(Qe))]) >= 0.95
    for m, st in enumerate(learned):
        true = float(np.sqrt(((Qe[m].astype(np.float64) - X[st["seed_index"]]) ** 2).sum()))
        assert abs(st["seed_dist"] - true) <= 1e-4 * true + 1e-6
    surv0 = np.array([st["lb_survivors"] for st in plain], np.float64)
    surv1 = np.array([st["lb_survivors"] for st in learned], np.float64)
    seed0 = np.array([st["seed_dist"] for st in plain])
    seed1 = np.array([st["seed_dist"] for st in learned])
    print("survivors plain/learned mean", surv0.mean(), surv1.mean(), "seed ratio plain/learned",
          np.mean(seed0 / np.sqrt(s["rd"])), np.mean(seed1 / np.sqrt(s["rd"])), "loss", s["hist"])
    assert surv1.mean() < 0.8 * surv0.mean()
    assert np.mean(seed1 <= seed0) >= 0.6
    idx.set_seed_model(None, False)


def test_learned_seed_in_the_batched_pipeline(learned_setup):
    s = learned_setup
    idx, net = s["idx"], s["net"]
    Qd = torch.from_numpy(s["Qe"]).cuda()
    idx.set_seed_model(net, True)
    I, D, st = idx.query_batch(Qd, with_stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), s["ri"])
    assert np.array_equal(D.cpu().numpy(), np.sqrt(s["rd"]))
    idx.set_seed_model(None, False)
    I2, _, st2 = idx.query_batch(Qd, with_stats=True)
    assert np.array_equal(I2.cpu().numpy(), s["ri"])
    print("screen candidates learned / plain", st["lb_survivors"], st2["lb_survivors"])
    assert st["lb_survivors"] <= st2["lb_survivors"]
