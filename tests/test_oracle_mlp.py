"""Pins of the learned-seed oracle (oracle/mlp.py), CPU only.

Every check compares the oracle with something it does not compute itself: finite differences of
its own loss (which test the back-propagation formulas, not their retyping), torch's autograd and
Adam in float64, torch's bfloat16 conversion, closed forms of the loss and of Adam's first steps,
brute force for the leaf of a series, and the plain seed as the one-leaf special case.
"""
import numpy as np
import pytest

import oracle.mlp as M
from oracle import equal_count_bounds, exact_search, isax, paa, query_summary, seed_window, sorted_order
import synth

torch = pytest.importorskip("torch")

N_OUT = 64


def _theta(seed=0, n_out=N_OUT, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in M.param_shapes(n_out):
        fan_in = shp[1] if len(shp) == 2 else 1
        s = scale * (np.sqrt(2.0 / fan_in) if len(shp) == 2 else 0.1)
        parts[name] = rng.standard_normal(shp) * s
    return M.pack(parts, n_out)


def _batch(B=6, seed=1, n_out=N_OUT):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((B, 16)).astype(np.float32)
    y = rng.integers(0, n_out, size=B)
    return P, y


def test_param_count_of_the_full_network():
    assert M.n_params(4096) == 1_122_816


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(3)
    vals = [rng.standard_normal(20000).astype(np.float32),
            (rng.standard_normal(5000) * 1e30).astype(np.float32),
            (rng.standard_normal(5000) * 1e-30).astype(np.float32),
            np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.0e38, -3.0e38], np.float32)]
    # exact ties: a bfloat16 value plus half of its last place (both parities of the last bit)
    base = rng.standard_normal(4000).astype(np.float32)
    b_bits = base.view(np.uint32) & np.uint32(0xFFFF0000)
    ties = (b_bits | np.uint32(0x8000)).view(np.float32)
    vals.append(ties)
    x = np.concatenate(vals)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16_round(x)
    assert np.array_equal(got, ref)
    nan = M.bf16_round(np.array([np.nan], np.float32))
    assert np.isnan(nan[0])


def _dir_deriv_check(theta, P, y, n_out, tol):
    _, g = M.loss_and_grad(theta, P, y, n_out, rounding=False)
    rng = np.random.default_rng(7)
    off = 0
    for name, shp in M.param_shapes(n_out):
        k = int(np.prod(shp))
        for _ in range(3):
            d = np.zeros_like(theta)
            d[off:off + k] = rng.standard_normal(k)
            h = 1e-6
            fd = (M.loss(theta + h * d, P, y, n_out, False) - M.loss(theta - h * d, P, y, n_out, False)) / (2 * h)
            an = float(g @ d)
            assert abs(fd - an) <= tol * max(abs(an), 1e-8), (name, fd, an)
        off += k


def test_gradient_matches_finite_differences():
    _dir_deriv_check(_theta(0), *_batch(), N_OUT, 1e-6)


def test_gradient_matches_finite_differences_at_larger_weights():
    _dir_deriv_check(_theta(5, scale=3.0), *_batch(B=9, seed=4), N_OUT, 1e-6)


def test_loss_and_gradient_match_torch_autograd():
    theta = _theta(2)
    P, y = _batch(B=7, seed=2)
    parts = M.unpack(theta, N_OUT)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in parts.items()}
    X = torch.tensor(P.astype(np.float64))
    h1 = torch.relu(X @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    z = h2 @ tp["W3"].T + tp["b3"]
    ls = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    ls.backward()
    L, g = M.loss_and_grad(theta, P, y, N_OUT, rounding=False)
    assert abs(L - ls.item()) <= 1e-12 * abs(L)
    gt = M.pack({k: v.grad.numpy() for k, v in tp.items()}, N_OUT)
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_rounded_forward_uses_bf16_operands():
    theta = _theta(3)
    P, _ = _batch(B=4, seed=3)
    f = M.forward(theta, P, N_OUT, rounding=True)
    for k in ("W1", "W2", "W3", "H1r", "H2r"):
        v = f[k]
        assert np.array_equal(v, torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()), k
    # the rounded network is close to the exact one (bfloat16 keeps 8 significant bits)
    f0 = M.forward(theta, P, N_OUT, rounding=False)
    assert np.max(np.abs(f["Z"] - f0["Z"])) < 0.05 * np.max(np.abs(f0["Z"]))


def test_loss_closed_forms():
    zero = np.zeros(M.n_params(N_OUT))
    P, y = _batch(B=5)
    L, g = M.loss_and_grad(zero, P, y, N_OUT)
    assert L == pytest.approx(np.log(N_OUT), rel=1e-15)
    gb3 = M.unpack(g, N_OUT)["b3"]
    onehot = np.zeros((5, N_OUT))
    onehot[np.arange(5), y] = 1
    assert np.allclose(gb3, (1.0 / N_OUT - onehot).mean(axis=0), rtol=1e-14, atol=1e-17)
    assert abs(gb3.sum()) < 1e-15
    # a dominant correct logit drives the loss to zero
    parts = M.unpack(zero.copy(), N_OUT)
    parts["b3"][:] = -1e3
    parts["b3"][y[0]] = 1e3
    assert M.loss(M.pack(parts, N_OUT), P[:1], y[:1], N_OUT) == pytest.approx(0.0, abs=1e-300)


def test_adam_first_steps_closed_form_and_torch():
    rng = np.random.default_rng(11)
    th = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    lr = 1e-3
    t1, m, v = M.adam_step(th, g, m, v, 1, lr)
    # first step: m_hat = g and v_hat = g^2, so every parameter moves by lr * g / (|g| + eps)
    assert np.allclose(t1, th - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    t2, m, v = M.adam_step(t1, g, m, v, 2, lr)
    assert np.allclose(t2, t1 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # torch's Adam, float64, over several steps with changing gradients
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    mine, m, v = th.copy(), np.zeros(1000), np.zeros(1000)
    for t in range(1, 6):
        gt = rng.standard_normal(1000)
        p.grad = torch.tensor(gt)
        opt.step()
        mine, m, v = M.adam_step(mine, gt, m, v, t, lr)
    assert np.allclose(mine, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_top_leaves_order_and_ties():
    Z = np.array([[0.5, 2.0, 2.0, -1.0, 3.0, 2.0, 0.5, 0.5, 0.5, 0.0]])
    assert M.top_leaves(Z, 8)[0].tolist() == [4, 1, 2, 5, 0, 6, 7, 8]
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((20, 300))
    t = M.top_leaves(Z, 8)
    for b in range(20):
        assert t[b].tolist() == list(np.argsort(-Z[b], kind="stable")[:8])


def test_leaf_of_index_by_brute_force():
    X = synth.random_walks(3001, 64, seed=4)
    sym8 = isax(paa(X), 8)
    perm, _ = sorted_order(sym8)
    for nl in (1, 7, 64, 3001):
        bnd = equal_count_bounds(3001, nl)
        idx = np.arange(3001)
        got = M.leaf_of_index(perm, nl, idx)
        for i in range(0, 3001, 37):
            pos = int(np.nonzero(perm == i)[0][0])
            ell = int(np.nonzero(bnd[:-1] <= pos)[0][-1])
            assert bnd[ell] <= pos < bnd[ell + 1]
            assert got[i] == ell


def test_learned_seed_over_the_plain_leaf_is_the_plain_seed():
    X = synth.random_walks(20000, 64, seed=6)
    Q, _, _ = synth.noisy_queries(X, 12, seed=6, sigma=0.3)
    sym8 = isax(paa(X), 8)
    perm, keys = sorted_order(sym8)
    nl = 32
    bnd = equal_count_bounds(20000, nl)
    for q in Q:
        qs = query_summary(q)
        a, b = seed_window(qs, keys, 64 // 16, mode="equal_count", n_leaves=nl)
        ell = int(np.searchsorted(bnd, a, side="right") - 1)
        assert (bnd[ell], bnd[ell + 1]) == (a, b)
        i, d2, _ = M.learned_seed(q, X, perm, nl, [ell])
        _, _, st = exact_search(q, X, sym8, mode="equal_count", n_leaves=nl)
        assert (i, d2) == (st.seed_index, st.seed_d2)
        # more leaves can only lower the seed, and it stays a true distance >= the 1-NN distance
        i8, d8, _ = M.learned_seed(q, X, perm, nl, [ell] + [(ell + k) % nl for k in range(1, 8)])
        assert d8 <= d2
        true = ((q.astype(np.float64) - X[i8].astype(np.float64)) ** 2).sum()
        assert d8 == pytest.approx(true, rel=1e-12)
        assert d8 >= exact_search(q, X, sym8, use_seed=False)[1]


def test_features_are_the_float32_paa():
    Q = synth.fresh_walk_queries(5, 256, seed=3)
    F = M.features(Q)
    assert F.dtype == np.float32
    for q, f in zip(Q, F):
        segs = q.astype(np.float64).reshape(16, 16).mean(axis=1)
        assert np.allclose(f, segs.astype(np.float32), rtol=1e-6, atol=1e-7)
