"""Generator checks (Section 4, random-walk generator; z-normalisation per Section 2.1)."""
import numpy as np

import synth


def test_increments_are_standard_normal():
    steps = synth.raw_steps_for_test(20000, 256, seed=0)
    assert abs(steps.mean()) < 3e-3
    assert abs(steps.var() - 1.0) < 3e-3


def test_walks_are_z_normalised_float32():
    X = synth.random_walks(5000, 256, seed=1)
    assert X.dtype == np.float32 and X.shape == (5000, 256)
    m = X.astype(np.float64).mean(axis=1)
    s = X.astype(np.float64).std(axis=1)
    assert np.max(np.abs(m)) < 1e-6
    assert np.max(np.abs(s - 1.0)) < 1e-6
    sq = (X.astype(np.float64) ** 2).sum(axis=1)
    assert np.max(np.abs(sq - 256.0)) < 1e-3


def test_walk_is_cumulative_sum_of_steps():
    steps = synth.raw_steps_for_test(1000, 64, seed=2)
    w = np.cumsum(steps, axis=1)
    z = ((w - w.mean(1, keepdims=True)) / w.std(1, keepdims=True)).astype(np.float32)
    X = synth.random_walks(1000, 64, seed=2)
    assert np.array_equal(X, z)


def test_deterministic_and_thread_independent():
    a = synth.random_walks(2_100_000 // 100, 32, seed=3, threads=1)
    b = synth.random_walks(2_100_000 // 100, 32, seed=3, threads=4)
    assert np.array_equal(a, b)
    old = synth.CHUNK
    try:
        synth.CHUNK = 5000  # several chunks: thread count must not matter
        c = synth.random_walks(21000, 32, seed=3, threads=1)
        d = synth.random_walks(21000, 32, seed=3, threads=4)
        assert np.array_equal(c, d)
    finally:
        synth.CHUNK = old
    assert not np.array_equal(a, synth.random_walks(21000, 32, seed=4))


def test_queries_near_sources():
    X = synth.random_walks(3000, 128, seed=5)
    Q, src, sig = synth.noisy_queries(X, 50, seed=5, sigma=0.1)
    assert Q.dtype == np.float32 and np.all(sig == 0.1)
    d = np.sqrt(((Q.astype(np.float64) - X[src]) ** 2).sum(1))
    assert np.median(d) < 0.1 * np.sqrt(128) * 1.5
    Q2, _, sig2 = synth.noisy_queries(X, 200, seed=5, sigma=(0.01, 0.5))
    assert sig2.min() >= 0.01 and sig2.max() <= 0.5
    F = synth.fresh_walk_queries(10, 128, seed=1)
    assert F.shape == (10, 128)
    T, tsrc, tsig = synth.training_queries(X, 20, seed=5)
    assert not np.array_equal(tsrc, src[:20]) and tsig.min() >= 0.05
