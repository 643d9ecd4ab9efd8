"""GPU test of the allocation-free per-query entry point (paris_query_exact_noalloc), through the
C ABI: on the same indexes and queries it returns exactly what paris_query_exact returns (and
what the brute-force oracle returns), on consecutive calls whose second input is smaller (an
index of shorter and fewer series), and it reports an overflow of its fixed survivor list as
PARIS_EOVERFLOW while the regular entry point answers that query."""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(index, q):
    a = index.query(q, with_stats=True)
    b = index.query_noalloc(q, with_stats=True)
    return a, b


def _same(a, b, ref_i, ref_d2):
    assert b[0] == a[0] == int(ref_i)
    assert b[1] == a[1] == math.sqrt(ref_d2)
    # the scan works on the same seed, so it keeps the same survivors
    assert b[2]["lb_survivors"] == a[2]["lb_survivors"]
    assert b[2]["seed_index"] == a[2]["seed_index"]


def test_noalloc_equals_query_exact_on_consecutive_calls(oracle_native):
    _need_gpu()
    import paper_2009_00166_amd as paris
    XA = synth.random_walks(300_000, 256, seed=11)
    QA, _, _ = synth.noisy_queries(XA, 12, seed=3, sigma=(0.05, 0.5))
    QA = np.concatenate([QA, synth.fresh_walk_queries(4, 256, seed=5)])
    XB = synth.random_walks(20_000, 128, seed=12)          # the smaller second input
    QB, _, _ = synth.noisy_queries(XB, 8, seed=4, sigma=(0.05, 0.5))
    ra_i, ra_d2, _ = oracle_native.nn_many(QA, XA, threads=16)
    rb_i, rb_d2, _ = oracle_native.nn_many(QB, XB, threads=16)
    A = paris.build(torch.from_numpy(XA).cuda())
    B = paris.build(torch.from_numpy(XB).cuda())
    QAd, QBd = torch.from_numpy(QA).cuda(), torch.from_numpy(QB).cuda()
    # the larger input, then the smaller one, alternating: every call starts from the previous
    # call's leftovers in the shared array
    for m in range(QB.shape[0]):
        print(f"noalloc: index A query {m}, index B query {m}", flush=True)
        a, b = _both(A, QAd[m])
        _same(a, b, ra_i[m], ra_d2[m])
        a, b = _both(B, QBd[m])
        _same(a, b, rb_i[m], rb_d2[m])
    for m in range(QB.shape[0], QA.shape[0]):
        a, b = _both(A, QAd[m])
        _same(a, b, ra_i[m], ra_d2[m])
    A.close()
    B.close()


def test_noalloc_survivor_overflow_is_reported(oracle_native):
    """2,200,000 identical series and a query equal to them: every lower bound is 0, so all of
    them survive the scan, more than the fixed list holds (2^21)."""
    _need_gpu()
    import paper_2009_00166_amd as paris
    N, n = 2_200_000, 64
    base = synth.random_walks(1, n, seed=21)[0]
    Xd = torch.from_numpy(base).cuda().repeat(N, 1).contiguous()
    q = Xd[0].clone()
    C = paris.build(Xd)
    print("noalloc: overflow index built", flush=True)
    with pytest.raises(paris.ParisError) as ei:
        C.query_noalloc(q)
    assert ei.value.status == -5   # PARIS_EOVERFLOW
    i, d = C.query(q)
    assert (i, d) == (0, 0.0)
    # a later call on another index is unaffected by the overflowed one
    X = synth.random_walks(5_000, 64, seed=22)
    Q, _, _ = synth.noisy_queries(X, 3, seed=6, sigma=0.2)
    ri, rd2, _ = oracle_native.nn_many(Q, X, threads=16)
    D = paris.build(torch.from_numpy(X).cuda())
    for m in range(3):
        got = D.query_noalloc(torch.from_numpy(Q[m]).cuda())
        assert got == (int(ri[m]), math.sqrt(rd2[m]))
    C.close()
    D.close()
