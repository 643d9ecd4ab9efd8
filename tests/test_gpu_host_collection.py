"""Out-of-core collections: the raw series in pinned host memory (paris_host_alloc), the index in
HBM; the kernels read raw rows over PCIe. Exact answers (per query, batched, k-NN, in the root
subtree and ADS+ tree leaf modes) equal brute force and the answers of the same collection in
HBM."""
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


@pytest.mark.parametrize("leaf", ["root16", "ads"])
def test_host_collection_answers(oracle_native, leaf):
    _need_gpu()
    import paper_2009_00166_amd as paris
    N, n = 200_000, 256
    coll = paris.HostCollection(N, n)
    synth.random_walks(N, n, seed=51, out=coll.array)
    X = coll.array
    Qn, _, _ = synth.noisy_queries(X, 24, seed=52, sigma=(0.05, 0.5))
    Q = np.ascontiguousarray(np.concatenate([Qn, synth.fresh_walk_queries(8, n, seed=53)]))
    ri, rd, _ = oracle_native.nn_many_blocked(Q, X, threads=16)
    cfg = dict(leaf_mode=paris.LEAF_ADS, leaf_cap=1024) if leaf == "ads" else {}
    host = paris.build(coll, **cfg)
    dev = paris.build(torch.from_numpy(X.copy()).cuda(), **cfg)
    Qd = torch.from_numpy(Q).cuda()
    assert np.array_equal(host.sax().cpu().numpy(), dev.sax().cpu().numpy())
    for m in range(Q.shape[0]):
        a = host.query(Qd[m])
        assert a == (int(ri[m]), math.sqrt(rd[m])) == dev.query(Qd[m])
    host.attach_batch(max_batch=16)
    I, D = host.query_batch(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri) and np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    for m in range(0, Q.shape[0], 8):
        ki, kd = knn_bruteforce(Q[m], X, 10)
        idx, dist = host.query_knn(Qd[m], 10)
        assert np.array_equal(idx, ki) and np.array_equal(dist, np.sqrt(kd))
    host.close()
    dev.close()
    coll.close()


def test_host_alloc_errors():
    _need_gpu()
    import ctypes
    import paper_2009_00166_amd as paris
    from paper_2009_00166_amd import _binding as B
    lib = paris.load_library()
    h, d = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.paris_host_alloc(0, ctypes.byref(h), ctypes.byref(d)) == B.PARIS_EINVAL
    assert lib.paris_host_alloc(1024, None, ctypes.byref(d)) == B.PARIS_EINVAL
    assert lib.paris_host_free(None) == B.PARIS_OK
