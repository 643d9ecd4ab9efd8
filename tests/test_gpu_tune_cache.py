"""Tuned launch shapes kept in the file that PARIS_TUNE_CACHE names: the scan's online decision
and the screen's timed choice are appended to it, a later build or attach with a matching line
takes that line's shape without timing anything, and the answers stay exact (brute force)."""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, LEN = 50_000, 256
SCAN_SHAPES = [(512, 2, 1), (512, 2, 2), (512, 4, 1), (512, 1, 4), (256, 4, 1), (256, 4, 2), (256, 8, 1), (256, 3, 4)]
SCREEN_SHAPES = [(32, 2, 2, 32), (64, 2, 1, 32), (32, 2, 1, 32)]   # forms the block bound accepts


def _lines(path, kind):
    return [ln.split() for ln in path.read_text().splitlines() if ln.startswith(kind + " ")]


def test_tune_cache_round_trip(tmp_path, monkeypatch, oracle_native):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_00166_amd as paris
    for var in ("PARIS_SCAN_SHAPE", "PARIS_SCREEN_SHAPE", "PARIS_BLOCK_LB"):
        monkeypatch.delenv(var, raising=False)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("PARIS_TUNE_CACHE", str(path))
    X = synth.random_walks(N, LEN, seed=41)
    Q, _, _ = synth.noisy_queries(X, 60, seed=42, sigma=0.2)
    ri, rd, _ = oracle_native.nn_many(Q, X, threads=16)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    nbucket = str(int(math.floor(math.log2(N))))

    def answers(index):
        for m in range(Q.shape[0]):
            i, d = index.query(Qd[m])
            assert i == int(ri[m]) and d == math.sqrt(rd[m]), m

    # no file yet: timed at build, refined on the first 48 queries, decision appended
    index = paris.build(Xd)
    answers(index)
    lay = index.layout()
    scan = _lines(path, "scan")
    assert len(scan) == 1
    arch = scan[0][1]
    assert scan[0][2:6] == [str(LEN), nbucket, "0", ":"]
    tuned = (lay.scan_threads, lay.scan_blocks_per_cu, lay.scan_unroll)
    assert tuple(int(v) for v in scan[0][6:9]) == tuned
    # the screen's choice at attach (block bound on, chunks of 64)
    index.attach_batch(max_batch=64)
    lay = index.layout()
    screen = _lines(path, "screen")
    assert len(screen) == 1 and screen[0][1] == arch
    assert screen[0][2:6] == [str(LEN), nbucket, str(2 * 64 + 1), ":"]
    picked = (lay.screen_rows, lay.screen_blocks_per_cu, lay.screen_subtiles, lay.screen_mfma)
    assert tuple(int(v) for v in screen[0][6:10]) == picked
    index.close()

    # a hand-written line that differs from the tuned shapes is taken as it stands
    other_scan = next(s for s in SCAN_SHAPES if s != tuned)
    other_screen = next(s for s in SCREEN_SHAPES if s != picked)
    with open(path, "a") as f:
        f.write("this line does not parse\n")
        f.write(f"scan {arch} {LEN} {nbucket} 0 : {other_scan[0]} {other_scan[1]} {other_scan[2]} 0\n")
        f.write(f"screen {arch} {LEN} {nbucket} {2 * 64 + 1} : " + " ".join(str(v) for v in other_screen) + "\n")
    index = paris.build(Xd)
    lay = index.layout()
    assert (lay.scan_threads, lay.scan_blocks_per_cu, lay.scan_unroll) == other_scan
    answers(index)
    lay = index.layout()   # no online phase: the shape stays
    assert (lay.scan_threads, lay.scan_blocks_per_cu, lay.scan_unroll) == other_scan
    assert len(_lines(path, "scan")) == 2
    index.attach_batch(max_batch=64)
    lay = index.layout()
    assert (lay.screen_rows, lay.screen_blocks_per_cu, lay.screen_subtiles, lay.screen_mfma) == other_screen
    assert len(_lines(path, "screen")) == 2
    I, D = index.query_batch(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(I.cpu().numpy(), ri) and np.array_equal(D.cpu().numpy(), np.sqrt(rd))
    index.close()
