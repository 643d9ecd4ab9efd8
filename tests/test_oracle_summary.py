"""Pins for PAA, iSAX symbols, root key and leaf key of the oracle (Section 2.2, Section 3)."""
import json
import os

import numpy as np
import pytest

from oracle import breakpoints, isax, k64, paa, root_key, query_summary

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_word_example():
    """The printed word 10_2 00_2 11_2 (Section 2.2) at cardinality 4."""
    with open(os.path.join(GOLDEN, "word_example.json")) as f:
        g = json.load(f)
    sym = isax(np.array(g["paa"]), bits=g["bits"])
    assert [format(int(c), "0%db" % g["bits"]) for c in sym] == g["word_binary"]


def test_constant_series_paa_is_the_constant():
    for c in (0.1, -2.75, 3.0e-3, 1.0):
        x = np.full((3, 256), c, dtype=np.float32)
        p = paa(x)
        assert np.all(p == np.float64(np.float32(c)))


def test_paa_with_one_point_segments_is_the_series():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 16)).astype(np.float32)
    assert np.array_equal(paa(x), x.astype(np.float64))


def test_paa_matches_library_mean():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((50, 256)).astype(np.float32)
    ref = x.astype(np.float64).reshape(50, 16, 16).mean(axis=2)
    assert np.allclose(paa(x), ref, rtol=1e-14, atol=1e-15)


def test_paa_segment_order_and_hand_values():
    # n = 8, w = 2: segments [1,1,1,1] and [-0.5]*4 -> (1, -0.5)
    x = np.array([1, 1, 1, 1, -0.5, -0.5, -0.5, -0.5], dtype=np.float32)
    assert list(paa(x, w=2)) == [1.0, -0.5]
    x = np.arange(32, dtype=np.float32)
    # segment s holds 2s, 2s+1 -> mean 2s + 0.5
    assert np.array_equal(paa(x), np.arange(16) * 2 + 0.5)


def test_length_not_multiple_of_segments_rejected():
    with pytest.raises(ValueError):
        paa(np.zeros((2, 250), np.float32))


def test_symbol_on_boundary_goes_up_and_extremes():
    b = breakpoints()
    for k in (1, 2, 64, 127, 128, 129, 200, 255):
        assert isax(np.array([b[k]]))[0] == k
        assert isax(np.array([np.nextafter(b[k], -np.inf)]))[0] == k - 1
    assert isax(np.array([1e30]))[0] == 255
    assert isax(np.array([-1e30]))[0] == 0


def test_symbol_counts_boundaries_below():
    """Symbol = number of boundaries <= value: brute force over the 255 boundaries."""
    b = breakpoints()
    rng = np.random.default_rng(3)
    v = rng.standard_normal(2000) * 1.5
    sym = isax(v)
    brute = np.array([(b[1:256] <= t).sum() for t in v])
    assert np.array_equal(sym, brute)


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5, 6, 7])
def test_lower_cardinality_is_a_prefix(bits):
    rng = np.random.default_rng(4)
    v = rng.standard_normal(5000) * 1.3
    assert np.array_equal(isax(v, bits), isax(v, 8) >> (8 - bits))


def test_root_key_bit_order():
    sym = np.zeros((3, 16), np.uint8)
    sym[0, 0] = 200          # only segment 0 in the upper half -> MSB
    sym[1, 15] = 128         # only segment 15 -> LSB
    sym[2, :] = 255
    assert list(root_key(sym)) == [0x8000, 0x0001, 0xFFFF]
    sym = np.full((1, 16), 127, np.uint8)
    assert root_key(sym)[0] == 0


def test_k64_against_bit_strings():
    rng = np.random.default_rng(5)
    sym = rng.integers(0, 256, size=(200, 16), dtype=np.uint8)
    keys = k64(sym)
    for i in range(200):
        bits = "".join(format(int(sym[i, s]), "08b")[7 - p] for p in (7, 6, 5, 4) for s in range(16))
        assert int(keys[i]) == int(bits, 2)
        assert int(keys[i]) >> 48 == int(root_key(sym[i:i + 1])[0])


def test_query_summary_consistent():
    rng = np.random.default_rng(6)
    q = rng.standard_normal(256).astype(np.float32)
    s = query_summary(q)
    assert np.array_equal(s.paa, paa(q))
    assert np.array_equal(s.sym, isax(paa(q)))
    assert s.root == int(root_key(s.sym))
