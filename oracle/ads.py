"""ADS+ tree oracle (test infrastructure only): the index tree of Section 2.2 ("ADS+ Index") grown
by the node-splitting rule of Section 2.2 / Section 3.1 (IndexConstruction, SplitNode), in plain
numpy, plus the approximate search's descent to the query's leaf (Section 3.3, first paragraph).

The tree (Section 2.2):
  * the root's children are the root subtrees: the series whose first bit (cardinality 2) of
    every one of the 16 segments is the same, i.e. equal root keys;
  * every node carries a cardinality per segment (bits of the symbol it fixes); a root subtree
    fixes 1 bit of every segment;
  * a leaf holding more than ``cap`` series splits: it becomes an inner node with two children
    that fix one more bit of one segment s (child b holds the series whose next bit of s is b);
    s is the segment whose extra bit divides the node's series most evenly.

Readings (the paper gives no leaf capacity, no tie rule and inserts series one at a time):
  * bulk loading: a node splits on its whole contents (every series is summarised before the
    tree grows), so the tree is a function of the set of words, not of an insertion order;
  * most even split = smallest |n1 - n0| over the segments with fewer than 8 bits; ties go to
    the lowest segment; a node whose segments all have 8 bits stays a leaf whatever its size;
  * node numbering (a layout convention shared with the library so trees can be compared):
    nodes 0 .. 65535 are the root subtrees (node r = root key r); the tree grows in rounds, each
    round splitting, in ascending node id, every leaf that must split, the i-th of them getting
    children ``next + 2i`` (bit 0) and ``next + 2i + 1`` (bit 1), ``next`` the node count before
    the round;
  * leaf order: series sorted by (64-bit leaf key, index) (``reference.sorted_order``), every split
    a stable partition of its node's range (bit 0 first), so a node's series are contiguous.
  * the approximate search descends from the query's root subtree (an empty one is replaced as
    in ``reference.seed_window``) following the query's next bit at every split; when that child
    is empty it takes the other child.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .reference import W, lower_bound_sq, root_key, root_offsets, sorted_order


@dataclass
class AdsTree:
    start: np.ndarray    # int64 [nodes]: first position of the node in the leaf order
    end: np.ndarray      # int64 [nodes]
    child0: np.ndarray   # int64 [nodes]: -1 for a leaf; the bit-1 child is child0 + 1
    split: np.ndarray    # int64 [nodes]: segment refined by the split (-1 for a leaf)
    card: np.ndarray     # int64 [nodes][16]: bits fixed per segment
    perm: np.ndarray     # int64 [N]: series at every position of the leaf order

    @property
    def n_nodes(self) -> int:
        return self.start.shape[0]

    def leaves(self) -> np.ndarray:
        return np.nonzero(self.child0 < 0)[0]


def next_bit(sym: np.ndarray, card: int) -> np.ndarray:
    """Bit number ``card`` (counted from the most significant, 0-based) of 8-bit symbols: the bit a
    node with ``card`` bits of this segment fixed adds when it splits on it."""
    return (np.asarray(sym, np.int64) >> (7 - card)) & 1


def ads_tree(sym8: np.ndarray, cap: int) -> AdsTree:
    """The bulk-loaded ADS+ tree of the words ``sym8`` (uint8 [N][16]) with leaf capacity ``cap``."""
    sym8 = np.asarray(sym8, dtype=np.uint8)
    N = sym8.shape[0]
    perm, keys = sorted_order(sym8)
    off = root_offsets(keys)
    start = [int(off[r]) for r in range(65536)]
    end = [int(off[r + 1]) for r in range(65536)]
    child0 = [-1] * 65536
    split = [-1] * 65536
    card = [np.ones(W, np.int64) for _ in range(65536)]

    def must_split(v: int) -> bool:
        return end[v] - start[v] > cap and bool(np.any(card[v] < 8))

    todo = [v for v in range(65536) if must_split(v)]
    while todo:
        nxt = len(start)
        new_todo = []
        for i, v in enumerate(todo):
            a, b = start[v], end[v]
            words = sym8[perm[a:b]].astype(np.int64)
            m = b - a
            best_s, best_gap = -1, None
            for s in range(W):
                if card[v][s] >= 8:
                    continue
                ones = int(next_bit(words[:, s], int(card[v][s])).sum())
                gap = abs(2 * ones - m)
                if best_gap is None or gap < best_gap:      # strict: ties keep the lowest segment
                    best_s, best_gap = s, gap
            s = best_s
            bits = next_bit(words[:, s], int(card[v][s]))
            zeros = perm[a:b][bits == 0]
            ones_ = perm[a:b][bits == 1]
            perm[a:b] = np.concatenate([zeros, ones_])
            c0, c1 = nxt + 2 * i, nxt + 2 * i + 1
            child0[v], split[v] = c0, s
            cc = card[v].copy()
            cc[s] += 1
            for c, (lo, hi) in ((c0, (a, a + len(zeros))), (c1, (a + len(zeros), b))):
                start.append(lo)
                end.append(hi)
                child0.append(-1)
                split.append(-1)
                card.append(cc.copy())
                assert len(start) - 1 == c
        for c in range(nxt, len(start)):
            if must_split(c):
                new_todo.append(c)
        todo = new_todo
    return AdsTree(np.array(start, np.int64), np.array(end, np.int64), np.array(child0, np.int64),
                   np.array(split, np.int64), np.array(card, np.int64).reshape(-1, W), perm)


def ads_query_leaf(tree: AdsTree, qsym: np.ndarray, qpaa: np.ndarray, L: int) -> int:
    """Leaf reached by the approximate search for a query with symbols ``qsym`` and PAA ``qpaa``."""
    qsym = np.asarray(qsym, np.int64)
    r = int(root_key(np.asarray(qsym, np.uint8)))
    if tree.end[r] == tree.start[r]:
        # an empty root subtree: the non-empty one with the smallest cardinality-2 lower bound
        sizes = tree.end[:65536] - tree.start[:65536]
        nonempty = np.nonzero(sizes > 0)[0]
        bits = ((nonempty[:, None] >> (15 - np.arange(W))[None, :]) & 1).astype(np.int64)
        lb = lower_bound_sq(np.asarray(qpaa, np.float64)[None, :], bits, L, bits=1)
        r = int(nonempty[np.lexsort((nonempty, lb))[0]])
    v = r
    while tree.child0[v] >= 0:
        s = int(tree.split[v])
        b = int(next_bit(qsym[s], int(tree.card[v][s])))
        c = int(tree.child0[v]) + b
        if tree.end[c] == tree.start[c]:
            c = int(tree.child0[v]) + (1 - b)
        v = c
    return v
