"""numpy oracle for exact 1-NN search over iSAX summaries (test infrastructure only).

Every function states the passage of the paper (arXiv 2009.00166, ParIS+) it follows, and the
reading taken where the paper is silent. Floating point is float64 with a fixed operation order
(numpy never fuses a multiply and an add). The result of the search is the plain definition of
the 1-NN problem (Section 2.1, "Similarity Search"); the exact-search twin in ``exact_search``
follows the steps of the ParIS+ ExactSearch / LBC-worker / RDC-worker algorithms (Section 3.3.3)
in serial form and must reach the same answer.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .breakpoints import breakpoints, breakpoints_at_cardinality

W = 16  # segments of the iSAX word (Section 3, overview: w is fixed to 16)


# --------------------------------------------------------------------------------------------
# Summarisation: PAA (Section 2.2) and iSAX symbols (Section 2.2)
# --------------------------------------------------------------------------------------------
def paa(x: np.ndarray, w: int = W) -> np.ndarray:
    """Piecewise Aggregate Approximation: the mean of each of ``w`` equal-length segments.

    Section 2.2 ("iSAX Representation"). Reading of the arithmetic: the ``L = n / w`` values of
    a segment are converted exactly from float32 to float64, summed in ascending position from
    0.0 with one rounding per addition, and the sum is divided by ``L`` (correctly rounded).
    ``n mod w != 0`` is never discussed in the paper; it is rejected here.
    """
    x = np.asarray(x)
    if x.dtype != np.float32:
        raise TypeError("series must be float32")
    single = x.ndim == 1
    X = x[None, :] if single else x
    N, n = X.shape
    if n % w != 0:
        raise ValueError("length must be a multiple of the segment count")
    L = n // w
    X3 = X.reshape(N, w, L)
    acc = np.zeros((N, w), dtype=np.float64)
    for j in range(L):  # ascending position inside every segment
        acc = acc + X3[:, :, j].astype(np.float64)
    out = acc / np.float64(L)
    return out[0] if single else out


def isax(paa_values: np.ndarray, bits: int = 8) -> np.ndarray:
    """iSAX symbol of every PAA value at cardinality ``2^bits`` (Section 2.2).

    Symbol = number of region boundaries ``beta_k`` (k = 1 .. 2^bits - 1) that are <= the PAA
    value, so symbol c covers the half-open region ``[beta_c, beta_{c+1})``; a value equal to a
    boundary goes to the upper region (reading: the paper does not say which side). Higher
    regions get higher symbols, matching the printed word example 10_2 00_2 11_2.
    """
    b = breakpoints_at_cardinality(bits)
    inner = b[1:-1]
    sym = np.searchsorted(inner, np.asarray(paa_values, dtype=np.float64), side="right")
    return sym.astype(np.uint8 if bits <= 8 else np.uint16)


def root_key(sym8: np.ndarray) -> np.ndarray:
    """16-bit root-subtree key: the first (top) bit of each of the 16 segments (Section 3,
    overview of the pipeline). Reading of the bit order: segment 0 is the most significant bit."""
    sym8 = np.asarray(sym8, dtype=np.uint8)
    top = (sym8 >> 7).astype(np.uint32)
    key = np.zeros(top.shape[:-1], dtype=np.uint32)
    for s in range(W):
        key = key | (top[..., s] << np.uint32(15 - s))
    return key


def k64(sym8: np.ndarray) -> np.ndarray:
    """64-bit leaf key (build decision; the paper's leaves come from ADS+ node splits).

    Bit planes 7, 6, 5, 4 of the 16 symbols are interleaved: for plane p = 7..4 and segment
    s = 0..15 the next lower bit is bit p of symbol s. The top 16 bits equal ``root_key``, and
    sorting by this key groups series that share ever longer iSAX prefixes in every segment.
    """
    sym8 = np.asarray(sym8, dtype=np.uint8)
    key = np.zeros(sym8.shape[:-1], dtype=np.uint64)
    for p in (7, 6, 5, 4):
        for s in range(W):
            bit = ((sym8[..., s] >> p) & 1).astype(np.uint64)
            key = (key << np.uint64(1)) | bit
    return key


@dataclass
class QuerySummary:
    paa: np.ndarray   # float64[16]
    sym: np.ndarray   # uint8[16]
    root: int
    k64: int


def query_summary(q: np.ndarray, w: int = W) -> QuerySummary:
    """The query side of the summaries: PAA, iSAX, root key and leaf key of the query series
    (ExactSearch takes the query and its iSAX, Section 3.3.3)."""
    qp = paa(np.asarray(q, dtype=np.float32), w)
    qs = isax(qp, 8)
    return QuerySummary(qp, qs, int(root_key(qs)), int(k64(qs)))


# --------------------------------------------------------------------------------------------
# Lower bound (Section 3.3.1) and Euclidean distance (Section 2.1)
# --------------------------------------------------------------------------------------------
def _delta(qp: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Distance from the query PAA value to the region [lo, hi): the three branches of the
    lower-bound computation (Section 3.3.1): BELOW the region, ABOVE it, or IN it."""
    below = qp < lo
    above = qp > hi
    d = np.zeros(np.broadcast(qp, lo).shape, dtype=np.float64)
    d = np.where(below, lo - qp, d)
    d = np.where(above, qp - hi, d)
    return d


def lower_bound_sq(qpaa: np.ndarray, sym: np.ndarray, L: int, bits: int = 8) -> np.ndarray:
    """Squared iSAX lower bound (mindist) between a query PAA and iSAX words.

    Section 3.3.1 gives the three-branch structure (ABOVE / BELOW / IN) but no formula. The
    formula is the PAA bound of the cited dimensionality-reduction work:
    ``LB^2 = L * sum_s delta_s^2`` with ``delta_s`` the distance from the query's segment mean to
    the symbol's region. Summed over ascending s in float64, then multiplied by L.
    """
    b = breakpoints_at_cardinality(bits)
    sym = np.asarray(sym).astype(np.int64)
    qp = np.asarray(qpaa, dtype=np.float64)
    lo = b[sym]
    hi = b[sym + 1]
    d = _delta(qp, lo, hi)
    acc = np.zeros(d.shape[:-1], dtype=np.float64)
    for s in range(d.shape[-1]):
        acc = acc + d[..., s] * d[..., s]
    return np.float64(L) * acc


def block_lower_bound_sq(qpaa: np.ndarray, sym_run: np.ndarray, L: int, bits: int = 8) -> np.float64:
    """Squared lower bound of a query against a whole run of iSAX words (build decision of the
    batched screen, lifted from the Section 3.3.1 bound).

    In segment s every word of the run lies in a region between the lower edge of the run's
    smallest symbol and the upper edge of its largest; ``delta_s`` is the distance from the
    query's segment mean to that interval (the same three branches), and the bound is
    ``L * sum_s delta_s^2`` (ascending s, float64). The interval contains each member's own
    region, so this is at most ``lower_bound_sq`` of every member.
    """
    b = breakpoints_at_cardinality(bits)
    sym_run = np.asarray(sym_run).astype(np.int64).reshape(-1, W)
    lo = b[sym_run.min(axis=0)]
    hi = b[sym_run.max(axis=0) + 1]
    d = _delta(np.asarray(qpaa, dtype=np.float64), lo, hi)
    acc = np.float64(0.0)
    for s in range(W):
        acc = acc + d[s] * d[s]
    return np.float64(L) * acc


def lb_table(qpaa: np.ndarray, L: int, bits: int = 8) -> np.ndarray:
    """float64[w][2^bits]: the per-segment lower-bound term ``L * delta(q_s, c)^2`` for every
    symbol c, i.e. the summand of ``lower_bound_sq`` tabulated over the alphabet."""
    b = breakpoints_at_cardinality(bits)
    c = np.arange(1 << bits)
    qp = np.asarray(qpaa, dtype=np.float64)[:, None]
    d = _delta(qp, b[c][None, :], b[c + 1][None, :])
    return np.float64(L) * (d * d)


def ed_sq(q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance (Section 2.1), float64, fixed operation order.

    acc = 0; for ascending j: d = q_j - x_j; t = d * d; acc = acc + t (each operation rounded
    separately; numpy does not fuse). All comparisons in the search use the squared distance.
    """
    q = np.asarray(q, dtype=np.float32).astype(np.float64)
    X = np.asarray(X, dtype=np.float32)
    single = X.ndim == 1
    Xm = X[None, :] if single else X
    acc = np.zeros(Xm.shape[0], dtype=np.float64)
    for j in range(Xm.shape[1]):
        d = q[j] - Xm[:, j].astype(np.float64)
        acc = acc + d * d
    return acc[0] if single else acc


def nn_bruteforce(q: np.ndarray, X: np.ndarray):
    """1-NN by definition (Section 2.1): the series of the collection with the smallest
    Euclidean distance to the query. Ties go to the lowest index (reading: the paper speaks of
    "the" answer). Returns ``(index, squared distance, distance)``."""
    d2 = ed_sq(q, X)
    i = int(np.argmin(d2))  # first occurrence: lowest index among equal minima
    return i, float(d2[i]), float(np.sqrt(d2[i]))


# --------------------------------------------------------------------------------------------
# Leaves (build decision) and the approximate-search seed (Section 3.3)
# --------------------------------------------------------------------------------------------
def sorted_order(sym8: np.ndarray):
    """Series positions sorted by (leaf key, position); returns ``(perm, keys_sorted)``.

    Reading of the index layout: the root subtrees of Section 3 are the runs of equal root key
    in this order; the equal-count leaves are equal slices of it."""
    keys = k64(sym8)
    perm = np.argsort(keys, kind="stable")
    return perm.astype(np.int64), keys[perm]


def root_offsets(keys_sorted: np.ndarray) -> np.ndarray:
    """uint64[65537]: start of each root subtree in the sorted order (and N at the end)."""
    N = keys_sorted.shape[0]
    r = np.arange(65536, dtype=np.uint64) << np.uint64(48)
    off = np.empty(65537, dtype=np.int64)
    off[:65536] = np.searchsorted(keys_sorted, r, side="left")
    off[65536] = N
    return off


def equal_count_bounds(N: int, n_leaves: int) -> np.ndarray:
    """Leaf l covers sorted positions [floor(l N / n_leaves), floor((l+1) N / n_leaves))."""
    ell = np.arange(n_leaves + 1, dtype=np.int64)
    return (ell * np.int64(N)) // np.int64(n_leaves)


def seed_window(qs: QuerySummary, keys_sorted: np.ndarray, L: int, mode: str = "root16",
                seed_cap: int = 16384, n_leaves: int = 4096, off: np.ndarray | None = None):
    """Sorted-position window [a, b) scanned by the approximate search (Section 3.3, first
    paragraph: descend to the leaf whose iSAX is most similar to the query's and take the
    minimum distance over that leaf's series as the first best-so-far).

    Reading (leaf capacity and the empty-child case are not given in the paper):
      * ``root16``: the query's root subtree; if it is empty, the non-empty subtree with the
        smallest cardinality-2 lower bound to the query PAA (ties: lowest root key). Inside it,
        ``seed_cap`` consecutive sorted positions centred on the lower bound of the query's leaf
        key, clipped to the subtree.
      * ``equal_count``: the equal-count leaf containing the lower bound of the query's leaf key.
    Any seed is a true distance, so the search answer does not depend on this rule.
    """
    N = keys_sorted.shape[0]
    if N == 0:
        return 0, 0
    if mode == "equal_count":
        c = int(np.searchsorted(keys_sorted, np.uint64(qs.k64), side="left"))
        # largest leaf l with floor(l N / n_leaves) <= c
        ell = ((c + 1) * n_leaves + N - 1) // N - 1
        ell = min(max(ell, 0), n_leaves - 1)
        bnd = equal_count_bounds(N, n_leaves)
        return int(bnd[ell]), int(bnd[ell + 1])
    if off is None:
        off = root_offsets(keys_sorted)
    r = qs.root
    lo, hi = int(off[r]), int(off[r + 1])
    if hi == lo:
        sizes = off[1:] - off[:-1]
        nonempty = np.nonzero(sizes > 0)[0]
        # cardinality-2 symbol of segment s of root key r = bit (15 - s) of r
        bits = ((nonempty[:, None] >> (15 - np.arange(W))[None, :]) & 1).astype(np.int64)
        lb = lower_bound_sq(qs.paa[None, :], bits, L, bits=1)
        j = int(np.lexsort((nonempty, lb))[0])
        r = int(nonempty[j])
        lo, hi = int(off[r]), int(off[r + 1])
    size = hi - lo
    if size <= seed_cap:
        return lo, hi
    c = int(np.searchsorted(keys_sorted[lo:hi], np.uint64(qs.k64), side="left")) + lo
    a = min(max(c - seed_cap // 2, lo), hi - seed_cap)
    return a, a + seed_cap


def approximate_seed(q: np.ndarray, X: np.ndarray, members: np.ndarray):
    """The approximate answer that opens exact search (Section 3.3, first paragraph; the first
    step of both ExactSearch algorithms, Section 3.3.2 and 3.3.3): the real distance from the
    query to every series of the reached leaf is computed and the smallest becomes the first
    best-so-far. ``members`` are the series of that leaf (here the window ``seed_window`` gives,
    through the sorted order). Ties go to the lowest series index.

    Returns ``(index, squared distance)``; ``(-1, +inf)`` for an empty leaf.
    """
    members = np.asarray(members, dtype=np.int64)
    if members.shape[0] == 0:
        return -1, float("inf")
    d2 = ed_sq(q, X[members])
    j = int(np.lexsort((members, d2))[0])
    return int(members[j]), float(d2[j])


def approximate_seed_k(q: np.ndarray, X: np.ndarray, members: np.ndarray, k: int):
    """The approximate search generalised to k answers: the ``min(k, len(members))`` members of
    the reached leaf with the smallest (squared distance, index), in that order.
    Returns ``(indices int64[], squared distances float64[])``."""
    members = np.asarray(members, dtype=np.int64)
    if members.shape[0] == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.float64)
    d2 = ed_sq(q, X[members])
    order = np.lexsort((members, d2))[:k]
    return members[order], d2[order]


# --------------------------------------------------------------------------------------------
# Exact search twin (Section 3.3.3: ExactSearch, LBC worker, RDC worker), serial
# --------------------------------------------------------------------------------------------
@dataclass
class ExactStats:
    seed_index: int = -1
    seed_d2: float = float("inf")
    lb_survivors: int = 0
    refined: int = 0
    abandoned: int = 0
    bsf_updates: int = 0
    candidates: list = field(default_factory=list)


def seed_members(qs: QuerySummary, sym8: np.ndarray, L: int, mode: str = "root16", seed_cap: int = 16384,
                 n_leaves: int = 4096, leaf_cap: int = 2048) -> np.ndarray:
    """Series of the leaf the approximate search reaches (Section 3.3): the window of
    ``seed_window`` in the ``root16`` and ``equal_count`` modes; in the ``ads`` mode the ADS+
    tree's leaf reached by the query's descent (``ads.ads_query_leaf``), at most ``seed_cap`` of
    its positions from its start."""
    if mode == "ads":
        from .ads import ads_query_leaf, ads_tree
        tree = ads_tree(sym8, leaf_cap)
        v = ads_query_leaf(tree, qs.sym, qs.paa, L)
        a, b = int(tree.start[v]), int(tree.end[v])
        return tree.perm[a:min(b, a + seed_cap)]
    perm, keys_sorted = sorted_order(sym8)
    a, b = seed_window(qs, keys_sorted, L, mode, seed_cap, n_leaves)
    return perm[a:b]


def exact_search(q: np.ndarray, X: np.ndarray, sym8: np.ndarray | None = None,
                 mode: str = "root16", seed_cap: int = 16384, n_leaves: int = 4096,
                 use_seed: bool = True, leaf_cap: int = 2048):
    """Serial twin of ParIS+ exact search; returns ``(index, squared distance, ExactStats)``.

    1. BSF <- approximate search (``seed_members``, then ``approximate_seed``: the smallest
       squared distance over every member of the reached leaf, ties to the lowest index), or
       +inf when ``use_seed`` is False.
    2. LBC step: candidates = {i : LB^2_i <= BSF^2}. The paper keeps i when minDist < BSF;
       reading: prune only on ">", so a series tied with the BSF at a lower index survives.
    3. Candidates are processed in ascending (LB^2, i) (the paper sorts by file position for
       disk locality; any order gives the same answer).
    4. RDC step: skip i if LB^2_i > BSF^2 (the re-check against the current BSF); otherwise the
       squared distance with early abandoning (stop once the partial sum exceeds BSF^2; the
       paper mentions early abandoning only as a property of prior SIMD distance code). Accept if
       ED^2 < BSF^2, or ED^2 == BSF^2 at a lower index.

    The lower bound is computed from rounded PAA values, so for a PAA within an ulp of a
    breakpoint it can exceed the distance by ~1e-15 relative; pruning therefore uses a relative
    slack of 1e-9 (absolute 1e-12), which keeps the twin equal to brute force.
    """
    X = np.asarray(X, dtype=np.float32)
    N, n = X.shape
    L = n // W
    qf = np.asarray(q, dtype=np.float32)
    qs = query_summary(qf)
    if sym8 is None:
        sym8 = isax(paa(X), 8)
    st = ExactStats()
    bsf, bsf_i = np.inf, -1
    if use_seed and N > 0:
        bsf_i, bsf = approximate_seed(qf, X, seed_members(qs, sym8, L, mode, seed_cap, n_leaves, leaf_cap))
        st.seed_index, st.seed_d2 = bsf_i, bsf
    lb = lower_bound_sq(qs.paa[None, :], sym8, L)

    def pruned(v: float) -> bool:
        return v > bsf * (1.0 + 1e-9) + 1e-12

    cand = [int(i) for i in np.nonzero(~(lb > bsf * (1.0 + 1e-9) + 1e-12))[0]]
    st.lb_survivors = len(cand)
    cand.sort(key=lambda i: (lb[i], i))
    qd = qf.astype(np.float64)
    for i in cand:
        if pruned(lb[i]):
            continue
        st.refined += 1
        x = X[i].astype(np.float64)
        acc = 0.0
        abandoned = False
        for j in range(n):
            d = qd[j] - x[j]
            acc = acc + d * d
            if acc > bsf:
                abandoned = True
                break
        if abandoned:
            st.abandoned += 1
            continue
        if acc < bsf or (acc == bsf and i < bsf_i):
            bsf, bsf_i = acc, i
            st.bsf_updates += 1
    return bsf_i, bsf, st


def exact_search_nb(q: np.ndarray, X: np.ndarray, workers: int, sym8: np.ndarray | None = None,
                    mode: str = "root16", seed_cap: int = 16384, n_leaves: int = 4096):
    """Serial twin of nb-ParIS+ exact search (Section 3.3, the non-balanced variant): returns
    ``(index, squared distance, refined rows per worker)``.

    1. BSF <- approximate search, as in ``exact_search``.
    2. The collection is split into ``workers`` contiguous blocks of positions. Each worker
       keeps its own BSF copy, starting from the approximate answer, and walks its block in
       position order: a series whose lower bound exceeds the worker's copy is pruned; otherwise
       its squared distance is computed (early abandoning against the copy), and the copy is
       lowered when the distance is smaller (ties to the lower index).
    3. The answer is the smallest of the copies (ties to the lowest index).

    The same slack as ``exact_search`` keeps the pruning test safe against rounding of the
    PAA values.
    """
    X = np.asarray(X, dtype=np.float32)
    N, n = X.shape
    L = n // W
    qf = np.asarray(q, dtype=np.float32)
    qs = query_summary(qf)
    if sym8 is None:
        sym8 = isax(paa(X), 8)
    seed, seed_i = np.inf, -1
    if N > 0:
        perm, keys_sorted = sorted_order(sym8)
        a, b = seed_window(qs, keys_sorted, L, mode, seed_cap, n_leaves)
        seed_i, seed = approximate_seed(qf, X, perm[a:b])
    lb = lower_bound_sq(qs.paa[None, :], sym8, L)
    qd = qf.astype(np.float64)
    copies = []
    refined = []
    edges = [w * N // workers for w in range(workers + 1)]
    for w in range(workers):
        bsf, bsf_i, r = seed, seed_i, 0
        for i in range(edges[w], edges[w + 1]):
            if lb[i] > bsf * (1.0 + 1e-9) + 1e-12:
                continue
            r += 1
            x = X[i].astype(np.float64)
            acc = 0.0
            for j in range(n):
                d = qd[j] - x[j]
                acc = acc + d * d
                if acc > bsf:
                    break
            if acc < bsf or (acc == bsf and i < bsf_i):
                bsf, bsf_i = acc, i
        copies.append((bsf, bsf_i))
        refined.append(r)
    best, best_i = min(copies) if copies else (np.inf, -1)
    return best_i, best, refined


def knn_bruteforce(q: np.ndarray, X: np.ndarray, k: int):
    """k-NN by definition (the k-NN classification experiment of Section 4 uses the k nearest
    series): the k pairs (squared distance, index) with the smallest squared distance, in
    ascending (distance, index) order (reading: ties go to the lower index, as for 1-NN).
    Returns ``(indices int64[min(k, N)], squared distances float64[min(k, N)])``."""
    d2 = ed_sq(q, X)
    order = np.lexsort((np.arange(len(d2)), d2))[:k]
    return order.astype(np.int64), d2[order]


def exact_search_knn(q: np.ndarray, X: np.ndarray, k: int, sym8: np.ndarray | None = None,
                     mode: str = "root16", seed_cap: int = 16384, n_leaves: int = 4096):
    """Serial twin of exact search generalised to k answers (the paper defines exact search for
    one answer; this generalisation is checked against the definition, ``knn_bruteforce``).

    The best-so-far becomes the k-th smallest distance found so far (+inf while fewer than k
    are known): every member of the approximate search's window is offered to the list first
    (their distances are all computed, as the approximate search computes them); a series whose lower bound
    exceeds the k-th best is pruned; the others are processed in ascending (LB², index), their
    distance abandoned once it exceeds the k-th best, and kept when it enters the list.
    Returns ``(indices, squared distances, refined count)`` like ``knn_bruteforce``.
    """
    X = np.asarray(X, dtype=np.float32)
    N, n = X.shape
    L = n // W
    qf = np.asarray(q, dtype=np.float32)
    qs = query_summary(qf)
    if sym8 is None:
        sym8 = isax(paa(X), 8)
    best = []                                   # sorted list of (d2, index), at most k long

    def kth() -> float:
        return best[-1][0] if len(best) >= k else np.inf

    def offer(d: float, i: int) -> None:
        if len(best) < k or (d, i) < best[-1]:
            best.append((d, i))
            best.sort()
            del best[k:]

    if N > 0:
        perm, keys_sorted = sorted_order(sym8)
        a, b = seed_window(qs, keys_sorted, L, mode, seed_cap, n_leaves)
        members = perm[a:b]
        for m, d in zip(members, ed_sq(qf, X[members]) if len(members) else []):
            offer(float(d), int(m))
        seeded = {int(m) for m in members}
    else:
        seeded = set()
    lb = lower_bound_sq(qs.paa[None, :], sym8, L)
    cand = sorted(range(N), key=lambda i: (lb[i], i))
    qd = qf.astype(np.float64)
    refined = 0
    for i in cand:
        if i in seeded or lb[i] > kth() * (1.0 + 1e-9) + 1e-12:
            continue
        refined += 1
        x = X[i].astype(np.float64)
        acc, limit = 0.0, kth()
        for j in range(n):
            d = qd[j] - x[j]
            acc = acc + d * d
            if acc > limit:
                break
        else:
            offer(acc, i)
    idx = np.array([i for _, i in best], dtype=np.int64)
    return idx, np.array([d for d, _ in best], dtype=np.float64), refined
