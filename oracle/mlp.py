"""Float64 oracle of the learned best-so-far seed (test infrastructure only).

The approximate search that opens exact search (Section 3.3, and Section 3.3.3 where ExactSearch
starts from its result) descends to the single leaf whose iSAX word is closest to the query's and
takes the smallest real distance inside that leaf as the first best-so-far (BSF). The learned
variant changes only which leaves are visited: a small multilayer perceptron reads the query's
PAA, scores every equal-count leaf, and the seed is taken over the eight best-scoring leaves. Any
seed is a true distance, so the answer of the exact search does not depend on the network.

The paper has no such network; its definition here is a build decision:

* layers 16 -> 256 -> 256 -> n_leaves, ReLU after both hidden layers, logits out;
* the first layer multiplies the float32 PAA features by bfloat16-rounded weights; the two
  larger layers multiply bfloat16-rounded activations by bfloat16-rounded weights; biases stay
  float32; the GPU accumulates in float32, this oracle in float64 after the same roundings;
* loss: mean softmax cross-entropy against the leaf that holds the exact nearest neighbour;
* backward: the gradients that enter a product (logit gradient, second-layer gradient) are
  rounded to bfloat16 like the forward operands; bias gradients are sums of the unrounded
  gradients; the weight gradient is taken as the gradient of the bfloat16 copy (the master weight
  receives it unchanged);
* optimiser: Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015, Algorithm 1)
  on float32 master weights.

Every rounding can be switched off (``rounding=False``): the result is then the exact float64
gradient of the float64 loss, which the finite-difference pins in ``tests/test_oracle_mlp.py``
check; bfloat16 rounding is pinned against torch's conversion, the loss and Adam against closed
forms. The quality of the network's predictions is parity unpinned: it is assessed only by the
seed's effect on the search (survivors, time), never by a stored value.
"""
from __future__ import annotations

import numpy as np

from .reference import approximate_seed, equal_count_bounds, query_summary

IN, HID = 16, 256
TOP_LEAVES = 8


# --------------------------------------------------------------------------------------------
# Parameter layout: one packed float32 vector [W1 (256x16), b1, W2 (256x256), b2,
# W3 (n_out x 256), b3], each matrix row-major with rows indexed by the layer's output unit.
# --------------------------------------------------------------------------------------------
def param_shapes(n_out: int):
    return [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
            ("W3", (n_out, HID)), ("b3", (n_out,))]


def n_params(n_out: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(n_out))


def unpack(theta: np.ndarray, n_out: int) -> dict:
    out, off = {}, 0
    for name, shp in param_shapes(n_out):
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[off:off + k]).reshape(shp)
        off += k
    if off != theta.shape[0]:
        raise ValueError("parameter vector has the wrong length")
    return out


def pack(parts: dict, n_out: int) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1)
                           for name, _ in param_shapes(n_out)])


# --------------------------------------------------------------------------------------------
# bfloat16 rounding: 8 significant bits, round to nearest, ties to even, same exponent range as
# float32. Written from the definition: x = m * 2^e with 0.5 <= |m| < 1, the representable
# neighbours are multiples of 2^(e-8); numpy's round() breaks ties to even.
# --------------------------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    r = np.ldexp(np.round(m * 256.0) / 256.0, e)
    r = np.where(np.isfinite(x), r, x)
    big = np.abs(r) > 3.3895313892515355e38   # largest finite bfloat16
    return np.where(big & np.isfinite(x), np.copysign(np.inf, x), r)


def _maybe(x, rounding: bool):
    return bf16_round(x) if rounding else np.asarray(x, np.float64)


# --------------------------------------------------------------------------------------------
# Forward, loss, backward
# --------------------------------------------------------------------------------------------
def forward(theta: np.ndarray, P: np.ndarray, n_out: int, rounding: bool = True) -> dict:
    """Intermediates of the forward pass for features ``P`` (float32 [B][16])."""
    p = unpack(np.asarray(theta, np.float64), n_out)
    W1, W2, W3 = (_maybe(p[k], rounding) for k in ("W1", "W2", "W3"))
    X = np.asarray(P, np.float32).astype(np.float64)
    A1 = X @ W1.T + p["b1"]
    H1 = np.maximum(A1, 0.0)
    H1r = _maybe(H1, rounding)
    A2 = H1r @ W2.T + p["b2"]
    H2 = np.maximum(A2, 0.0)
    H2r = _maybe(H2, rounding)
    Z = H2r @ W3.T + p["b3"]
    return dict(X=X, W1=W1, W2=W2, W3=W3, A1=A1, H1=H1, H1r=H1r, A2=A2, H2=H2, H2r=H2r, Z=Z)


def logsumexp_rows(Z: np.ndarray) -> np.ndarray:
    m = Z.max(axis=1, keepdims=True)
    return (m + np.log(np.exp(Z - m).sum(axis=1, keepdims=True)))[:, 0]


def loss(theta: np.ndarray, P: np.ndarray, y: np.ndarray, n_out: int, rounding: bool = True) -> float:
    """Mean over the batch of logsumexp(z) - z[label]."""
    f = forward(theta, P, n_out, rounding)
    y = np.asarray(y, np.int64)
    Z = f["Z"]
    return float(np.mean(logsumexp_rows(Z) - Z[np.arange(Z.shape[0]), y]))


def loss_and_grad(theta: np.ndarray, P: np.ndarray, y: np.ndarray, n_out: int,
                  rounding: bool = True):
    """(mean loss, packed float64 gradient) by back-propagation through the forward above."""
    f = forward(theta, P, n_out, rounding)
    y = np.asarray(y, np.int64)
    Z = f["Z"]
    B = Z.shape[0]
    lse = logsumexp_rows(Z)
    L = float(np.mean(lse - Z[np.arange(B), y]))
    G3 = np.exp(Z - lse[:, None])
    G3[np.arange(B), y] -= 1.0
    G3 /= B                                   # d loss / d Z
    G3r = _maybe(G3, rounding)
    dW3 = G3r.T @ f["H2r"]
    db3 = G3.sum(axis=0)
    G2 = (G3r @ f["W3"]) * (f["A2"] > 0)      # d loss / d A2
    G2r = _maybe(G2, rounding)
    dW2 = G2r.T @ f["H1r"]
    db2 = G2.sum(axis=0)
    G1 = (G2r @ f["W2"]) * (f["A1"] > 0)      # d loss / d A1
    dW1 = G1.T @ f["X"]
    db1 = G1.sum(axis=0)
    g = pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3), n_out)
    return L, g


def adam_step(theta, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1), step number ``t`` >= 1.
    Returns the new (theta, m, v)."""
    theta, g, m, v = (np.asarray(a, np.float64) for a in (theta, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * (g * g)
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def top_leaves(Z: np.ndarray, k: int = TOP_LEAVES) -> np.ndarray:
    """The ``k`` largest logits of every row, best first; equal logits: lowest leaf id first."""
    Z = np.asarray(Z, np.float64)
    out = np.empty((Z.shape[0], k), np.int64)
    ids = np.arange(Z.shape[1])
    for b in range(Z.shape[0]):
        order = np.lexsort((ids, -Z[b]))
        out[b] = order[:k]
    return out


# --------------------------------------------------------------------------------------------
# Features, labels and the seed they choose
# --------------------------------------------------------------------------------------------
def features(Q: np.ndarray) -> np.ndarray:
    """float32 PAA of every query (the float64 PAA of Section 2.2, rounded to float32)."""
    Q = np.asarray(Q, np.float32)
    return np.stack([query_summary(q).paa for q in Q]).astype(np.float32)


def leaf_of_index(perm: np.ndarray, n_leaves: int, idx) -> np.ndarray:
    """Equal-count leaf holding series ``idx``: the leaf whose slice of the sorted order
    [floor(l N / n_leaves), floor((l+1) N / n_leaves)) contains the series' sorted position."""
    perm = np.asarray(perm, np.int64)
    N = perm.shape[0]
    pos = np.empty(N, np.int64)
    pos[perm] = np.arange(N)
    p = pos[np.asarray(idx, np.int64)]
    return ((p + 1) * n_leaves + N - 1) // N - 1


def learned_seed(q: np.ndarray, X: np.ndarray, perm: np.ndarray, n_leaves: int, leaves) -> tuple:
    """Seed over the given leaves: the approximate search of Section 3.3 (the smallest real
    distance over every series of the leaf) taken over all series of the listed equal-count
    leaves together; ties go to the lowest index.
    Returns (index, squared distance, members examined)."""
    bnd = equal_count_bounds(X.shape[0], n_leaves)
    parts = [np.asarray(perm[bnd[ell]:bnd[ell + 1]], np.int64) for ell in leaves]
    members = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    bi, best = approximate_seed(q, X, members)
    return bi, best, members
