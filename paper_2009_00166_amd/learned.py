"""Learned best-so-far seed: the network handle (paris_mlp_* in include/paris.h) and its training
loop. Argument marshalling and the loop's bookkeeping only: features, labels, forward and backward
passes and the optimiser step all run in the library's HIP kernels.

The approximate search that opens exact search (Section 3.3) normally visits the one leaf chosen
by the query's own iSAX word; with a trained network attached (``Index.set_seed_model``) it visits
the 8 best-scoring equal-count leaves instead. Training pairs come from the exact search itself:
the features are the queries' PAA, the label is the leaf holding each query's exact nearest
neighbour.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._binding import ParisAdam, check, load_library


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    from . import _current_stream
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else _current_stream())


def _dev(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous CUDA (HIP) {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def param_count(n_leaves: int) -> int:
    out = ctypes.c_int64(0)
    check(load_library().paris_mlp_param_count(int(n_leaves), ctypes.byref(out)), "paris_mlp_param_count")
    return int(out.value)


def init_params(n_leaves: int, seed: int = 0) -> np.ndarray:
    """Initial float32 parameters (packed as in include/paris.h): weights drawn from
    N(0, 2 / fan_in) (He initialisation for ReLU layers), biases zero. Seeded numpy draws."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    parts = []
    for fan_out, fan_in in ((256, 16), (256, 256), (n_leaves, 256)):
        parts.append((rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)).astype(np.float32).ravel())
        parts.append(np.zeros(fan_out, np.float32))
    out = np.concatenate(parts)
    assert out.shape[0] == param_count(n_leaves)
    return out


def query_features(Q, stream=None):
    """float32 [M, 16]: the PAA of every query row of a float32 [M, n] device tensor."""
    torch = _torch()
    if Q.dim() != 2:
        raise ValueError("queries must be [M, n]")
    F = torch.empty((Q.shape[0], 16), dtype=torch.float32, device=Q.device)
    check(load_library().paris_query_features(_dev(Q, torch.float32, "queries"), int(Q.shape[0]), int(Q.shape[1]),
                                              ctypes.c_void_p(F.data_ptr()), _stream_ptr(stream)),
          "paris_query_features")
    return F


class SeedModel:
    """The 16 -> 256 -> 256 -> n_leaves seed network; its device workspace is a torch tensor."""

    def __init__(self, n_leaves: int, max_rows: int = 4096, params=None, device="cuda"):
        torch = _torch()
        self.n_leaves = int(n_leaves)
        self.max_rows = int(max_rows)
        self.n_params = param_count(self.n_leaves)
        lib = load_library()
        nb = ctypes.c_int64()
        check(lib.paris_mlp_workspace_size(self.n_leaves, self.max_rows, ctypes.byref(nb)), "paris_mlp_workspace_size")
        # torch's caching allocator hands out 512-byte aligned blocks
        self._ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib.paris_mlp_create(self.n_leaves, self.max_rows, ctypes.c_void_p(self._ws.data_ptr()), int(nb.value),
                                   ctypes.byref(h)), "paris_mlp_create")
        self._h = h
        if params is not None:
            self.set_params(params)

    def set_params(self, params, stream=None) -> None:
        torch = _torch()
        if isinstance(params, np.ndarray):
            params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
        if params.numel() != self.n_params:
            raise ValueError("parameter vector has the wrong length")
        self._params_in = params   # the copy is asynchronous: keep the source alive
        check(load_library().paris_mlp_set_params(self._h, _dev(params, torch.float32, "params"),
                                                  _stream_ptr(stream)), "paris_mlp_set_params")

    def params(self, stream=None):
        torch = _torch()
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(load_library().paris_mlp_get_params(self._h, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
              "paris_mlp_get_params")
        return out

    def forward(self, F, stream=None):
        torch = _torch()
        Z = torch.empty((F.shape[0], self.n_leaves), dtype=torch.float32, device=F.device)
        check(load_library().paris_mlp_forward(self._h, _dev(F, torch.float32, "features"), int(F.shape[0]),
                                               ctypes.c_void_p(Z.data_ptr()), _stream_ptr(stream)),
              "paris_mlp_forward")
        return Z

    def top_leaves(self, F, stream=None):
        torch = _torch()
        out = torch.empty((F.shape[0], 8), dtype=torch.int32, device=F.device)
        check(load_library().paris_mlp_top_leaves(self._h, _dev(F, torch.float32, "features"), int(F.shape[0]),
                                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
              "paris_mlp_top_leaves")
        return out

    def grad(self, F, y, sel=None, stream=None):
        """(packed float32 gradient, mean loss as a 1-element tensor) of one batch."""
        torch = _torch()
        rows = int(sel.shape[0]) if sel is not None else int(F.shape[0])
        g = torch.empty(self.n_params, dtype=torch.float32, device=F.device)
        loss = torch.empty(1, dtype=torch.float32, device=F.device)
        sp = _dev(sel, torch.int32, "row selection") if sel is not None else None
        check(load_library().paris_mlp_grad(self._h, _dev(F, torch.float32, "features"), _dev(y, torch.int32, "labels"),
                                            sp, rows, ctypes.c_void_p(g.data_ptr()),
                                            ctypes.c_void_p(loss.data_ptr()), _stream_ptr(stream)),
              "paris_mlp_grad")
        return g, loss

    def train_step(self, F, y, sel=None, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, loss_out=None, stream=None):
        torch = _torch()
        rows = int(sel.shape[0]) if sel is not None else int(F.shape[0])
        opt = ParisAdam(float(lr), float(betas[0]), float(betas[1]), float(eps))
        sp = _dev(sel, torch.int32, "row selection") if sel is not None else None
        lp = ctypes.c_void_p(loss_out.data_ptr()) if loss_out is not None else None
        check(load_library().paris_mlp_train_step(self._h, _dev(F, torch.float32, "features"),
                                                  _dev(y, torch.int32, "labels"), sp, rows, ctypes.byref(opt), lp,
                                                  _stream_ptr(stream)), "paris_mlp_train_step")

    def apply(self, g, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, stream=None):
        """One Adam update with a given packed float32 gradient."""
        torch = _torch()
        opt = ParisAdam(float(lr), float(betas[0]), float(betas[1]), float(eps))
        check(load_library().paris_mlp_apply(self._h, _dev(g, torch.float32, "gradient"), ctypes.byref(opt),
                                             _stream_ptr(stream)), "paris_mlp_apply")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().paris_mlp_free(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None   # after the free: the network never outlives its workspace

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exact_labels(index, Q, stream=None):
    """(features float32 [M, 16], labels int32 [M], nearest-neighbour indices int64 [M]) of
    training queries: every query is answered by the exact search and labelled with the leaf
    that holds its nearest neighbour."""
    I, _ = index.query_batch(Q, stream=stream)
    return query_features(Q, stream), index.leaf_of(I, stream), I


def train_seed_model(model: SeedModel, F, y, epochs: int = 10, batch: int = 1024, lr: float = 1e-3,
                     seed: int = 0, stream=None):
    """Mini-batch Adam over (features, labels) for ``epochs`` passes; the example order of every
    pass is a seeded permutation (drawn on the host, passed to the kernels as row indices).
    Returns the mean training loss of every pass."""
    torch = _torch()
    M = int(F.shape[0])
    if batch > model.max_rows or batch % 64:
        raise ValueError("batch must be a multiple of 64 and at most max_rows")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    losses = torch.zeros(((M + batch - 1) // batch) * epochs, dtype=torch.float32, device=F.device)
    history = []
    k = 0
    for _ in range(epochs):
        order = torch.from_numpy(rng.permutation(M).astype(np.int32)).to(F.device)
        k0 = k
        for b0 in range(0, M, batch):
            sel = order[b0:b0 + batch]
            model.train_step(F, y, sel=sel, lr=lr, loss_out=losses[k:k + 1], stream=stream)
            k += 1
        history.append((k0, k))
    per_step = losses.cpu().numpy()
    return [float(np.mean(per_step[a:b])) for a, b in history]
