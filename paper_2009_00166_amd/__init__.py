"""MI355X-native exact 1-NN search over iSAX summaries (ParIS+, arXiv 2009.00166).

Python face of libparis.so (include/paris.h). PyTorch provides device memory and the HIP
stream; every step of the search runs in the library's HIP kernels. There is no CPU fallback:
if the library is missing or no GPU is present, the calls raise.

    import torch, paper_2009_00166_amd as paris
    X = torch.from_numpy(series).cuda()        # float32 [N, n], z-normalised
    index = paris.build(X)                      # iSAX summaries + leaf order on the GPU
    i, d = index.query(q_dev)                   # exact 1-NN of one query
    I, D = index.query_batch(Q_dev)             # exact 1-NN of many queries
"""
from __future__ import annotations

import ctypes

from ._binding import (LEAF_ADS, LEAF_EQUAL_COUNT, LEAF_ROOT16, PARIS_OK, ParisConfig, ParisError,  # noqa: F401
                       ParisLayout, ParisQueryInfo, ParisStats, check, load_library)

__all__ = ["build", "Index", "HostCollection", "ParisError", "LEAF_ROOT16", "LEAF_EQUAL_COUNT", "LEAF_ADS", "load_library"]


def _torch():
    import torch
    return torch


def _current_stream(device_index=None) -> int:
    """Raw handle of torch's current stream on a device (default: the current device). The raw
    accessor avoids building a Stream object, which costs microseconds per call."""
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is None:
        return torch.cuda.current_stream(device_index).cuda_stream
    return raw(torch.cuda.current_device() if device_index is None else device_index)


def _stream_ptr(stream=None):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else _current_stream())


def _dev_ptr(t, dtype, ndim=None, what="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{what} must have {ndim} dimensions")
    return ctypes.c_void_p(t.data_ptr())


def default_config(**kw) -> ParisConfig:
    cfg = ParisConfig()
    check(load_library().paris_default_config(ctypes.byref(cfg)), "paris_default_config")
    for k, v in kw.items():
        setattr(cfg, k, int(v))
    return cfg


def workspace_size(n_series: int, length: int, cfg: ParisConfig | None = None) -> int:
    cfg = cfg or default_config()
    out = ctypes.c_size_t(0)
    check(load_library().paris_workspace_size(int(n_series), int(length), ctypes.byref(cfg),
                                              ctypes.byref(out)), "paris_workspace_size")
    return int(out.value)


class HostCollection:
    """A collection kept out of HBM: pinned host memory from paris_host_alloc, mapped for the
    device. Fill ``array`` (numpy float32 [n_series, length]) and pass the object to ``build``:
    the index lives in HBM, the raw series are read over PCIe."""

    def __init__(self, n_series: int, length: int):
        import numpy as np
        self.n_series, self.length = int(n_series), int(length)
        host, dev = ctypes.c_void_p(), ctypes.c_void_p()
        check(load_library().paris_host_alloc(4 * self.n_series * self.length, ctypes.byref(host),
                                              ctypes.byref(dev)), "paris_host_alloc")
        self._host, self.dev_ptr = host, int(dev.value)
        buf = (ctypes.c_float * (self.n_series * self.length)).from_address(host.value)
        self.array = np.ctypeslib.as_array(buf).reshape(self.n_series, self.length)
        self.shape = (self.n_series, self.length)

    def close(self):
        if getattr(self, "_host", None) is not None and self._host.value:
            self.array = None
            load_library().paris_host_free(self._host)
            self._host = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Index:
    """A built index. Borrows the series (a device tensor or a HostCollection) and owns a
    workspace tensor."""

    def __init__(self, series, cfg: ParisConfig | None = None, stream=None):
        torch = _torch()
        lib = load_library()
        if isinstance(series, HostCollection):
            p = ctypes.c_void_p(series.dev_ptr)
            device = torch.device("cuda", torch.cuda.current_device())
        else:
            p = _dev_ptr(series, torch.float32, 2, "series")
            device = series.device
        n_series, length = series.shape
        self.cfg = cfg or default_config()
        nbytes = workspace_size(n_series, length, self.cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.series = series  # keep the borrowed collection alive
        self.n_series, self.length = int(n_series), int(length)
        self._h = ctypes.c_void_p()
        check(lib.paris_build(p, n_series, length, ctypes.byref(self.cfg),
                              ctypes.c_void_p(self.workspace.data_ptr()), nbytes, _stream_ptr(stream),
                              ctypes.byref(self._h)), "paris_build")
        # reused by every query() call (the per-query path is latency-bound)
        self._torch = torch
        self._dev = device.index if device.index is not None else torch.cuda.current_device()
        self._query_fn = lib.paris_query_exact
        self._idx = ctypes.c_int64(-1)
        self._dist = ctypes.c_double(0.0)
        self._idx_ref = ctypes.pointer(self._idx)
        self._dist_ref = ctypes.pointer(self._dist)

    # -- queries --------------------------------------------------------------------------
    def query(self, q, stream=None, with_stats: bool = False):
        """Exact 1-NN of one query (float32 [length] on the device): (index, distance[, stats])."""
        torch = self._torch
        if not (isinstance(q, torch.Tensor) and q.is_cuda and q.dtype == torch.float32 and q.dim() == 1
                and q.is_contiguous()):
            _dev_ptr(q, torch.float32, 1, "query")   # raises with the reason
        if q.shape[0] != self.length:
            raise ValueError("query length differs from the collection's")
        st = ParisStats() if with_stats else None
        s = stream.cuda_stream if stream is not None else _current_stream(self._dev)
        rc = self._query_fn(self._h, q.data_ptr(), self._idx_ref, self._dist_ref,
                            ctypes.byref(st) if with_stats else None, s)
        if rc != PARIS_OK:
            check(rc, "paris_query_exact")
        if with_stats:
            return int(self._idx.value), float(self._dist.value), st.as_dict()
        return int(self._idx.value), float(self._dist.value)

    def query_knn(self, q, k: int, stream=None, with_stats: bool = False):
        """Exact k-NN of one query (float32 [length] on the device), k in 1 .. 64: (indices,
        distances[, stats]) as numpy arrays of min(k, n_series) entries in ascending (distance,
        index) order."""
        import numpy as np
        torch = self._torch
        _dev_ptr(q, torch.float32, 1, "query")
        if q.shape[0] != self.length:
            raise ValueError("query length differs from the collection's")
        idx = np.zeros(max(int(k), 1), np.int64)
        dist = np.zeros(max(int(k), 1), np.float64)
        found = ctypes.c_int32(0)
        st = ParisStats() if with_stats else None
        s = stream.cuda_stream if stream is not None else _current_stream(self._dev)
        check(load_library().paris_query_knn(self._h, q.data_ptr(), int(k), idx.ctypes.data_as(ctypes.c_void_p),
                                             dist.ctypes.data_as(ctypes.c_void_p), ctypes.byref(found),
                                             ctypes.byref(st) if with_stats else None, s), "paris_query_knn")
        f = found.value
        if with_stats:
            return idx[:f].copy(), dist[:f].copy(), st.as_dict()
        return idx[:f].copy(), dist[:f].copy()

    def query_noalloc(self, q, stream=None, with_stats: bool = False):
        """As ``query``, through paris_query_exact_noalloc: the per-query scratch comes from the
        library's static device array (no allocation; at most 2^21 lower-bound survivors, else
        ParisError with PARIS_EOVERFLOW)."""
        torch = self._torch
        _dev_ptr(q, torch.float32, 1, "query")
        if q.shape[0] != self.length:
            raise ValueError("query length differs from the collection's")
        st = ParisStats() if with_stats else None
        s = stream.cuda_stream if stream is not None else _current_stream(self._dev)
        check(load_library().paris_query_exact_noalloc(self._h, q.data_ptr(), self._idx_ref, self._dist_ref,
                                                       ctypes.byref(st) if with_stats else None, s),
              "paris_query_exact_noalloc")
        if with_stats:
            return int(self._idx.value), float(self._dist.value), st.as_dict()
        return int(self._idx.value), float(self._dist.value)

    def query_batch(self, Q, stream=None, with_stats: bool = False, out=None):
        """Exact 1-NN of every row of Q (float32 [M, length] on the device).

        Returns device tensors (int64 [M], float64 [M]); asynchronous unless ``with_stats``."""
        torch = _torch()
        qp = _dev_ptr(Q, torch.float32, 2, "queries")
        if Q.shape[1] != self.length:
            raise ValueError("query length differs from the collection's")
        M = Q.shape[0]
        if out is None:
            I = torch.empty(M, dtype=torch.int64, device=Q.device)
            D = torch.empty(M, dtype=torch.float64, device=Q.device)
        else:
            I, D = out
        st = ParisStats()
        check(load_library().paris_query_batch(self._h, qp, M, ctypes.c_void_p(I.data_ptr()),
                                               ctypes.c_void_p(D.data_ptr()),
                                               ctypes.byref(st) if with_stats else None,
                                               _stream_ptr(stream)), "paris_query_batch")
        if with_stats:
            return I, D, st.as_dict()
        return I, D

    # -- inspection -----------------------------------------------------------------------
    def layout(self) -> ParisLayout:
        lay = ParisLayout()
        check(load_library().paris_get_layout(self._h, ctypes.byref(lay)), "paris_get_layout")
        return lay

    def sax(self):
        """uint8 [N, 16] device view of the iSAX words (row i = series i)."""
        torch = _torch()
        off = self.layout().sax_dev - self.workspace.data_ptr()
        return self.workspace[off:off + 16 * self.n_series].view(self.n_series, 16)

    def sorted_keys(self):
        torch = _torch()
        off = self.layout().keys_dev - self.workspace.data_ptr()
        return self.workspace[off:off + 8 * self.n_series].view(torch.int64)

    def sorted_positions(self):
        torch = _torch()
        off = self.layout().perm_dev - self.workspace.data_ptr()
        return self.workspace[off:off + 4 * self.n_series].view(torch.int32)

    def root_offsets(self):
        torch = _torch()
        off = self.layout().roff_dev - self.workspace.data_ptr()
        return self.workspace[off:off + 4 * 65537].view(torch.int32)

    def tree_nodes(self):
        """ADS+ leaf mode: the tree's nodes as a dict of host numpy arrays (start, end, child0,
        split, card [nodes, 16]); None in the other leaf modes."""
        import numpy as np
        lay = self.layout()
        if not lay.tree_nodes_dev:
            return None
        off = lay.tree_nodes_dev - self.workspace.data_ptr()
        raw = self.workspace[off:off + 32 * lay.n_tree_nodes].cpu().numpy().reshape(-1, 32)
        u32 = raw[:, :16].copy().view(np.uint32).reshape(-1, 4)
        return {"start": u32[:, 0].astype(np.int64), "end": u32[:, 1].astype(np.int64),
                "child0": u32[:, 2].view(np.int32).astype(np.int64),
                "split": u32[:, 3].view(np.int32).astype(np.int64),
                "card": raw[:, 16:].astype(np.int64), "max_leaf": int(lay.tree_max_leaf)}

    def query_info(self, q, stream=None, tables: bool = False):
        torch = _torch()
        qp = _dev_ptr(q, torch.float32, 1, "query")
        info = ParisQueryInfo()
        t8 = None
        if tables:
            t8 = torch.empty((16, 256), dtype=torch.float32, device=q.device)
        check(load_library().paris_query_info_get(
            self._h, qp, ctypes.byref(info), ctypes.c_void_p(t8.data_ptr()) if tables else None,
            _stream_ptr(stream)), "paris_query_info_get")
        d = {"paa": list(info.paa), "sym": list(info.sym), "root": int(info.root), "k64": int(info.k64),
             "win_lo": int(info.win_lo), "win_hi": int(info.win_hi)}
        if tables:
            d["table"] = t8
        return d

    def lb_scan(self, q, threshold_sq: float, capacity: int | None = None, stream=None):
        """(indices int32 [k], bounds float32 [k]) of every series whose bound is <= threshold."""
        torch = _torch()
        qp = _dev_ptr(q, torch.float32, 1, "query")
        cap = self.n_series if capacity is None else int(capacity)
        I = torch.empty(max(cap, 1), dtype=torch.int32, device=q.device)
        B = torch.empty(max(cap, 1), dtype=torch.float32, device=q.device)
        cnt = ctypes.c_int64(0)
        st = load_library().paris_lb_scan(self._h, qp, ctypes.c_float(threshold_sq),
                                          ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                          cap, ctypes.byref(cnt), _stream_ptr(stream))
        if st not in (PARIS_OK, -5):
            check(st, "paris_lb_scan")
        k = min(int(cnt.value), cap)
        return I[:k], B[:k], int(cnt.value), st

    # -- batched pipeline -----------------------------------------------------------------
    def attach_batch(self, max_batch: int = 4096, stream=None) -> int:
        """Allocate (torch) and attach the batched-pipeline workspace; returns its bytes."""
        torch = _torch()
        lib = load_library()
        nbytes = ctypes.c_size_t(0)
        check(lib.paris_batch_workspace_size(self._h, int(max_batch), ctypes.byref(nbytes)),
              "paris_batch_workspace_size")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.workspace.device)
        check(lib.paris_batch_attach(self._h, ctypes.c_void_p(ws.data_ptr()), int(nbytes.value),
                                     int(max_batch), _stream_ptr(stream)), "paris_batch_attach")
        self.batch_workspace = ws
        self.max_batch = int(max_batch)
        return int(nbytes.value)

    def screen_dots(self, Q, stream=None):
        """float32 [M, N] dot products of the bfloat16 rows, as accumulated by the screen."""
        torch = _torch()
        qp = _dev_ptr(Q, torch.float32, 2, "queries")
        out = torch.empty((Q.shape[0], self.n_series), dtype=torch.float32, device=Q.device)
        check(load_library().paris_screen_dots(self._h, qp, int(Q.shape[0]), ctypes.c_void_p(out.data_ptr()),
                                               _stream_ptr(stream)), "paris_screen_dots")
        return out

    def screen_tiles(self, reset: bool = False):
        """(query tiles the batched screen ran, tiles a screen of every pair would have run)
        since the attach or the last reset."""
        run = ctypes.c_int64(0)
        dense = ctypes.c_int64(0)
        check(load_library().paris_batch_screen_tiles(self._h, ctypes.byref(run), ctypes.byref(dense),
                                                      1 if reset else 0), "paris_batch_screen_tiles")
        return int(run.value), int(dense.value)

    def block_bound_bits(self, Q, sqdist, item_series: int = 256, stream=None):
        """uint64 [ceil(N / item_series), ceil(M / 64)] alive bits of the screen's block bound for
        queries Q (float32 [M, length]) with thresholds sqdist (float32 [M], squared distances)."""
        torch = _torch()
        qp = _dev_ptr(Q, torch.float32, 2, "queries")
        up = _dev_ptr(sqdist, torch.float32, 1, "thresholds")
        M = Q.shape[0]
        if sqdist.shape[0] != M:
            raise ValueError("one threshold per query")
        out = torch.zeros(((self.n_series + item_series - 1) // item_series, (M + 63) // 64),
                          dtype=torch.int64, device=Q.device)
        check(load_library().paris_block_bound_bits(self._h, qp, up, int(M), int(item_series),
                                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
              "paris_block_bound_bits")
        return out

    def set_bsf_sharing(self, shared: bool = True) -> None:
        """Shared best-so-far during refinement (ParIS+) or one private copy per distance
        worker (nb-ParIS+, Section 3.3; the default, faster here); answers are identical."""
        check(load_library().paris_set_bsf_sharing(self._h, 1 if shared else 0), "paris_set_bsf_sharing")

    def set_timing(self, enable: bool = True, scan_only: bool = False, sampled: bool = False) -> None:
        """Enable HIP-event timing of query() and zero the totals: all three phases (events
        between them), or the scan kernel alone (events bound to its dispatch; sampled: the scan
        of every 8th query)."""
        mode = (3 if sampled else 2 if scan_only else 1) if enable else 0
        check(load_library().paris_set_timing(self._h, mode), "paris_set_timing")

    def timing(self):
        """(summed ms per phase [prepare+seed, lbscan, refine+resolve], timed calls)."""
        ms = (ctypes.c_double * 3)()
        n = ctypes.c_int64(0)
        check(load_library().paris_get_timing(self._h, ms, ctypes.byref(n)), "paris_get_timing")
        return list(ms), int(n.value)

    def batch_timing(self):
        """(summed ms per batch stage [seeds, block bound, screen, rescore, resolve], timed chunks)."""
        ms = (ctypes.c_double * 5)()
        n = ctypes.c_int64(0)
        check(load_library().paris_get_batch_timing(self._h, ms, ctypes.byref(n)), "paris_get_batch_timing")
        return list(ms), int(n.value)

    # -- learned seed ------------------------------------------------------------------------
    def leaf_of(self, series_idx, stream=None):
        """int32 [k] equal-count leaf of every series index (int64 device tensor)."""
        torch = _torch()
        ip = _dev_ptr(series_idx, torch.int64, 1, "series indices")
        out = torch.empty(series_idx.shape[0], dtype=torch.int32, device=series_idx.device)
        check(load_library().paris_leaf_of(self._h, ip, int(series_idx.shape[0]),
                                           ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "paris_leaf_of")
        return out

    def set_seed_model(self, model, enabled: bool = True) -> None:
        """Use (or stop using) a trained SeedModel for the approximate-search seed."""
        check(load_library().paris_set_seed_model(self._h, model._h if model is not None else None,
                                                  1 if enabled else 0), "paris_set_seed_model")
        self._seed_model = model if enabled else None   # keep the network alive while in use

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().paris_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_batch_multi(indexes, queries, stream=None, with_stats: bool = False):
    """Exact 1-NN of the rows of queries[c] (float32 [M_c, n_c] on the device) against
    indexes[c], for every collection c, in one call: [(I_c, D_c)] (and the summed stats)."""
    torch = _torch()
    k = len(indexes)
    if k != len(queries) or k == 0:
        raise ValueError("one query tensor per index")
    outs = []
    qp, nq, ip, dp = (ctypes.c_void_p * k)(), (ctypes.c_int64 * k)(), (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)()
    hs = (ctypes.c_void_p * k)()
    for c, (ix, Q) in enumerate(zip(indexes, queries)):
        if Q.dim() != 2 or Q.shape[1] != ix.length:
            raise ValueError("query length differs from the collection's")
        _dev_ptr(Q, torch.float32, 2, "queries")
        I = torch.empty(Q.shape[0], dtype=torch.int64, device=Q.device)
        D = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
        outs.append((I, D))
        hs[c], qp[c], nq[c] = ix._h.value, Q.data_ptr(), int(Q.shape[0])
        ip[c], dp[c] = I.data_ptr(), D.data_ptr()
    st = ParisStats()
    check(load_library().paris_query_batch_multi(hs, k, qp, nq, ip, dp, ctypes.byref(st) if with_stats else None,
                                                 _stream_ptr(stream)), "paris_query_batch_multi")
    return (outs, st.as_dict()) if with_stats else outs


__all__ += ["query_batch_multi"]

from .learned import SeedModel, init_params, query_features, train_seed_model  # noqa: E402,F401

__all__ += ["SeedModel", "init_params", "query_features", "train_seed_model"]


def build(series, cfg: ParisConfig | None = None, stream=None, **cfg_kw) -> Index:
    """Summarise a float32 [N, n] device tensor (or a HostCollection) and build its index
    (synchronous)."""
    if cfg is None:
        cfg = default_config(**cfg_kw)
    return Index(series, cfg, stream)
