"""Early-abandoning pruned DTW (Herrmann & Webb, arXiv 2010.05371) on MI355X.

Thin Python binding over the C ABI of ``libeapdtw.so`` (include/eapdtw.h):
argument marshalling only -- every step of the method runs in the gfx950 HIP
kernels.  PyTorch provides device memory and the current stream.  There is no
CPU fallback: without the built library or a gfx950 device every call raises.

Functions (names follow the C ABI):

* ``dtw(S, T, window, ub=inf)``            -- one pair (Section 2, Eq. 1-5;
  Section 2.1 window; Section 2.2 bound) -> float
* ``dtw_pairs(X, Y, window, ub=None|tensor|'ed')`` -- batch of pairs -> tensor
* ``pairwise(X, window)``                  -- all i<j distances (ub = squared ED)
* ``nn_search(query, series, window)``     -- best (offset, distance)
* ``nn_search_batch([(query, window), ...], series)``
* ``nn_dists(query, series, window, ub)``  -- per-candidate bounded distances
* ``window_stats(series, m)``, ``znorm(x)`` -- exposed steps of the search
* ``DTWFunction.apply(S, T, window)``      -- differentiable batch (autograd)
* ``dtw_path(S, T, window)``               -- the optimal path ranges the backward follows
* ``dtw_pairs_batch(S_list, T_list, windows, ub=None)`` -- uneven pairs in pools
* ``DTWBatchFunction.apply(S_pool, T_pool, pairs, ...)`` -- differentiable uneven batch
* ``dtw_batch_path(...)``                  -- path ranges of an uneven batch
* ``dba_step(B, X, window)``               -- one DTW barycentre averaging update
* ``window_from_ratio(ratio, m)``          -- integer window, rounded up
* ``autotune(query, series, window)``, ``tune_get``, ``tune_save``,
  ``tune_load``                            -- the kernel-choice tuning cache
"""
from __future__ import annotations

import ctypes
import math
import threading

import torch

from . import _lib
from ._lib import EapdtwError, LbStats, Pair, Query, Result, Stats, Tune

__all__ = ["dtw", "dtw_pairs", "pairwise", "nn_search", "nn_search_batch", "nn_dists",
           "window_stats", "znorm", "window_from_ratio", "DTWFunction", "Context",
           "knn_search_batch",
           "EapdtwError", "Stats", "set_option", "get_option", "pairwise_index", "autotune",
           "tune_bucket", "tune_get", "tune_save", "tune_load", "nn_search_lb", "nn_dists_lb",
           "nn_lower_bounds", "LbStats", "knn_search", "knn_search_lb", "nn1", "nn_search_w", "nn_dists_w",
           "nn1_ref", "dtw_path", "dtw_pairs_batch", "pack_pairs", "DTWBatchFunction",
           "dtw_batch_path", "dba_step", "unpack_ranges", "erp_pairs",
           "nn_search_erp"]


def window_from_ratio(ratio: float, m: int) -> int:
    """Integer Sakoe-Chiba window for a ratio of the series length, rounded up."""
    if ratio < 0:
        raise ValueError("ratio must be >= 0")
    return int(math.ceil(ratio * m - 1e-9))


class Context:
    """One library context (device, stream, scratch)."""

    def __init__(self, device: int | None = None):
        lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self._lib = lib
        h = ctypes.c_void_p()
        rc = lib.eapdtw_create(self.device, None, ctypes.byref(h))
        if rc != 0:
            raise EapdtwError(rc, lib.eapdtw_last_error(None).decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                self._lib.eapdtw_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def check(self, rc: int):
        if rc != 0:
            raise EapdtwError(rc, self._lib.eapdtw_last_error(self._h).decode())

    def bind_stream(self):
        st = torch.cuda.current_stream(self.device).cuda_stream
        self.check(self._lib.eapdtw_set_stream(self._h, ctypes.c_void_p(st)))

    def set_option(self, key: str, value: int):
        self.check(self._lib.eapdtw_set_option(self._h, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        self.check(self._lib.eapdtw_get_option(self._h, key.encode(), ctypes.byref(v)))
        return v.value


_ctx_lock = threading.Lock()
_ctxs: dict = {}


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    key = (threading.get_ident(), int(device))
    with _ctx_lock:
        c = _ctxs.get(key)
        if c is None:
            c = Context(device)
            _ctxs[key] = c
    return c


def set_option(key: str, value: int, device: int | None = None):
    context(device).set_option(key, value)


def get_option(key: str, device: int | None = None) -> int:
    return context(device).get_option(key)


def _dev(x, device=None) -> torch.Tensor:
    """float32 contiguous tensor on the GPU (host data is copied)."""
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(x)
    if device is None:
        device = torch.cuda.current_device() if not x.is_cuda else x.device.index
    x = x.to(device=f"cuda:{device}", dtype=torch.float32)
    return x.contiguous()


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(0)


def dtw(S, T, window: int, ub: float = math.inf, stats: bool = False):
    S, T = _dev(S), _dev(T)
    ctx = context(S.device.index)
    ctx.bind_stream()
    out = ctypes.c_double()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_dtw(ctx.handle, _ptr(S), S.numel(), _ptr(T), T.numel(), int(window),
                                  float(ub), ctypes.byref(out), ctypes.byref(st)))
    return (out.value, st.as_dict()) if stats else out.value


def dtw_pairs(X, Y, window: int, ub=None, stats: bool = False):
    """DTW of pairs (X[p], Y[p]).  ub: None (plain DTW), a per-pair tensor, or
    'ed' for the squared Euclidean distance of each pair (Section 2.3)."""
    X, Y = _dev(X), _dev(Y)
    if X.shape != Y.shape or X.dim() != 2:
        raise ValueError("X and Y must both be [npairs, len]")
    ctx = context(X.device.index)
    ctx.bind_stream()
    out = torch.empty(X.shape[0], device=X.device, dtype=torch.float32)
    if ub is None:
        mode, ubt = 0, None
    elif isinstance(ub, str):
        if ub != "ed":
            raise ValueError("ub must be None, 'ed' or a tensor")
        mode, ubt = 2, None
    else:
        mode, ubt = 1, _dev(ub, X.device.index)
        if ubt.numel() != X.shape[0]:
            raise ValueError("ub must have one entry per pair")
    st = Stats()
    ctx.check(ctx._lib.eapdtw_dtw_pairs(ctx.handle, _ptr(X), _ptr(Y), X.shape[0], X.shape[1],
                                        int(window), mode, _ptr(ubt) if ubt is not None else None,
                                        _ptr(out), ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def pairwise_index(N: int, i: int, j: int) -> int:
    """Position of pair (i, j), i < j, in the upper-triangle output of pairwise()."""
    return i * N - i * (i + 1) // 2 + (j - i - 1)


def pairwise(X, window: int, stats: bool = False):
    X = _dev(X)
    if X.dim() != 2:
        raise ValueError("X must be [N, len]")
    N = X.shape[0]
    ctx = context(X.device.index)
    ctx.bind_stream()
    out = torch.empty(N * (N - 1) // 2, device=X.device, dtype=torch.float32)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_pairwise(ctx.handle, _ptr(X), N, X.shape[1], int(window), _ptr(out),
                                       ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def nn_search(query, series, window: int, stats: bool = False):
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    off = ctypes.c_int64()
    dist = ctypes.c_double()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_search(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                        int(window), ctypes.byref(off), ctypes.byref(dist),
                                        ctypes.byref(st) if stats else None))
    res = (off.value, dist.value)
    return (res, st.as_dict()) if stats else res


def nn_search_batch(queries, series, stats: bool = False):
    """queries: list of (query, window).  Returns a list of (offset, distance)."""
    x = _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    qs = [(_dev(q, x.device.index), int(w)) for q, w in queries]
    arr = (Query * len(qs))()
    for i, (q, w) in enumerate(qs):
        arr[i].query = q.data_ptr()
        arr[i].m = q.numel()
        arr[i].window = w
    res = (Result * len(qs))()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_search_batch(ctx.handle, arr, len(qs), _ptr(x), x.numel(), res,
                                              ctypes.byref(st) if stats else None))
    out = [(r.offset, r.dist) for r in res]
    return (out, st.as_dict()) if stats else out


def knn_search_batch(queries, series, k: int, stats: bool = False):
    """queries: list of (query, window).  Returns, per query, its k nearest
    offsets as a list of (offset, distance) in (distance, offset) order."""
    x = _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    qs = [(_dev(q, x.device.index), int(w)) for q, w in queries]
    arr = (Query * max(len(qs), 1))()
    for i, (q, w) in enumerate(qs):
        arr[i].query = q.data_ptr()
        arr[i].m = q.numel()
        arr[i].window = w
    kk = int(k)
    offs = (ctypes.c_int64 * max(len(qs) * kk, 1))()
    dists = (ctypes.c_double * max(len(qs) * kk, 1))()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_knn_search_batch(ctx.handle, arr, len(qs), _ptr(x), x.numel(), kk,
                                               offs, dists, ctypes.byref(st) if stats else None))
    out = [[(offs[q * kk + j], dists[q * kk + j]) for j in range(kk)] for q in range(len(qs))]
    return (out, st.as_dict()) if stats else out


def nn_dists(query, series, window: int, ub: float = math.inf, stats: bool = False):
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    out = torch.empty(x.numel() - q.numel() + 1, device=x.device, dtype=torch.float32)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_dists(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                       int(window), float(ub), _ptr(out),
                                       ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def nn_search_lb(query, series, window: int, stats: bool = False):
    """nn_search with the lower-bound cascade (LB_Kim, LB_Keogh with the query's
    and with the candidate's envelope) in front of the DTW.  With stats=True
    returns ((offset, distance), stats) where stats also holds the cascade's
    counters."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    off = ctypes.c_int64()
    dist = ctypes.c_double()
    st, ls = Stats(), LbStats()
    ctx.check(ctx._lib.eapdtw_nn_search_lb(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                           int(window), ctypes.byref(off), ctypes.byref(dist),
                                           ctypes.byref(st) if stats else None,
                                           ctypes.byref(ls) if stats else None))
    res = (off.value, dist.value)
    return (res, {**st.as_dict(), **ls.as_dict()}) if stats else res


def nn_dists_lb(query, series, window: int, ub: float = math.inf, stats: bool = False):
    """nn_dists with the lower-bound cascade against the fixed bound ub."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    out = torch.empty(x.numel() - q.numel() + 1, device=x.device, dtype=torch.float32)
    st, ls = Stats(), LbStats()
    ctx.check(ctx._lib.eapdtw_nn_dists_lb(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                          int(window), float(ub), _ptr(out),
                                          ctypes.byref(st) if stats else None,
                                          ctypes.byref(ls) if stats else None))
    return (out, {**st.as_dict(), **ls.as_dict()}) if stats else out


def knn_search(query, series, window: int, k: int, stats: bool = False):
    """The k nearest candidate offsets: a list of (offset, distance) in
    (distance, offset) order (offset -1 / distance inf past the available
    offsets)."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    kk = int(k)
    offs = (ctypes.c_int64 * max(kk, 1))()
    dists = (ctypes.c_double * max(kk, 1))()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_knn_search(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                         int(window), kk, offs, dists,
                                         ctypes.byref(st) if stats else None))
    res = [(offs[i], dists[i]) for i in range(kk)]
    return (res, st.as_dict()) if stats else res


def erp_pairs(X, Y, window: int, g: float = 0.0, ub=None, stats: bool = False):
    """ERP (edit distance with real penalty, gap value g) of every row pair
    (X[p], Y[p]) of two [npairs, len] float32 device tensors under the window
    (at most 64 after clamping to len - 1); with ub (a [npairs] tensor) the
    distance if <= ub[p], else +inf."""
    x, y = _dev(X), _dev(Y)
    if x.dim() != 2 or x.shape != y.shape:
        raise ValueError("X and Y must be [npairs, len] tensors of one shape")
    u = None
    if ub is not None:
        u = _dev(ub, x.device.index)
        if u.numel() != x.shape[0]:
            raise ValueError("ub must hold one bound per pair")
    ctx = context(x.device.index)
    ctx.bind_stream()
    out = torch.empty(x.shape[0], device=x.device, dtype=torch.float32)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_erp_pairs(ctx.handle, _ptr(x), _ptr(y), x.shape[0], x.shape[1],
                                        int(window), float(g), _ptr(u) if u is not None else None,
                                        _ptr(out), ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def nn_search_erp(query, series, window: int, g: float = 0.0, stats: bool = False):
    """Nearest-neighbour search under ERP (gap value g in normalised units,
    window at most 64 after clamping to m - 1): (offset, distance)."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    off = ctypes.c_int64()
    dist = ctypes.c_double()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_search_erp(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                            int(window), float(g), ctypes.byref(off),
                                            ctypes.byref(dist), ctypes.byref(st) if stats else None))
    res = (off.value, dist.value)
    return (res, st.as_dict()) if stats else res


def knn_search_lb(query, series, window: int, k: int, stats: bool = False):
    """knn_search with the lower-bound cascade in front of the DTW (the k-th
    best distance as the bound in force).  With stats=True returns
    (list, stats) where stats also holds the cascade's counters."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    kk = int(k)
    offs = (ctypes.c_int64 * max(kk, 1))()
    dists = (ctypes.c_double * max(kk, 1))()
    st, ls = Stats(), LbStats()
    ctx.check(ctx._lib.eapdtw_knn_search_lb(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                            int(window), kk, offs, dists,
                                            ctypes.byref(st) if stats else None,
                                            ctypes.byref(ls) if stats else None))
    res = [(offs[i], dists[i]) for i in range(kk)]
    return (res, {**st.as_dict(), **ls.as_dict()}) if stats else res


def nn_search_w(query, series, window: int, g: float, stats: bool = False):
    """nn_search under weighted DTW (cost w(|i-j|) (a-b)^2, modified logistic
    weight with parameter g)."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    off = ctypes.c_int64()
    dist = ctypes.c_double()
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_search_w(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                          int(window), float(g), ctypes.byref(off),
                                          ctypes.byref(dist), ctypes.byref(st) if stats else None))
    res = (off.value, dist.value)
    return (res, st.as_dict()) if stats else res


def nn_dists_w(query, series, window: int, g: float, ub: float = math.inf, stats: bool = False):
    """nn_dists under weighted DTW."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    out = torch.empty(x.numel() - q.numel() + 1, device=x.device, dtype=torch.float32)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn_dists_w(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                         int(window), float(g), float(ub), _ptr(out),
                                         ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def nn1(X, window: int, stats: bool = False):
    """Leave-one-out nearest neighbour of every row of X [N][len]: (index,
    distance) numpy arrays, the smaller index among equal distances."""
    import numpy as np

    X = _dev(X)
    assert X.dim() == 2, "X must be [N][len]"
    N, L = X.shape
    ctx = context(X.device.index)
    ctx.bind_stream()
    idx = np.empty(N, dtype=np.int64)
    dist = np.empty(N, dtype=np.float64)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn1(ctx.handle, _ptr(X), N, L, int(window),
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  dist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(st) if stats else None))
    return ((idx, dist), st.as_dict()) if stats else (idx, dist)


def nn1_ref(Q, R, window: int, stats: bool = False):
    """Nearest neighbour of every row of the test set Q [nq][len] among the rows
    of the reference set R [nr][len]: (index, distance) numpy arrays."""
    import numpy as np

    Q, R = _dev(Q), _dev(R)
    assert Q.dim() == 2 and R.dim() == 2 and Q.shape[1] == R.shape[1], "Q, R must be [n][len]"
    nq, L = Q.shape
    ctx = context(Q.device.index)
    ctx.bind_stream()
    idx = np.empty(nq, dtype=np.int64)
    dist = np.empty(nq, dtype=np.float64)
    st = Stats()
    ctx.check(ctx._lib.eapdtw_nn1_ref(ctx.handle, _ptr(Q), nq, _ptr(R), R.shape[0], L, int(window),
                                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      dist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(st) if stats else None))
    return ((idx, dist), st.as_dict()) if stats else (idx, dist)


def nn_lower_bounds(query, series, window: int):
    """(LB_Kim, LB_Keogh query envelope, LB_Keogh candidate envelope) of every
    candidate offset, float32 tensors on the series' device."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    K = x.numel() - q.numel() + 1
    out = [torch.empty(max(K, 0), device=x.device, dtype=torch.float32) for _ in range(3)]
    ctx.check(ctx._lib.eapdtw_nn_lower_bounds(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                              int(window), _ptr(out[0]), _ptr(out[1]),
                                              _ptr(out[2])))
    return tuple(out)


def autotune(query, series, window: int, sample_n: int = 1 << 18) -> dict:
    """Times the kernel choices for (len(query), window) on a sample of the
    series, records the fastest in the context's cache and returns it."""
    q, x = _dev(query), _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    t = Tune()
    ctx.check(ctx._lib.eapdtw_autotune(ctx.handle, _ptr(q), q.numel(), _ptr(x), x.numel(),
                                       int(window), int(sample_n), ctypes.byref(t)))
    return t.as_dict()


def tune_bucket(m: int, window: int) -> int:
    return int(_lib.load().eapdtw_tune_bucket(int(m), int(window)))


def tune_get(m: int, window: int, device: int | None = None):
    """The cached choices of (m, window)'s bucket, or None."""
    ctx = context(device)
    t = Tune()
    rc = ctx._lib.eapdtw_tune_get(ctx.handle, tune_bucket(m, window), ctypes.byref(t))
    return t.as_dict() if rc == 0 else None


def tune_save(path: str, device: int | None = None):
    ctx = context(device)
    ctx.check(ctx._lib.eapdtw_tune_save(ctx.handle, str(path).encode()))


def tune_load(path: str, device: int | None = None):
    ctx = context(device)
    ctx.check(ctx._lib.eapdtw_tune_load(ctx.handle, str(path).encode()))


def window_stats(series, m: int):
    x = _dev(series)
    ctx = context(x.device.index)
    ctx.bind_stream()
    K = x.numel() - m + 1
    mean = torch.empty(max(K, 0), device=x.device, dtype=torch.float64)
    sd = torch.empty(max(K, 0), device=x.device, dtype=torch.float64)
    ctx.check(ctx._lib.eapdtw_window_stats(ctx.handle, _ptr(x), x.numel(), int(m), _ptr(mean),
                                           _ptr(sd)))
    return mean, sd


def znorm(x):
    x = _dev(x)
    ctx = context(x.device.index)
    ctx.bind_stream()
    out = torch.empty_like(x)
    ctx.check(ctx._lib.eapdtw_znorm(ctx.handle, _ptr(x), x.numel(), _ptr(out)))
    return out


def unpack_ranges(rng: torch.Tensor):
    """(lo, hi) int64 tensors of packed path ranges (lo | hi << 16)."""
    r = rng.to(torch.int64) & 0xFFFFFFFF
    return r & 0xFFFF, r >> 16


def dtw_path(S, T, window: int):
    """(distances, rowrng, colrng) of equal-length pairs S, T [npairs, len]:
    the optimal warping path the backward follows, as packed ranges per row
    (columns jlo..jhi) and per column (rows ilo..ihi); see unpack_ranges."""
    S, T = _dev(S), _dev(T)
    if S.shape != T.shape or S.dim() != 2:
        raise ValueError("S and T must both be [npairs, len]")
    ctx = context(S.device.index)
    ctx.bind_stream()
    P, L = S.shape
    dist = torch.empty(P, device=S.device, dtype=torch.float32)
    rr = torch.zeros((P, L), device=S.device, dtype=torch.int32)
    cr = torch.zeros((P, L), device=S.device, dtype=torch.int32)
    ctx.check(ctx._lib.eapdtw_dtw_path(ctx.handle, _ptr(S), _ptr(T), P, L, int(window), _ptr(dist),
                                       _ptr(rr), _ptr(cr)))
    return dist, rr, cr


def dtw_kernel_class(npairs: int, len_: int, window: int, recorded: bool, device=None) -> dict:
    """The wavefront kernel class eapdtw_dtw_fwd picks for such a batch: lanes
    per pair, rows per lane and, for a recorded forward, whether the codes stay
    in LDS."""
    ctx = context(device)
    lanes, slots, lds = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    ctx.check(ctx._lib.eapdtw_dtw_kernel_class(ctx.handle, int(npairs), int(len_), int(window),
                                               1 if recorded else 0, ctypes.byref(lanes),
                                               ctypes.byref(slots), ctypes.byref(lds)))
    return {"lanes": lanes.value, "slots": slots.value, "codes_in_lds": bool(lds.value)}


def pack_pairs(S_list, T_list, windows, device=None):
    """Pools and descriptors of an uneven batch: S_list / T_list are sequences
    of 1-D series, windows an int or a sequence.  Returns (S_pool, T_pool,
    pairs), pairs a ctypes array of Pair (host)."""
    n = len(S_list)
    if len(T_list) != n:
        raise ValueError("S_list and T_list differ in length")
    if isinstance(windows, int):
        windows = [windows] * n
    Ss = [_dev(x, device).reshape(-1) for x in S_list]
    Ts = [_dev(x, device).reshape(-1) for x in T_list]
    dev = Ss[0].device if n else torch.device("cuda", torch.cuda.current_device())
    S_pool = torch.cat(Ss) if n else torch.empty(0, device=dev)
    T_pool = torch.cat(Ts) if n else torch.empty(0, device=dev)
    pairs = (Pair * max(n, 1))()
    so = to = 0
    for p in range(n):
        pairs[p].s_off, pairs[p].s_len = so, Ss[p].numel()
        pairs[p].t_off, pairs[p].t_len = to, Ts[p].numel()
        pairs[p].window = int(windows[p])
        so += Ss[p].numel()
        to += Ts[p].numel()
    return S_pool, T_pool, pairs


def dtw_pairs_batch(S_list, T_list, windows, ub=None, stats: bool = False):
    """DTW of pairs of uneven length and window (one launch per lane class);
    ub: None or a per-pair bound (a distance strictly above it is +inf)."""
    S_pool, T_pool, pairs = pack_pairs(S_list, T_list, windows)
    n = len(S_list)
    ctx = context(S_pool.device.index)
    ctx.bind_stream()
    out = torch.empty(n, device=S_pool.device, dtype=torch.float32)
    ubt = None if ub is None else _dev(ub, S_pool.device.index)
    if ubt is not None and ubt.numel() != n:
        raise ValueError("ub must have one entry per pair")
    st = Stats()
    ctx.check(ctx._lib.eapdtw_dtw_pairs_batch(
        ctx.handle, _ptr(S_pool), S_pool.numel(), _ptr(T_pool), T_pool.numel(), pairs, n,
        _ptr(ubt) if ubt is not None else None, _ptr(out), ctypes.byref(st) if stats else None))
    return (out, st.as_dict()) if stats else out


def dtw_batch_path(S_pool, T_pool, pairs, n: int):
    """(rowrng [len(S_pool)], colrng [len(T_pool)]) path ranges of an uneven
    batch (disjoint pairs), pool-shaped; see unpack_ranges."""
    S_pool, T_pool = _dev(S_pool), _dev(T_pool)
    ctx = context(S_pool.device.index)
    ctx.bind_stream()
    rr = torch.zeros(S_pool.numel(), device=S_pool.device, dtype=torch.int32)
    cr = torch.zeros(T_pool.numel(), device=S_pool.device, dtype=torch.int32)
    ctx.check(ctx._lib.eapdtw_dtw_batch_path(ctx.handle, _ptr(S_pool), S_pool.numel(),
                                             _ptr(T_pool), T_pool.numel(), pairs, int(n),
                                             _ptr(rr), _ptr(cr)))
    return rr, cr


def dba_step(B, X, window: int, counts: bool = False):
    """One DBA update of barycentre B [lb] against the series X [n, len]."""
    B, X = _dev(B).reshape(-1), _dev(X)
    if X.dim() != 2:
        raise ValueError("X must be [n, len]")
    ctx = context(B.device.index)
    ctx.bind_stream()
    out = torch.empty_like(B)
    cnt = torch.empty_like(B) if counts else None
    ctx.check(ctx._lib.eapdtw_dba_step(ctx.handle, _ptr(B), B.numel(), _ptr(X), X.shape[0],
                                       X.shape[1], int(window), _ptr(out),
                                       _ptr(cnt) if cnt is not None else None))
    return (out, cnt) if counts else out


from .autograd import DTWBatchFunction, DTWFunction  # noqa: E402
