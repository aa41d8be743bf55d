"""FP64 CPU oracle for early-abandoning pruned DTW -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this package.  The product path (``paper_2010_05371_amd``) never
does, and shares no code with it.

Thin ctypes wrapper over ``oracle.c`` (plain C, built with gcc).  Every
function is the plain definition from the paper (Herrmann & Webb, arXiv
2010.05371):

* ``dtw``         -- Section 2, Eq. 1-5 with the Sakoe-Chiba window of
  Section 2.1, full (lS+1)x(lT+1) matrix in double precision;
* ``erp``, ``erp_pairs`` -- the edit distance with real penalty (Chen & Ng,
  VLDB 2004), an elastic distance with DTW's three moves and gap costs, of
  the kind the paper's closing outlook names; same matrix and window;
  ``erp_nn_search`` -- the nearest-neighbour search under ERP (every offset,
  z-normalised windows, first minimum);
* ``eap``         -- Section 2.2's threshold contract: DTW if <= ub else +inf;
* ``znorm``       -- z-normalisation (population sigma), the UCR-Suite step the
  paper's search inherits (Section 5);
* ``nn_search``   -- brute-force nearest neighbour over every offset,
  lexicographic minimum of (distance, offset);
* ``dtw_grad``    -- optimal warping path (Section 2) and the gradient of the
  path cost with respect to both series;
* ``path_cost``, ``path_grad``, ``is_warping_path`` -- the cost of a given
  warping path, its gradient, and the definition of a warping path (Section 2;
  used to check a GPU path on its own terms);
* ``dba_step``, ``dba_of_paths`` -- one DTW barycentre averaging update (each
  barycentre point becomes the mean of the values the optimal paths align with
  it), the barycentre use of the path;
* ``eap_model``   -- a model of Algorithm 3 (Section 4), kept only to check the
  threshold contract and the worked example (never a reference value);
  ``eap_scan`` -- the nearest-neighbour scan with that model bounded by the
  shared best-so-far: the paper's method on the CPU, a timed baseline (its
  answer must be the brute-force answer);
* ``envelope``, ``lb_kim``, ``lb_keogh``, ``nn_lower_bounds`` -- the lower
  bounds of Section 2.2 that the search experiments of Section 5 put in front
  of the DTW (LB_Kim, LB_Keogh with the query's and with the candidate's
  envelope);
* ``nn_search_lb`` -- the search with that cascade (a sequential scan; it must
  return the brute-force answer);
* ``knn_search`` -- the k best offsets of the search (every distance, then a
  lexicographic sort of (distance, offset));
* ``nn1`` -- leave-one-out nearest neighbour of every series of a set (every
  pair, then row minima); ``nn1_ref`` -- nearest neighbour of every test
  series in a separate reference set;
* ``wdtw``, ``wdtw_weights``, ``nn_dists_w``, ``nn_search_w`` -- weighted DTW
  (DTW's recurrence, cost w(|i-j|) (a-b)^2 with the modified logistic weight),
  one of the elastic distances with DTW's structure that the paper's outlook
  names, and its search.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, -O2, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ORACLE_LIB names another build of oracle.c (the sanitizer run of the
    # pins loads an AddressSanitizer / UndefinedBehaviorSanitizer build)
    path = os.environ.get("ORACLE_LIB")
    if not path:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        path = _LIB
    lib = ctypes.CDLL(path)
    i64, dp, ip = ctypes.c_int64, _c_double_p, _c_int64_p
    lib.oracle_znorm.argtypes = [dp, i64, dp]
    lib.oracle_znorm.restype = None
    lib.oracle_window_stats.argtypes = [dp, i64, i64, dp, dp]
    lib.oracle_window_stats.restype = None
    lib.oracle_dtw.argtypes = [dp, i64, dp, i64, i64]
    lib.oracle_dtw.restype = ctypes.c_double
    lib.oracle_erp.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double]
    lib.oracle_erp.restype = ctypes.c_double
    lib.oracle_erp_nn_search.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double, ip, dp]
    lib.oracle_erp_nn_search.restype = ctypes.c_int
    lib.oracle_dtw_matrix.argtypes = [dp, i64, dp, i64, i64, dp]
    lib.oracle_dtw_matrix.restype = ctypes.c_int
    lib.oracle_eap.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double]
    lib.oracle_eap.restype = ctypes.c_double
    lib.oracle_dtw_grad.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double, dp, dp, ip, ip, dp, dp]
    lib.oracle_dtw_grad.restype = i64
    lib.oracle_nn_dists.argtypes = [dp, i64, dp, i64, i64, ip, i64, ctypes.c_int, dp]
    lib.oracle_nn_dists.restype = ctypes.c_int
    lib.oracle_nn_search.argtypes = [dp, i64, dp, i64, i64, i64, i64, ctypes.c_int, ip, dp]
    lib.oracle_nn_search.restype = ctypes.c_int
    lib.oracle_eap_scan.argtypes = [dp, i64, dp, i64, i64, ip, i64, ctypes.c_int, ip, dp, ip]
    lib.oracle_eap_scan.restype = ctypes.c_int
    lib.oracle_dtw_pairs.argtypes = [dp, dp, i64, i64, ip, ip, i64, ctypes.c_int, dp]
    lib.oracle_dtw_pairs.restype = ctypes.c_int
    lib.oracle_eap_model.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double, ip, ip, ip, ip]
    lib.oracle_eap_model.restype = ctypes.c_double
    lib.oracle_envelope.argtypes = [dp, i64, i64, dp, dp]
    lib.oracle_envelope.restype = None
    lib.oracle_lb_kim.argtypes = [dp, dp, i64]
    lib.oracle_lb_kim.restype = ctypes.c_double
    lib.oracle_lb_keogh.argtypes = [dp, dp, dp, i64]
    lib.oracle_lb_keogh.restype = ctypes.c_double
    lib.oracle_nn_lower_bounds.argtypes = [dp, i64, dp, i64, i64, ip, i64, dp, dp, dp]
    lib.oracle_nn_lower_bounds.restype = ctypes.c_int
    lib.oracle_nn_search_lb.argtypes = [dp, i64, dp, i64, i64, ip, dp, ip]
    lib.oracle_nn_search_lb.restype = ctypes.c_int
    lib.oracle_knn_search.argtypes = [dp, i64, dp, i64, i64, i64, ctypes.c_int, ip, dp, ip]
    lib.oracle_knn_search.restype = ctypes.c_int
    lib.oracle_nn1.argtypes = [dp, i64, i64, i64, ctypes.c_int, ip, dp]
    lib.oracle_nn1.restype = ctypes.c_int
    lib.oracle_nn1_ref.argtypes = [dp, i64, dp, i64, i64, i64, ctypes.c_int, ip, dp]
    lib.oracle_nn1_ref.restype = ctypes.c_int
    lib.oracle_wdtw_weights.argtypes = [i64, ctypes.c_double, dp]
    lib.oracle_wdtw_weights.restype = None
    lib.oracle_wdtw.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double]
    lib.oracle_wdtw.restype = ctypes.c_double
    lib.oracle_nn_dists_w.argtypes = [dp, i64, dp, i64, i64, ctypes.c_double, ip, i64, ctypes.c_int,
                                      dp]
    lib.oracle_nn_dists_w.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_c_double_p)
    return a.ctypes.data_as(_c_int64_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def znorm(x) -> np.ndarray:
    x = _f64(x)
    z = np.empty_like(x)
    _load().oracle_znorm(_ptr(x), x.size, _ptr(z))
    return z


def window_stats(x, m: int):
    x = _f64(x)
    k = x.size - m + 1
    mu = np.empty(max(k, 0))
    sd = np.empty(max(k, 0))
    if k > 0:
        _load().oracle_window_stats(_ptr(x), x.size, m, _ptr(mu), _ptr(sd))
    return mu, sd


def dtw(S, T, window: int | None = None) -> float:
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    return float(_load().oracle_dtw(_ptr(S), S.size, _ptr(T), T.size, r))


def erp(S, T, window: int | None = None, g: float = 0.0) -> float:
    """The edit distance with real penalty (Chen & Ng 2004; an elastic distance
    of the paper's closing outlook) under the Sakoe-Chiba window: the plain
    full-matrix recurrence, L1 costs, gap value g."""
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    return float(_load().oracle_erp(_ptr(S), S.size, _ptr(T), T.size, r, float(g)))


def erp_pairs(X, Y, window: int, g: float = 0.0, ub=None) -> np.ndarray:
    """ERP of every row pair (X[p], Y[p]); with ub (one bound per pair) the
    threshold contract of Section 2.2: the distance if <= ub[p], else +inf."""
    X, Y = np.atleast_2d(_f64(X)), np.atleast_2d(_f64(Y))
    out = np.array([erp(X[p], Y[p], window, g) for p in range(X.shape[0])])
    if ub is not None:
        out = np.where(out <= np.asarray(ub, dtype=np.float64), out, np.inf)
    return out


def erp_nn_search(query, series, window: int, g: float = 0.0):
    """(offset, distance) of the first smallest ERP between the z-normalised
    query and the z-normalised window at each offset (rows = the window)."""
    q, x = _f64(query), _f64(series)
    k = ctypes.c_int64()
    d = ctypes.c_double()
    rc = _load().oracle_erp_nn_search(_ptr(q), q.size, _ptr(x), x.size, int(window), float(g),
                                      ctypes.byref(k), ctypes.byref(d))
    if rc != 0:
        raise MemoryError("oracle_erp_nn_search")
    return k.value, d.value


def dtw_matrix(S, T, window: int | None = None) -> np.ndarray:
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    out = np.empty((S.size + 1, T.size + 1))
    rc = _load().oracle_dtw_matrix(_ptr(S), S.size, _ptr(T), T.size, r, _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_dtw_matrix")
    return out


def eap(S, T, window: int | None, ub: float) -> float:
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    return float(_load().oracle_eap(_ptr(S), S.size, _ptr(T), T.size, r, float(ub)))


def dtw_grad(S, T, window: int | None, gout: float = 1.0):
    """Returns (dist, dS, dT, path[(i,j) 1-based, from (lS,lT) back to (1,1)], min_gap)."""
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    dS = np.empty(S.size)
    dT = np.empty(T.size)
    pi = np.empty(S.size + T.size, dtype=np.int64)
    pj = np.empty(S.size + T.size, dtype=np.int64)
    dist = np.empty(1)
    gap = np.empty(1)
    n = _load().oracle_dtw_grad(_ptr(S), S.size, _ptr(T), T.size, r, float(gout), _ptr(dS),
                                _ptr(dT), _ptr(pi), _ptr(pj), _ptr(dist), _ptr(gap))
    if n < 0:
        raise MemoryError("oracle_dtw_grad")
    path = list(zip(pi[:n].tolist(), pj[:n].tolist()))
    return float(dist[0]), dS, dT, path, float(gap[0])


def path_cost(S, T, path) -> float:
    """Cost of a warping path (Section 2): the sum of (S(i) - T(j))^2 over its
    cells, path given as 1-based (i, j) pairs in any order."""
    S, T = _f64(S), _f64(T)
    return float(sum((S[i - 1] - T[j - 1]) ** 2 for i, j in path))


def path_grad(S, T, path, gout: float = 1.0):
    """Gradient of a path's cost: dS(i) = 2 g sum (S(i) - T(j)), dT(j) = -2 g
    sum (S(i) - T(j)) over the path cells (1-based (i, j))."""
    S, T = _f64(S), _f64(T)
    dS, dT = np.zeros(S.size), np.zeros(T.size)
    for i, j in path:
        d = 2.0 * (S[i - 1] - T[j - 1]) * gout
        dS[i - 1] += d
        dT[j - 1] -= d
    return dS, dT


def is_warping_path(path, lS: int, lT: int, window: int | None) -> bool:
    """Section 2: a warping path runs from (1,1) to (lS,lT) in steps (1,0),
    (0,1), (1,1); with a window (Section 2.1) every cell has |i - j| <= r.
    path: 1-based cells in order from (1,1)."""
    r = max(lS, lT) if window is None else int(window)
    if not path or tuple(path[0]) != (1, 1) or tuple(path[-1]) != (lS, lT):
        return False
    for (i0, j0), (i1, j1) in zip(path, path[1:]):
        if (i1 - i0, j1 - j0) not in ((1, 0), (0, 1), (1, 1)):
            return False
    return all(abs(i - j) <= r for i, j in path)


def dba_of_paths(lb: int, X, paths) -> np.ndarray:
    """DBA average for given paths: point i of the barycentre becomes the mean
    of the values X[p][j] over the cells (i, j) of path p (1-based cells)."""
    X = [np.asarray(x, dtype=np.float64) for x in X]
    s, c = np.zeros(lb), np.zeros(lb)
    for x, path in zip(X, paths):
        for i, j in path:
            s[i - 1] += x[j - 1]
            c[i - 1] += 1.0
    with np.errstate(invalid="ignore", divide="ignore"):
        return s / c


def dba_step(B, X, window: int | None):
    """One DTW barycentre averaging update (Petitjean et al. 2011): the optimal
    path of every pair (B, X[p]) under the window (the backtrack of dtw_grad,
    ties diagonal, then (i-1, j), then (i, j-1)), then dba_of_paths.  Returns
    (new barycentre, counts)."""
    B = _f64(B)
    paths = [dtw_grad(B, x, window)[3] for x in X]
    c = np.zeros(B.size)
    for path in paths:
        for i, _ in path:
            c[i - 1] += 1.0
    return dba_of_paths(B.size, X, paths), c


def nn_dists(query, series, window: int, offsets, nthreads: int | None = None) -> np.ndarray:
    q, x = _f64(query), _f64(series)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    out = np.empty(offs.size)
    rc = _load().oracle_nn_dists(_ptr(q), q.size, _ptr(x), x.size, int(window), _ptr(offs),
                                 offs.size, nthreads or default_threads(), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_nn_dists failed ({rc})")
    return out


def nn_search(query, series, window: int, k_begin: int = 0, k_end: int | None = None,
              nthreads: int | None = None):
    """(best offset, best distance) over offsets [k_begin, k_end)."""
    q, x = _f64(query), _f64(series)
    if k_end is None:
        k_end = x.size - q.size + 1
    bk = np.empty(1, dtype=np.int64)
    bd = np.empty(1)
    rc = _load().oracle_nn_search(_ptr(q), q.size, _ptr(x), x.size, int(window), int(k_begin),
                                  int(k_end), nthreads or default_threads(), _ptr(bk), _ptr(bd))
    if rc != 0:
        raise ValueError(f"oracle_nn_search failed ({rc})")
    return int(bk[0]), float(bd[0])


def dtw_pairs(X, Y, window: int, ia, ib, nthreads: int | None = None) -> np.ndarray:
    X, Y = _f64(X), _f64(Y)
    L = X.shape[1]
    ia = np.ascontiguousarray(np.asarray(ia, dtype=np.int64))
    ib = np.ascontiguousarray(np.asarray(ib, dtype=np.int64))
    out = np.empty(ia.size)
    rc = _load().oracle_dtw_pairs(_ptr(X), _ptr(Y), L, int(window), _ptr(ia), _ptr(ib), ia.size,
                                  nthreads or default_threads(), _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_dtw_pairs")
    return out


def eap_model(S, T, window: int | None, ub: float):
    """Model of Algorithm 3: (value, evaluated cells, per-line pruning point, abandon cell)."""
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    cells = np.zeros(1, dtype=np.int64)
    nl = max(S.size, T.size)
    trace = np.zeros(max(nl, 1), dtype=np.int64)
    ai = np.zeros(1, dtype=np.int64)
    aj = np.zeros(1, dtype=np.int64)
    v = _load().oracle_eap_model(_ptr(S), S.size, _ptr(T), T.size, r, float(ub), _ptr(cells),
                                 _ptr(trace), _ptr(ai), _ptr(aj))
    return float(v), int(cells[0]), trace[:nl].tolist(), (int(ai[0]), int(aj[0]))


def eap_scan(query, series, window: int, offsets, nthreads: int | None = None):
    """The paper's method on the CPU: nearest-neighbour scan of the listed
    offsets with the EAPrunedDTW model (Algorithm 3) bounded by the shared
    best-so-far.  Returns (best offset, distance, evaluated cells)."""
    q, x = _f64(query), _f64(series)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    bk = np.zeros(1, dtype=np.int64)
    bd = np.zeros(1)
    cells = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_eap_scan(_ptr(q), q.size, _ptr(x), x.size, int(window), _ptr(offs),
                                 offs.size, nthreads or default_threads(), _ptr(bk), _ptr(bd),
                                 _ptr(cells))
    if rc != 0:
        raise RuntimeError(f"oracle_eap_scan failed ({rc})")
    return int(bk[0]), float(bd[0]), int(cells[0])


def envelope(a, window: int):
    """(U, L): running max and min of a over [t - r, t + r], clipped to the series."""
    a = _f64(a)
    U, L = np.empty_like(a), np.empty_like(a)
    _load().oracle_envelope(_ptr(a), a.size, int(window), _ptr(U), _ptr(L))
    return U, L


def lb_kim(q, c) -> float:
    """LB_Kim of two equal-length series (three levels from each end)."""
    q, c = _f64(q), _f64(c)
    assert q.size == c.size
    return float(_load().oracle_lb_kim(_ptr(q), _ptr(c), q.size))


def lb_keogh(a, U, L) -> float:
    """Sum of squared distances from a[t] to [L[t], U[t]]."""
    a, U, L = _f64(a), _f64(U), _f64(L)
    return float(_load().oracle_lb_keogh(_ptr(a), _ptr(U), _ptr(L), a.size))


def nn_lower_bounds(query, series, window: int, offsets):
    """(kim, eq, ec) arrays of the listed candidates of the z-normalised search."""
    q, x = _f64(query), _f64(series)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    kim, eq, ec = np.empty(offs.size), np.empty(offs.size), np.empty(offs.size)
    rc = _load().oracle_nn_lower_bounds(_ptr(q), q.size, _ptr(x), x.size, int(window),
                                        _ptr(offs), offs.size, _ptr(kim), _ptr(eq), _ptr(ec))
    if rc != 0:
        raise ValueError(f"oracle_nn_lower_bounds failed ({rc})")
    return kim, eq, ec


def nn_search_lb(query, series, window: int):
    """(best offset, best distance, counts) of the cascade search; counts =
    (skipped by LB_Kim, by LB_Keogh query envelope, by LB_Keogh candidate
    envelope, DTW computed)."""
    q, x = _f64(query), _f64(series)
    bk = np.empty(1, dtype=np.int64)
    bd = np.empty(1)
    counts = np.empty(4, dtype=np.int64)
    rc = _load().oracle_nn_search_lb(_ptr(q), q.size, _ptr(x), x.size, int(window), _ptr(bk),
                                     _ptr(bd), _ptr(counts))
    if rc != 0:
        raise ValueError(f"oracle_nn_search_lb failed ({rc})")
    return int(bk[0]), float(bd[0]), tuple(int(c) for c in counts)


def knn_search(query, series, window: int, k: int, nthreads: int | None = None):
    """The k smallest (offset, distance) pairs of the search, ordered by
    (distance, offset); all offsets when there are fewer than k."""
    q, x = _f64(query), _f64(series)
    ok = np.empty(max(k, 1), dtype=np.int64)
    od = np.empty(max(k, 1))
    cnt = np.empty(1, dtype=np.int64)
    rc = _load().oracle_knn_search(_ptr(q), q.size, _ptr(x), x.size, int(window), int(k),
                                   nthreads or default_threads(), _ptr(ok), _ptr(od), _ptr(cnt))
    if rc != 0:
        raise ValueError(f"oracle_knn_search failed ({rc})")
    c = int(cnt[0])
    return [(int(ok[t]), float(od[t])) for t in range(c)]


def nn1(X, window: int, nthreads: int | None = None):
    """(index, distance) arrays: for each row i of X [N][L], the row j != i with
    the smallest DTW (smaller j on ties)."""
    X = _f64(X)
    N, L = X.shape
    oj = np.empty(N, dtype=np.int64)
    od = np.empty(N)
    rc = _load().oracle_nn1(_ptr(X), N, L, int(window), nthreads or default_threads(), _ptr(oj),
                            _ptr(od))
    if rc != 0:
        raise ValueError(f"oracle_nn1 failed ({rc})")
    return oj, od


def wdtw_weights(length: int, g: float) -> np.ndarray:
    """w(k) = 1 / (1 + exp(-g (k - length/2))) for k = 0..length-1."""
    wt = np.empty(max(int(length), 1))
    _load().oracle_wdtw_weights(int(length), float(g), _ptr(wt))
    return wt[:int(length)]


def wdtw(S, T, window: int | None, g: float) -> float:
    S, T = _f64(S), _f64(T)
    r = max(S.size, T.size) if window is None else int(window)
    return float(_load().oracle_wdtw(_ptr(S), S.size, _ptr(T), T.size, r, float(g)))


def nn_dists_w(query, series, window: int, g: float, offsets,
               nthreads: int | None = None) -> np.ndarray:
    q, x = _f64(query), _f64(series)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    out = np.empty(offs.size)
    rc = _load().oracle_nn_dists_w(_ptr(q), q.size, _ptr(x), x.size, int(window), float(g),
                                   _ptr(offs), offs.size, nthreads or default_threads(), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_nn_dists_w failed ({rc})")
    return out


def nn_search_w(query, series, window: int, g: float):
    """(best offset, best weighted-DTW distance) over every offset (the first
    offset among equal minima)."""
    q = _f64(query)
    d = nn_dists_w(query, series, window, g, np.arange(_f64(series).size - q.size + 1))
    k = int(np.argmin(d))
    return k, float(d[k])


def nn1_ref(Q, R, window: int, nthreads: int | None = None):
    """(index, distance) arrays: for each row i of Q [nq][L], the row j of R
    [nr][L] with the smallest DTW (smaller j on ties)."""
    Q, R = _f64(Q), _f64(R)
    nq, L = Q.shape
    oj = np.empty(nq, dtype=np.int64)
    od = np.empty(nq)
    rc = _load().oracle_nn1_ref(_ptr(Q), nq, _ptr(R), R.shape[0], L, int(window),
                                nthreads or default_threads(), _ptr(oj), _ptr(od))
    if rc != 0:
        raise ValueError(f"oracle_nn1_ref failed ({rc})")
    return oj, od
