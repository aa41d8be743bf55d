"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (default options): whole answers where the FP64 oracle can
brute-force them, sampled outputs and size-independent properties otherwise."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_close_array, check_nn, close

pytestmark = pytest.mark.gpu


def _cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def c2():
    q32, x32, windows = gen.c2()
    return q32, x32, windows, torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()


@pytest.mark.parametrize("w", [0, 13, 26, 52])
def test_c2_full_search_vs_brute_force(c2, w):
    """2,000,000-point series, query 256: the oracle scans every offset."""
    q32, x32, _, q, x = c2
    k, d = eap.nn_search(q, x, w)
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(qo, xo, w)
    check_nn(k, d, ko, do, oracle.nn_dists(qo, xo, w, [k])[0])


def test_c2_full_dists_sampled(c2):
    """Every candidate's distance at window 52 (no bound), 4,096 sampled
    against the oracle, the rest against the search's minimum."""
    q32, x32, _, q, x = c2
    d = _cpu(eap.nn_dists(q, x, 52))
    offs = np.sort(gen.rng(4000).choice(d.size, 4096, replace=False))
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), 52, offs)
    assert_close_array(d[offs], want, what="c2 window 52 sampled")
    k, dk = eap.nn_search(q, x, 52)
    assert np.isfinite(d).all()
    assert d.min() == np.float32(dk) and int(np.argmin(d)) == k


@pytest.mark.parametrize("w,k", [(13, 10), (26, 10), (52, 10), (52, 64)])
def test_c2_full_knn_lb_vs_all_distances(c2, w, k):
    """The k nearest neighbours behind the cascade at full size: the k smallest
    of every candidate's distance (nn_dists, no bound), each reported distance
    the candidate's own distance bit for bit, and within tolerance of the
    oracle's distance at that offset."""
    q32, x32, _, q, x = c2
    res = eap.knn_search_lb(q, x, w, k)
    d = _cpu(eap.nn_dists(q, x, w))
    order = np.lexsort((np.arange(d.size), d))[:k]
    got = np.array([dd for _, dd in res])
    assert np.allclose(got, d[order].astype(np.float64), rtol=1e-5, atol=1e-6)
    offs = [o for o, _ in res]
    assert len(set(offs)) == k and all(o >= 0 for o in offs)
    assert all(d[o] == np.float32(dd) for o, dd in res)
    at = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, offs)
    for (o, dd), a in zip(res, at):
        assert close(dd, a), (o, dd, a)


@pytest.mark.parametrize("w", [13, 26, 52])
def test_erp_full_batch_sampled(w):
    """ERP of the 262,144-pair batch the benchmark times (length 256, g = 0):
    512 sampled pairs against the oracle within the float32 summation bound
    (2 len + 2) u, doubled; repeated pairs give the same bits."""
    X, Y = gen.erp_pairs()
    d = _cpu(eap.erp_pairs(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), w, 0.0))
    assert d.size == X.shape[0] and np.isfinite(d).all()
    idx = np.sort(gen.rng(7301).choice(d.size, 512, replace=False))
    want = oracle.erp_pairs(gen.as_oracle(X[idx]), gen.as_oracle(Y[idx]), w, 0.0)
    tol = 2 * (2 * X.shape[1] + 2) * 2.0 ** -24
    assert np.all(np.abs(d[idx] - want) <= tol * want + 1e-6)
    assert np.array_equal(d[:4096], d[-4096:])


def test_c3_full_pairwise_sampled():
    """1,999,000 pairs of length 512, full window: 512 sampled pairs against
    the oracle; DTW <= squared Euclidean distance on the same sample."""
    X, w = gen.c3()
    D = _cpu(eap.pairwise(torch.from_numpy(X).cuda(), w))
    N = X.shape[0]
    assert D.size == N * (N - 1) // 2
    g = gen.rng(4001)
    ia = g.integers(0, N - 1, 512)
    ib = np.array([g.integers(i + 1, N) for i in ia])
    k = np.array([eap.pairwise_index(N, int(i), int(j)) for i, j in zip(ia, ib)])
    Xo = gen.as_oracle(X)
    want = oracle.dtw_pairs(Xo, Xo, w, ia, ib)
    assert_close_array(D[k], want, what="c3 sampled")
    ed = np.sum((Xo[ia] - Xo[ib]) ** 2, axis=1)
    assert np.all(D[k] <= ed * (1 + 1e-6))
    assert np.isfinite(D).all() and (D >= 0).all()


@pytest.fixture(scope="module")
def c4():
    return gen.c4()


def test_c4_cut_batch_vs_brute_force(c4):
    """The 64 uneven queries (lengths 64-1024, windows 5-20 %) batched against
    the first 20,000 points of the series: the oracle scans every offset of
    every query (Section 2.2's search)."""
    qs, ws, x32 = c4
    cut = np.ascontiguousarray(x32[:20_000])
    x = torch.from_numpy(cut).cuda()
    batch = eap.nn_search_batch([(torch.from_numpy(q).cuda(), w) for q, w in zip(qs, ws)], x)
    xo = gen.as_oracle(cut)
    for (q32, w), (k, d) in zip(zip(qs, ws), batch):
        qo = gen.as_oracle(q32)
        ko, do = oracle.nn_search(qo, xo, w)
        check_nn(k, d, ko, do, oracle.nn_dists(qo, xo, w, [k])[0])


def test_c4_full_batch_properties(c4):
    """64 uneven queries against 10,000,000 points: the batched answers equal
    the single-query answers; each reported distance is the oracle's DTW at
    the reported offset; no sampled offset (4,096 random ones plus every
    offset within m of the answer) beats it."""
    qs, ws, x32 = c4
    x = torch.from_numpy(x32).cuda()
    qt = [(torch.from_numpy(q).cuda(), w) for q, w in zip(qs, ws)]
    batch = eap.nn_search_batch(qt, x)
    single = [eap.nn_search(q, x, w) for q, w in qt]
    assert batch == single
    xo = gen.as_oracle(x32)
    g = gen.rng(4002)
    for (q32, w), (k, d) in zip(zip(qs, ws), batch):
        qo = gen.as_oracle(q32)
        K = x32.size - q32.size + 1
        at = oracle.nn_dists(qo, xo, w, [k])[0]
        assert close(d, at), (q32.size, w, k, d, at)
        m = q32.size
        offs = np.unique(np.concatenate([g.integers(0, K, 4096),
                                         np.clip(np.arange(k - m, k + m + 1), 0, K - 1)]))
        others = oracle.nn_dists(qo, xo, w, offs)
        assert others.min() >= at * (1 - 1e-5) - 1e-6, (q32.size, w)
