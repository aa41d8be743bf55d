"""Pins of the oracle's k-nearest-neighbour search (CPU only): k = 1 is the
nearest-neighbour search, a brute force through the single-pair DTW and a
numpy lexicographic sort gives the same list, ties go to the smaller offset,
planted copies come first, and fewer offsets than k return all of them."""
import numpy as np
import pytest

import gen
import oracle


def _brute(q, x, w, k):
    m = q.size
    zq = oracle.znorm(q)
    d = np.array([oracle.dtw(zq, oracle.znorm(x[t:t + m]), w) for t in range(x.size - m + 1)])
    order = np.lexsort((np.arange(d.size), d))[:k]
    return [(int(t), float(d[t])) for t in order]


@pytest.mark.parametrize("w,k", [(0, 3), (2, 5), (6, 1), (6, 17), (30, 8)])
def test_knn_brute_force(w, k):
    g = gen.rng(600, w * 100 + k)
    q, x = gen.random_walk(24, g), gen.random_walk(400, g)
    assert oracle.knn_search(q, x, w, k) == _brute(q, x, w, k)


def test_knn_one_is_nn_search():
    q32, x32, _ = gen.c1(n=3000)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    (k, d), = oracle.knn_search(q, x, 13, 1)
    assert (k, d) == oracle.nn_search(q, x, 13)


def test_knn_ties_go_to_smaller_offset():
    # a periodic series: every period repeats the same windows exactly
    pattern = gen.random_walk(16, gen.rng(601))
    x = np.tile(pattern, 20)
    q = x[5:5 + 12] + 0.01 * gen.rng(602).standard_normal(12)
    res = oracle.knn_search(q, x, 3, 6)
    ds = [d for _, d in res]
    assert ds == sorted(ds)
    # equal distances appear in increasing offset order; the best six are
    # offsets 5, 21, 37, ... (one per period, all at the same distance)
    assert [k for k, _ in res] == [5 + 16 * j for j in range(6)]
    assert len(set(ds)) == 1


def test_knn_planted_copies_first():
    g = gen.rng(603)
    q = gen.random_walk(32, g)
    x = gen.random_walk(2000, g)
    x[300:332] = 2.0 * q + 1.0
    x[1500:1532] = 0.5 * q - 3.0
    res = oracle.knn_search(q, x, 4, 3)
    assert [k for k, _ in res[:2]] == [300, 1500]
    assert res[0][1] < 1e-9 and res[1][1] < 1e-9 and res[2][1] > 1e-6


def test_knn_more_than_offsets():
    g = gen.rng(604)
    q, x = gen.random_walk(10, g), gen.random_walk(14, g)
    res = oracle.knn_search(q, x, 2, 20)
    assert len(res) == 5 and res == _brute(q, x, 2, 20)


def _nn1_brute(X, w):
    N = X.shape[0]
    out = []
    for i in range(N):
        best = None
        for j in range(N):
            if j != i:
                d = oracle.dtw(X[i], X[j], w)
                if best is None or d < best[1]:
                    best = (j, d)
        out.append(best)
    return out


@pytest.mark.parametrize("w", [0, 3, 20])
def test_nn1_brute_force(w):
    X = gen.rng(605, w).standard_normal((30, 20))
    X[17] = X[4]  # an exact duplicate: each is the other's neighbour at 0
    X[25] = X[4]  # three copies: ties go to the smaller index
    oj, od = oracle.nn1(X, w)
    assert [(int(j), float(d)) for j, d in zip(oj, od)] == _nn1_brute(X, w)
    assert oj[4] == 17 and oj[17] == 4 and oj[25] == 4 and od[4] == 0.0


def test_nn1_two_series():
    X = gen.rng(606).standard_normal((2, 9))
    oj, od = oracle.nn1(X, 2)
    assert oj.tolist() == [1, 0] and od[0] == od[1] == oracle.dtw(X[0], X[1], 2)


@pytest.mark.parametrize("w", [0, 4, 30])
def test_nn1_ref_brute_force(w):
    g = gen.rng(607, w)
    Q, R = g.standard_normal((12, 16)), g.standard_normal((40, 16))
    R[9] = Q[5]    # a copy of a test series: its neighbour at 0
    R[31] = Q[5]   # a second copy: the smaller index wins
    oj, od = oracle.nn1_ref(Q, R, w)
    for i in range(12):
        ds = [oracle.dtw(Q[i], R[j], w) for j in range(40)]
        assert (int(oj[i]), float(od[i])) == (int(np.argmin(ds)), float(min(ds)))
    assert oj[5] == 9 and od[5] == 0.0
