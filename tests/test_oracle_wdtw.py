"""Pins of the oracle's weighted DTW (CPU only): a brute force over every
warping path with the weighted cost, the constant-weight closed form
(g = 0: every weight 1/2, half the DTW), window 0 (w(0) times the squared
Euclidean distance), the weight function's closed-form values, and the search
against its brute-force definition."""
import math

import numpy as np
import pytest

import gen
import oracle


def _brute_force_w(S, T, r, wt):
    lS, lT = len(S), len(T)
    best = math.inf

    def walk(i, j, acc):
        nonlocal best
        if abs(i - j) > r:
            return
        acc += wt[abs(i - j)] * (S[i - 1] - T[j - 1]) ** 2
        if acc >= best:
            return
        if i == lS and j == lT:
            best = acc
            return
        if i < lS and j < lT:
            walk(i + 1, j + 1, acc)
        if i < lS:
            walk(i + 1, j, acc)
        if j < lT:
            walk(i, j + 1, acc)

    walk(1, 1, 0.0)
    return best


def test_weights_closed_form():
    wt = oracle.wdtw_weights(10, 0.3)
    k = np.arange(10)
    np.testing.assert_allclose(wt, 1.0 / (1.0 + np.exp(-0.3 * (k - 5.0))), rtol=1e-15)
    assert wt[5] == 0.5 and np.all(np.diff(wt) > 0)
    assert np.all(oracle.wdtw_weights(7, 0.0) == 0.5)


def test_wdtw_brute_force():
    g = np.random.default_rng(700)
    for _ in range(150):
        lS, lT = (int(v) for v in g.integers(1, 7, 2))
        r = int(g.integers(0, 7))
        gg = float(g.uniform(0.0, 1.5))
        S, T = g.standard_normal(lS), g.standard_normal(lT)
        wt = oracle.wdtw_weights(max(lS, lT), gg)
        a, b = oracle.wdtw(S, T, r, gg), _brute_force_w(S, T, r, wt)
        if math.isinf(b):
            assert math.isinf(a)
        else:
            assert abs(a - b) <= 1e-12 * max(1.0, b), (S, T, r, gg)


def test_wdtw_constant_weight_and_window_zero():
    g = gen.rng(701)
    S, T = g.standard_normal(40), g.standard_normal(40)
    for r in (0, 3, 39):
        assert oracle.wdtw(S, T, r, 0.0) == pytest.approx(0.5 * oracle.dtw(S, T, r), rel=1e-13)
    w0 = oracle.wdtw_weights(40, 0.2)[0]
    assert oracle.wdtw(S, T, 0, 0.2) == pytest.approx(w0 * np.sum((S - T) ** 2), rel=1e-13)
    # the paper's worked example: DTW 9 at full window, weights all 1/2 at g = 0
    assert oracle.wdtw([3, 1, 4, 4, 1, 1], [1, 3, 2, 1, 2, 2], 6, 0.0) == 4.5


def test_wdtw_search_brute_force():
    g = gen.rng(702)
    q, x = g.standard_normal(16).cumsum(), g.standard_normal(300).cumsum()
    for w, gg in ((0, 0.1), (3, 0.25), (15, 0.05)):
        k, d = oracle.nn_search_w(q, x, w, gg)
        zq = oracle.znorm(q)
        ds = [oracle.wdtw(zq, oracle.znorm(x[t:t + 16]), w, gg) for t in range(x.size - 15)]
        assert k == int(np.argmin(ds)) and d == ds[k]
