"""Pins of the oracle's ERP (the edit distance with real penalty of Chen & Ng,
VLDB 2004; an elastic distance of the kind the paper's closing outlook names)
against what holds independently of its recurrence: brute force over every
alignment on tiny inputs, the window-0 closed form (the L1 distance), the
metric properties and the sum lower bound Chen & Ng prove, and hand-worked
examples."""
import itertools

import numpy as np
import pytest

import oracle


def brute_force_erp(S, T, r, g):
    """Minimum over every alignment: monotone paths from (0,0) to (lS,lT) with
    diagonal, vertical and horizontal steps, every visited cell within the
    window (|i-j| <= r), costing |S_i - T_j|, |S_i - g| and |T_j - g|."""
    lS, lT = len(S), len(T)
    best = np.inf
    stack = [(0, 0, 0.0)]
    while stack:
        i, j, c = stack.pop()
        if i == lS and j == lT:
            best = min(best, c)
            continue
        for di, dj in ((1, 1), (1, 0), (0, 1)):
            ni, nj = i + di, j + dj
            if ni > lS or nj > lT or abs(ni - nj) > r:
                continue
            if di and dj:
                step = abs(S[ni - 1] - T[nj - 1])
            elif di:
                step = abs(S[ni - 1] - g)
            else:
                step = abs(T[nj - 1] - g)
            stack.append((ni, nj, c + step))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_erp_equals_brute_force(seed):
    g0 = np.random.default_rng(7100 + seed)
    for lS, lT in itertools.product(range(0, 5), repeat=2):
        S, T = g0.normal(size=lS), g0.normal(size=lT)
        gap = float(g0.normal())
        for r in range(0, 5):
            want = brute_force_erp(S, T, r, gap)
            got = oracle.erp(S, T, r, gap)
            if np.isinf(want):
                assert np.isinf(got), (lS, lT, r)
            else:
                assert got == pytest.approx(want, rel=1e-12, abs=1e-12), (lS, lT, r)


def test_erp_window_zero_is_l1():
    g0 = np.random.default_rng(7110)
    for L in (1, 2, 7, 64):
        S, T = g0.normal(size=L), g0.normal(size=L)
        assert oracle.erp(S, T, 0, float(g0.normal())) == pytest.approx(np.abs(S - T).sum(), rel=1e-12)


def test_erp_metric_properties():
    g0 = np.random.default_rng(7120)
    for _ in range(40):
        a, b, c = (g0.normal(size=int(g0.integers(1, 9))) for _ in range(3))
        gap = float(g0.normal())
        assert oracle.erp(a, a, None, gap) == 0.0
        ab, ba = oracle.erp(a, b, None, gap), oracle.erp(b, a, None, gap)
        assert ab == pytest.approx(ba, rel=1e-12, abs=1e-12)
        assert oracle.erp(a, c, None, gap) <= ab + oracle.erp(b, c, None, gap) + 1e-12


def test_erp_sum_lower_bound():
    """With gap value 0, |sum(S) - sum(T)| <= ERP(S, T) (Chen & Ng)."""
    g0 = np.random.default_rng(7130)
    for _ in range(40):
        S, T = g0.normal(size=int(g0.integers(1, 20))), g0.normal(size=int(g0.integers(1, 20)))
        assert abs(S.sum() - T.sum()) <= oracle.erp(S, T, None, 0.0) + 1e-12


def test_erp_hand_examples():
    # S = (1), T = (2, 3), g = 0: match 1-2 then 3 against the gap, or 2 against
    # the gap then match 1-3: 4 either way; every other alignment costs more
    assert oracle.erp([1.0], [2.0, 3.0], None, 0.0) == 4.0
    assert oracle.erp([1.0], [2.0, 3.0], 1, 0.0) == 4.0
    assert np.isinf(oracle.erp([1.0], [2.0, 3.0], 0, 0.0))  # lengths differ by more than the window
    # S = (0, 1), T = (1, 0): with g = 0 the zeros align with the gap for free
    # and 1 matches 1, so ERP = 0 although S != T; with g = 0.5 the same
    # alignment costs 0.5 + 0 + 0.5 = 1 and every other one more
    assert oracle.erp([0.0, 1.0], [1.0, 0.0], None, 0.0) == 0.0
    assert oracle.erp([0.0, 1.0], [1.0, 0.0], None, 0.5) == 1.0
    assert oracle.erp([], [], 0, 0.3) == 0.0
    assert oracle.erp([], [2.0, -1.0], 2, 0.5) == pytest.approx(1.5 + 1.5)


def test_erp_pairs_threshold_contract():
    g0 = np.random.default_rng(7140)
    X, Y = g0.normal(size=(5, 12)), g0.normal(size=(5, 12))
    full = oracle.erp_pairs(X, Y, 3, 0.1)
    ub = full.copy()
    ub[::2] = full[::2] * 0.999
    out = oracle.erp_pairs(X, Y, 3, 0.1, ub)
    assert np.isinf(out[::2]).all() and (out[1::2] == full[1::2]).all()


def _znorm_np(w):
    sd = w.std()
    return (w - w.mean()) / sd if sd > 0 else np.zeros_like(w)


def test_erp_search_planted_copy_and_window_zero():
    g0 = np.random.default_rng(7150)
    q = g0.normal(size=24).cumsum()
    x = g0.normal(size=600).cumsum()
    x[311:335] = 2.5 * q - 4.0  # an affine copy: the same z-normalised window, ERP 0
    k, d = oracle.erp_nn_search(q, x, 3, 0.2)
    assert k == 311 and d == pytest.approx(0.0, abs=1e-9)
    # window 0: the L1 distance between z-normalised windows, written out with numpy
    x2 = g0.normal(size=400).cumsum()
    zq = _znorm_np(q)
    l1 = [np.abs(_znorm_np(x2[i:i + 24]) - zq).sum() for i in range(400 - 24 + 1)]
    k0, d0 = oracle.erp_nn_search(q, x2, 0, 0.7)
    assert k0 == int(np.argmin(l1)) and d0 == pytest.approx(min(l1), rel=1e-12)


def test_erp_search_ties_take_the_smallest_offset():
    pattern = np.random.default_rng(7160).normal(size=30)
    x = np.tile(pattern, 8)
    k, d = oracle.erp_nn_search(pattern[5:25], x, 4, 0.0)
    assert k == 5 and d == 0.0
