"""Pins of the oracle's lower bounds and cascade search (CPU only).

The bounds are checked against values worked out by hand on the paper's
worked example, closed forms (window 0: LB_Keogh is the squared Euclidean
distance), brute-force invariants (every bound <= DTW under its window on
random tiny inputs) and the brute-force search (the cascade must not change
the answer)."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
S = np.array(GOLD["S"], dtype=np.float64)
T = np.array(GOLD["T"], dtype=np.float64)


def test_envelope_by_hand():
    # T = (1,3,2,1,2,2), window 1: max / min over {t-1, t, t+1} clipped
    U, L = oracle.envelope(T, 1)
    assert U.tolist() == [3, 3, 3, 2, 2, 2]
    assert L.tolist() == [1, 1, 1, 1, 1, 2]
    U, L = oracle.envelope(S, 1)  # S = (3,1,4,4,1,1)
    assert U.tolist() == [3, 4, 4, 4, 4, 1]
    assert L.tolist() == [1, 1, 1, 1, 1, 1]


def test_envelope_closed_forms():
    a = gen.rng(500).standard_normal(40)
    U, L = oracle.envelope(a, 0)
    assert np.array_equal(U, a) and np.array_equal(L, a)
    U, L = oracle.envelope(a, 100)
    assert np.all(U == a.max()) and np.all(L == a.min())
    ramp = np.arange(30, dtype=np.float64)
    U, L = oracle.envelope(ramp, 4)
    t = np.arange(30)
    assert np.array_equal(U, np.minimum(t + 4, 29)) and np.array_equal(L, np.maximum(t - 4, 0))


def test_lb_keogh_worked_example_by_hand():
    # S against the envelope of T (window 1): S_t outside [L_t, U_t] at
    # t = 2 (4 > 3: 1), t = 3 (4 > 2: 4), t = 5 (1 < 2: 1) -> 6 <= DTW_1 = 11
    U, L = oracle.envelope(T, 1)
    assert oracle.lb_keogh(S, U, L) == 6.0
    # T against the envelope of S (window 1): only t = 5 (2 > 1: 1)
    U, L = oracle.envelope(S, 1)
    assert oracle.lb_keogh(T, U, L) == 1.0
    assert oracle.dtw(S, T, 1) == 11.0


def test_lb_keogh_window_zero_is_squared_ed():
    for a, b in ((S, T), (T, S)):
        U, L = oracle.envelope(b, 0)
        assert oracle.lb_keogh(a, U, L) == 23.0  # sum of (S_t - T_t)^2
    g = gen.rng(501)
    a, b = g.standard_normal(50), g.standard_normal(50)
    U, L = oracle.envelope(b, 0)
    assert oracle.lb_keogh(a, U, L) == pytest.approx(np.sum((a - b) ** 2), rel=1e-12)


def test_lb_kim_worked_example_by_hand():
    # levels (cells 0-based (i over S, j over T), cost (S_i - T_j)^2):
    #  1: (0,0) 4 + (5,5) 1                                  = 5
    #  2: front min{(0,1) 0, (1,0) 0, (1,1) 4}               = 0
    #     back  min{(4,5) 1, (5,4) 1, (4,4) 1}               = 1
    #  3: front min{(0,2) 1, (1,2) 1, (2,2) 4, (2,1) 1, (2,0) 9} = 1
    #     back  min{(3,3) 9, (3,4) 4, (3,5) 4, (4,3) 0, (5,3) 0} = 0
    assert oracle.lb_kim(S, T) == 7.0
    assert oracle.lb_kim(S, T) <= GOLD["dtw"]


def test_lb_kim_short_series():
    # m = 1: no level is disjoint from its mirror, bound 0; m = 2, 3: one level
    assert oracle.lb_kim([2.0], [5.0]) == 0.0
    assert oracle.lb_kim([1.0, 2.0], [3.0, 5.0]) == 4.0 + 9.0
    assert oracle.lb_kim([1.0, 0.0, 2.0], [3.0, 7.0, 5.0]) == 4.0 + 9.0


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 9, 12])
def test_bounds_below_dtw_brute_force(m):
    """Every bound is at most DTW under its window, on random tiny inputs,
    including ties (small integer values) and windows wider than the series."""
    g = gen.rng(502, m)
    for trial in range(300):
        if trial % 2:
            q, c = g.integers(0, 3, m).astype(np.float64), g.integers(0, 3, m).astype(np.float64)
        else:
            q, c = g.standard_normal(m), g.standard_normal(m)
        r = int(g.integers(0, m + 1))
        d = oracle.dtw(q, c, r)
        assert oracle.lb_kim(q, c) <= d + 1e-12
        Uq, Lq = oracle.envelope(q, r)
        Uc, Lc = oracle.envelope(c, r)
        assert oracle.lb_keogh(c, Uq, Lq) <= d + 1e-12
        assert oracle.lb_keogh(q, Uc, Lc) <= d + 1e-12


def test_nn_lower_bounds_below_nn_dists():
    """Per candidate of a z-normalised search: each bound <= the candidate's
    DTW; the candidate envelope reaching past the candidate stays a bound."""
    g = gen.rng(503)
    x = gen.random_walk(600, g)
    x[200:260] = 1.5  # flat stretch: windows normalise to all zeros
    q = gen.random_walk(40, g)
    offs = np.arange(x.size - q.size + 1)
    for r in (0, 1, 4, 13, 39):
        kim, eq, ec = oracle.nn_lower_bounds(q, x, r, offs)
        d = oracle.nn_dists(q, x, r, offs)
        assert np.all(kim <= d + 1e-9) and np.all(eq <= d + 1e-9) and np.all(ec <= d + 1e-9), r
        if r == 0:  # both envelopes are the series themselves
            np.testing.assert_allclose(eq, d, rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(ec, d, rtol=1e-12, atol=1e-12)


def test_nn_lower_bounds_flat_candidate():
    """A flat candidate normalises to zeros: LB_Keogh with its envelope is the
    query's squared norm (every query point pays its own square), equal to the
    DTW of any window."""
    q = gen.random_walk(30, gen.rng(504))
    x = np.concatenate([gen.random_walk(50, gen.rng(505)), np.full(40, 2.0)])
    k = 55
    zq = oracle.znorm(q)
    for r in (0, 3, 29):
        kim, eq, ec = oracle.nn_lower_bounds(q, x, r, [k])
        assert ec[0] == pytest.approx(np.sum(zq ** 2), rel=1e-12)
        assert ec[0] == pytest.approx(oracle.nn_dists(q, x, r, [k])[0], rel=1e-12)


@pytest.mark.parametrize("w", [1, 5, 13, 30])
def test_cascade_search_equals_brute_force(w):
    """C1-shaped inputs (random walks, query 128) on a shorter series: the
    cascade returns the brute-force answer; the counts add up."""
    q32, x32, _ = gen.c1(n=3000)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    k, d, counts = oracle.nn_search_lb(q, x, w)
    kb, db = oracle.nn_search(q, x, w)
    assert (k, d) == (kb, db)
    assert sum(counts) == x.size - q.size + 1
    assert counts[3] >= 1


def test_cascade_prunes_planted_search():
    """A planted copy is found at distance 0 and lets the bounds skip most
    candidates."""
    g = gen.rng(506)
    q = gen.random_walk(64, g)
    x = gen.plant(gen.random_walk(4000, g), q, 1234, a=2.0, b=3.0)
    k, d, counts = oracle.nn_search_lb(q, x, 6)
    assert k == 1234 and d == pytest.approx(0.0, abs=1e-9)
    assert counts[0] + counts[1] + counts[2] > 0.5 * (x.size - q.size + 1)
