"""Pins for the FP64 oracle (CPU only).

The oracle is checked against things other than itself: the values the paper
prints for its worked example (tests/golden/worked_example.json), brute force
over every warping path on tiny inputs, closed forms (window 0 = squared
Euclidean distance, z-normalised ramps, the window-0 gradient), invariants
(DTW(S,S)=0, symmetry, monotonicity in the window, DTW <= squared ED) and
central finite differences for the path gradient.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
S_EX = np.array(GOLD["S"], dtype=np.float64)
T_EX = np.array(GOLD["T"], dtype=np.float64)


# ----------------------------------------------------------------------------- worked example

def test_worked_example_distance():
    assert oracle.dtw(S_EX, T_EX) == GOLD["dtw"]
    assert oracle.dtw(T_EX, S_EX) == GOLD["dtw"]


def test_worked_example_cells():
    M = oracle.dtw_matrix(S_EX, T_EX)
    for i, j, v in GOLD["cells"]:
        assert M[i, j] == v
    for i, j, ub in GOLD["cells_above_ub"]:
        assert M[i, j] > ub
    assert M[1:, 1:].max() == GOLD["matrix_max"]
    # (2,2) > 6 but some later cell of line 2 is <= 6 (not a pruning point)
    i, j, ub = GOLD["line2_not_pruning_point"]
    assert M[i, j] > ub and (M[i, j + 1:] <= ub).any()


def test_worked_example_window_zero_is_squared_ed():
    assert GOLD["window0_is_squared_ed"]
    assert oracle.dtw(S_EX, T_EX, 0) == float(np.sum((S_EX - T_EX) ** 2))
    # a window as large as the series gives unconstrained DTW
    assert oracle.dtw(S_EX, T_EX, 6) == GOLD["dtw"]


def test_worked_example_threshold():
    assert oracle.eap(S_EX, T_EX, None, 9) == GOLD["ub9_result"]
    assert oracle.eap(S_EX, T_EX, None, 6) == math.inf


def test_worked_example_algorithm3_model():
    v9, _, _, ab9 = oracle.eap_model(S_EX, T_EX, None, 9)
    assert v9 == GOLD["ub9_result"] and ab9 == (0, 0)
    v6, _, trace, ab6 = oracle.eap_model(S_EX, T_EX, None, 6)
    assert v6 == math.inf
    assert list(ab6) == GOLD["ub6_abandon_cell"]
    for i, j in GOLD["ub6_pruning_points"]:
        assert trace[i - 1] == j


# ----------------------------------------------------------------------------- brute force

def _brute_force(S, T, r):
    """Minimum cost over every monotone, continuous warping path inside the window."""
    lS, lT = len(S), len(T)
    best = math.inf
    # enumerate step sequences from (1,1) to (lS,lT); steps (1,0), (0,1), (1,1)
    def walk(i, j, acc):
        nonlocal best
        if abs(i - j) > r:
            return
        acc += (S[i - 1] - T[j - 1]) ** 2
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


def test_brute_force_tiny():
    g = np.random.default_rng(11)
    n = 0
    for lS in range(1, 7):
        for lT in range(1, 7):
            for r in (0, 1, 2, 3, 6):
                S = g.integers(-3, 4, lS).astype(np.float64)
                T = g.integers(-3, 4, lT).astype(np.float64) * 0.5
                assert oracle.dtw(S, T, r) == _brute_force(S, T, r), (S, T, r)
                n += 1
    assert n == 180


def test_brute_force_real_values():
    g = np.random.default_rng(12)
    for _ in range(60):
        lS, lT = g.integers(1, 8, 2)
        r = int(g.integers(0, 8))
        S, T = g.standard_normal(lS), g.standard_normal(lT)
        a, b = oracle.dtw(S, T, r), _brute_force(S, T, r)
        if math.isinf(b):
            assert math.isinf(a)
        else:
            assert abs(a - b) <= 1e-12 * max(1.0, b)


# ----------------------------------------------------------------------------- invariants

def test_empty_series():
    assert oracle.dtw([], [], 3) == 0.0
    assert oracle.dtw([1.0], [], 3) == math.inf
    assert oracle.dtw([], [1.0, 2.0], 3) == math.inf


def test_no_admissible_path():
    assert oracle.dtw(np.zeros(5), np.zeros(9), 3) == math.inf
    assert oracle.dtw(np.zeros(5), np.zeros(8), 3) == 0.0


@pytest.mark.parametrize("L", [1, 17, 64])
def test_invariants(L):
    g = np.random.default_rng(L)
    for _ in range(8):
        S, T = g.standard_normal(L), g.standard_normal(L)
        ed = float(np.sum((S - T) ** 2))
        assert oracle.dtw(S, S, L) == 0.0
        assert oracle.dtw(S, T, 0) == pytest.approx(ed, rel=1e-14)
        prev = math.inf
        for r in range(0, L + 1, max(1, L // 8)):
            d = oracle.dtw(S, T, r)
            assert d <= ed * (1 + 1e-14)
            assert d <= prev * (1 + 1e-14)
            assert d == oracle.dtw(T, S, r)
            prev = d


def test_threshold_contract_against_algorithm3_model():
    """Algorithm 3 (model) reaches exactly DTW when <= ub and +inf otherwise,
    ties included, with and without a window, equal and unequal lengths."""
    g = np.random.default_rng(13)
    checked = 0
    for _ in range(3000):
        lS, lT = (int(v) for v in g.integers(1, 10, 2))
        r = int(g.integers(0, 10))
        S = g.integers(0, 5, lS).astype(np.float64)
        T = g.integers(0, 5, lT).astype(np.float64)
        d = oracle.dtw(S, T, r)
        choices = [d, d - 1, d + 1, 0.0, -1.0, math.inf, d * 0.5]
        for ub in choices:
            if math.isnan(ub):
                continue
            want = oracle.eap(S, T, r, ub)
            got, cells, _, _ = oracle.eap_model(S, T, r, ub)
            assert got == want, (S, T, r, ub)
            assert cells <= lS * lT
            checked += 1
    assert checked > 15000


# ----------------------------------------------------------------------------- z-normalisation

def test_znorm_ramp_closed_form():
    for m in (2, 5, 128):
        t = np.arange(m, dtype=np.float64)
        want = (t - (m - 1) / 2) / math.sqrt((m * m - 1) / 12.0)
        np.testing.assert_allclose(oracle.znorm(t), want, rtol=0, atol=1e-13)
        np.testing.assert_allclose(oracle.znorm(3.5 * t - 7.0), want, rtol=0, atol=1e-13)


def test_znorm_constant_window_is_zero():
    np.testing.assert_array_equal(oracle.znorm(np.full(9, 4.25)), np.zeros(9))


def test_znorm_flat_rule_is_relative_to_the_mean_square():
    """c + e (+1, -1, ...): mean c, sigma e.  Normalised to (+1, -1, ...)
    when e^2 > 1e-14 (c^2 + e^2), else flat (zeros)."""
    alt = np.tile([1.0, -1.0], 8)
    for c, e, flat in ((1000.0, 1e-3, False), (1000.0, 1e-5, True), (0.0, 1e-30, False),
                       (-3.0, 1e-9, True), (-3.0, 1e-6, False)):
        z = oracle.znorm(c + e * alt)
        if flat:
            np.testing.assert_array_equal(z, np.zeros(alt.size))
        else:
            np.testing.assert_allclose(z, alt, rtol=0, atol=1e-6)
        mu, sd = oracle.window_stats(c + e * alt, alt.size)
        assert (sd[0] == 0.0) == flat
        if not flat:
            assert sd[0] == pytest.approx(e, rel=1e-6)


def test_window_stats_ramp():
    x = np.arange(50, dtype=np.float64) * 2.0 + 1.0
    mu, sd = oracle.window_stats(x, 10)
    np.testing.assert_allclose(mu, 2.0 * (np.arange(41) + 4.5) + 1.0, rtol=1e-15)
    np.testing.assert_allclose(sd, np.full(41, 2.0 * math.sqrt(99 / 12.0)), rtol=1e-14)


# ----------------------------------------------------------------------------- NN search

def test_nn_planted_copy_and_affine_invariance():
    q32, x32, r = gen.c1(n=3000, m=64)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    k0 = 1234
    xp = gen.as_oracle(gen.plant(x32, q32, k0, a=2.5, b=-40.0))
    k, d = oracle.nn_search(q, xp, r, nthreads=4)
    assert k == k0 and d < 1e-6
    # affine map of the series with a > 0 leaves the z-normalised search unchanged
    k1, d1 = oracle.nn_search(q, x, r, nthreads=4)
    k2, d2 = oracle.nn_search(q, 3.0 * x + 100.0, r, nthreads=4)
    assert k1 == k2 and d2 == pytest.approx(d1, rel=1e-9)


def test_nn_tie_goes_to_smallest_offset():
    g = np.random.default_rng(5)
    q = g.standard_normal(16)
    x = g.standard_normal(400) * 3.0
    x[300:316] = q
    x[40:56] = q
    k, d = oracle.nn_search(q, x, 2, nthreads=3)
    assert k == 40 and d < 1e-20


def test_nn_independent_of_threads():
    q32, x32, r = gen.c1(n=1500, m=32)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    a = oracle.nn_search(q, x, r, nthreads=1)
    b = oracle.nn_search(q, x, r, nthreads=7)
    assert a == b
    ks = np.arange(0, x.size - 32 + 1)
    d = oracle.nn_dists(q, x, r, ks, nthreads=5)
    # brute force over the per-offset distances, scanned in order
    best = min(range(ks.size), key=lambda t: (d[t], t))
    assert (int(ks[best]), float(d[best])) == a


def test_nn_constant_window_normalises_to_zero():
    q = np.arange(8, dtype=np.float64)
    x = np.concatenate([np.linspace(0, 1, 30) ** 2 * 5, np.full(8, 2.0), np.linspace(3, 1, 30)])
    dists = oracle.nn_dists(q, x, 1, [30])
    zq = oracle.znorm(q)
    assert dists[0] == pytest.approx(oracle.dtw(zq, np.zeros(8), 1), rel=1e-15)


# ----------------------------------------------------------------------------- gradients

def _path_cost(S, T, path):
    return sum((S[i - 1] - T[j - 1]) ** 2 for i, j in path)


def test_grad_window_zero_closed_form():
    g = np.random.default_rng(3)
    S, T = g.standard_normal(20), g.standard_normal(20)
    d, dS, dT, path, _ = oracle.dtw_grad(S, T, 0, gout=1.5)
    np.testing.assert_allclose(dS, 2 * (S - T) * 1.5, rtol=1e-15)
    np.testing.assert_allclose(dT, -2 * (S - T) * 1.5, rtol=1e-15)
    assert path == [(i, i) for i in range(20, 0, -1)]


def test_grad_identical_series_is_zero():
    S = np.random.default_rng(4).standard_normal(33)
    d, dS, dT, _, _ = oracle.dtw_grad(S, S, 5)
    assert d == 0.0 and not dS.any() and not dT.any()


def test_grad_infinite_distance_is_zero():
    d, dS, dT, path, _ = oracle.dtw_grad(np.ones(4), np.ones(9), 2)
    assert d == math.inf and not dS.any() and not dT.any() and path == []


def test_path_is_valid_and_optimal():
    g = np.random.default_rng(6)
    for L, r in ((12, 3), (30, 30), (25, 0), (40, 7)):
        S, T = g.standard_normal(L), g.standard_normal(L)
        d, _, _, path, _ = oracle.dtw_grad(S, T, r)
        assert path[0] == (L, L) and path[-1] == (1, 1)
        for (i0, j0), (i1, j1) in zip(path, path[1:]):
            assert (i0 - i1, j0 - j1) in ((1, 1), (1, 0), (0, 1))
            assert abs(i1 - j1) <= r
        assert _path_cost(S, T, path) == pytest.approx(d, rel=1e-13)


# Path ties (Section 2: several optimal warping paths may exist).  The oracle
# takes, at every backtrack step, the diagonal predecessor, then (i-1, j), then
# (i, j-1) among those holding the minimum.  Among all optimal paths this is
# the one whose step sequence, read from (lS, lT) backwards with the order
# diagonal < top < left, is lexicographically smallest -- a definition the
# tests below evaluate by enumerating every warping path, without the DP
# matrix.

_STEP = {(1, 1): 0, (1, 0): 1, (0, 1): 2}  # diagonal, top (i-1, j), left (i, j-1)


def _all_paths(l1, l2, r):
    out = []

    def rec(i, j, acc):
        if abs(i - j) > r:
            return
        acc.append((i, j))
        if (i, j) == (l1, l2):
            out.append(list(acc))
        else:
            if i < l1 and j < l2:
                rec(i + 1, j + 1, acc)
            if i < l1:
                rec(i + 1, j, acc)
            if j < l2:
                rec(i, j + 1, acc)
        acc.pop()

    rec(1, 1, [])
    return out


def _backward_steps(path_from_start):
    rev = path_from_start[::-1]
    return [_STEP[(a[0] - b[0], a[1] - b[1])] for a, b in zip(rev, rev[1:])]


def _enumerated_choice(S, T, r, rank=(0, 1, 2)):
    """The optimal path (from the end back to (1,1)) that a backtrack preferring
    the steps in `rank` order takes, found by enumeration (exact: integer data)."""
    paths = _all_paths(len(S), len(T), r)
    cost = [sum((S[i - 1] - T[j - 1]) ** 2 for i, j in p) for p in paths]
    best = min(cost)
    opt = [p for p, c in zip(paths, cost) if c == best]
    pick = min(opt, key=lambda p: [rank[c] for c in _backward_steps(p)])
    return pick[::-1], best, len(opt)


def _grad_of_path(S, T, path):
    dS, dT = np.zeros(len(S)), np.zeros(len(T))
    for i, j in path:
        dS[i - 1] += 2 * (S[i - 1] - T[j - 1])
        dT[j - 1] -= 2 * (S[i - 1] - T[j - 1])
    return dS, dT


def test_worked_example_path_and_gradient():
    """The worked example's optimal path has a diagonal/left tie at (6,6); the
    path and gradient were derived by hand from the printed matrix."""
    d, dS, dT, path, _ = oracle.dtw_grad(S_EX, T_EX, None)
    assert d == GOLD["dtw"]
    assert path == [tuple(c) for c in GOLD["path_diag_top_left"]]
    assert dS.tolist() == GOLD["grad_S"] and dT.tolist() == GOLD["grad_T"]


def test_hand_worked_tie_case():
    case = GOLD["tie_case"]
    S, T = np.array(case["S"], float), np.array(case["T"], float)
    M = oracle.dtw_matrix(S, T)
    assert M[1:, 1:].tolist() == case["matrix"]
    d, dS, dT, path, gap = oracle.dtw_grad(S, T, None)
    assert d == case["dtw"] and gap == 0.0
    assert path == [tuple(c) for c in case["path_diag_top_left"]]
    assert dS.tolist() == case["grad_S"] and dT.tolist() == case["grad_T"]


def test_tie_order_against_enumeration():
    """On small integer cases the oracle's path is the enumerated choice, and the
    cases include every kind of tie on the chosen path where another order
    would choose a different path, so a changed tie order fails here."""
    g = np.random.default_rng(2010)
    seen = set()
    other_orders = [(2, 1, 0), (1, 0, 2), (0, 2, 1), (2, 0, 1), (1, 2, 0)]
    decisive = {o: 0 for o in other_orders}
    for _ in range(700):
        L1, L2 = int(g.integers(1, 6)), int(g.integers(1, 6))
        r = int(g.integers(abs(L1 - L2), max(L1, L2) + 1))
        S = g.integers(0, 4, L1).astype(float)
        T = g.integers(0, 4, L2).astype(float)
        want, best, nopt = _enumerated_choice(S, T, r)
        d, dS, dT, path, _ = oracle.dtw_grad(S, T, r)
        assert d == best
        assert path == want, (S, T, r)
        wS, wT = _grad_of_path(S, T, want)
        assert dS.tolist() == wS.tolist() and dT.tolist() == wT.tolist()
        if nopt < 2:
            continue
        M = oracle.dtw_matrix(S, T, r)
        for i, j in want[:-1]:
            pred = (M[i - 1, j - 1], M[i - 1, j], M[i, j - 1])
            tie = tuple(v == min(pred) for v in pred)
            if sum(tie) > 1:
                seen.add(tie)
        for o in other_orders:
            if _enumerated_choice(S, T, r, o)[0] != want:
                decisive[o] += 1
    # diagonal/top, diagonal/left, top/left and three-way ties all occur
    assert {(True, True, False), (True, False, True), (False, True, True),
            (True, True, True)} <= seen, seen
    assert all(v > 0 for v in decisive.values()), decisive


def test_grad_central_finite_differences():
    """With the optimal path fixed, DTW is a quadratic in each coordinate, so the
    central difference is exact up to rounding; skip coordinates whose
    perturbation changes the optimal path."""
    g = np.random.default_rng(7)
    h = 1e-4
    checked = 0
    for _ in range(6):
        L, r = 24, 5
        S, T = g.standard_normal(L), g.standard_normal(L)
        d, dS, dT, path, gap = oracle.dtw_grad(S, T, r, gout=1.0)
        for which, base, grad in (("S", S, dS), ("T", T, dT)):
            for k in range(L):
                xp, xm = base.copy(), base.copy()
                xp[k] += h
                xm[k] -= h
                if which == "S":
                    fp, _, _, pp, _ = oracle.dtw_grad(xp, T, r)
                    fm, _, _, pm, _ = oracle.dtw_grad(xm, T, r)
                else:
                    fp, _, _, pp, _ = oracle.dtw_grad(S, xp, r)
                    fm, _, _, pm, _ = oracle.dtw_grad(S, xm, r)
                if pp != path or pm != path:
                    continue
                fd = (fp - fm) / (2 * h)
                assert abs(fd - grad[k]) <= 1e-8 * max(1.0, abs(grad[k])), (which, k)
                checked += 1
    assert checked > 200


# ----------------------------------------------------------------------------- EAPrunedDTW scan

@pytest.mark.parametrize("m,w,threads", [(16, 2, 1), (32, 5, 4), (24, 23, 3), (20, 0, 2)])
def test_eap_scan_is_the_brute_force_search(m, w, threads):
    """The scan with the EAPrunedDTW model under the shared best-so-far
    returns the brute-force answer (lexicographic minimum of (distance,
    offset)) and evaluates no more cells than the window admits."""
    g = np.random.default_rng(m * 100 + w)
    x = np.cumsum(g.standard_normal(900))
    q = np.cumsum(g.standard_normal(m))
    x[500:500 + m] = q * 2.0 + 7.0          # a planted copy (same z-normalised shape)
    K = x.size - m + 1
    k, d, cells = oracle.eap_scan(q, x, w, np.arange(K), nthreads=threads)
    kb, db = oracle.nn_search(q, x, w)
    assert (k, d) == (kb, db) or (k == kb and d == pytest.approx(db, rel=1e-12, abs=1e-12))
    assert k == 500 and d == pytest.approx(0.0, abs=1e-9)
    per = sum(min(m - 1, i + w) - max(0, i - w) + 1 for i in range(m))
    assert 0 < cells <= per * K


def test_eap_scan_prunes_against_its_bound():
    """With the planted copy first in scan order, every later candidate meets
    a bound of 0 and stops early: far fewer cells than the window admits."""
    g = np.random.default_rng(9)
    m, w = 32, 6
    q = np.cumsum(g.standard_normal(m))
    x = np.concatenate([q, np.cumsum(g.standard_normal(2000))])
    K = x.size - m + 1
    k, d, cells = oracle.eap_scan(q, x, w, np.arange(K), nthreads=1)
    per = sum(min(m - 1, i + w) - max(0, i - w) + 1 for i in range(m))
    assert k == 0 and d == pytest.approx(0.0, abs=1e-9)
    assert cells < 0.2 * per * K
