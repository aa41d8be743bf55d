"""CPU pins of the oracle's path helpers and DBA update (Section 2's warping
path; the barycentre use of the path).  The worked example's path was derived
by hand from the printed matrix (tests/golden/worked_example.json)."""
import json
import os

import numpy as np
import pytest

import oracle
from test_oracle import _enumerated_choice

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
S_EX = np.array(GOLD["S"], dtype=np.float64)
T_EX = np.array(GOLD["T"], dtype=np.float64)
PATH_EX = [tuple(c) for c in GOLD["path_diag_top_left"]][::-1]  # from (1,1)


def test_path_grad_and_cost_on_the_worked_example():
    dS, dT = oracle.path_grad(S_EX, T_EX, PATH_EX)
    assert dS.tolist() == GOLD["grad_S"] and dT.tolist() == GOLD["grad_T"]
    assert oracle.path_cost(S_EX, T_EX, PATH_EX) == GOLD["dtw"]
    # gradient scale and a single-cell path
    dS2, dT2 = oracle.path_grad(S_EX, T_EX, PATH_EX, 0.5)
    assert np.array_equal(dS2, 0.5 * dS) and np.array_equal(dT2, 0.5 * dT)
    assert oracle.path_grad([3.0], [1.0], [(1, 1)])[0].tolist() == [4.0]


def test_is_warping_path():
    assert oracle.is_warping_path(PATH_EX, 6, 6, None)
    assert oracle.is_warping_path(PATH_EX, 6, 6, 2)       # every cell has |i-j| <= 2
    assert not oracle.is_warping_path(PATH_EX, 6, 6, 1)   # (4,2) and (5,3) leave window 1
    assert not oracle.is_warping_path(PATH_EX[1:], 6, 6, None)   # does not start at (1,1)
    assert not oracle.is_warping_path(PATH_EX[:-1], 6, 6, None)  # does not end at (6,6)
    skip = [(1, 1), (3, 1), (3, 2)]
    assert not oracle.is_warping_path(skip, 3, 2, None)
    back = [(1, 1), (2, 2), (2, 1), (2, 2)]
    assert not oracle.is_warping_path(back, 2, 2, None)


def test_dba_worked_example():
    B, cnt = oracle.dba_step(S_EX, [T_EX], None)
    want = np.array(GOLD["dba_sums"], dtype=np.float64) / np.array(GOLD["dba_counts"])
    assert np.allclose(B, want, rtol=0, atol=1e-15)
    assert cnt.tolist() == GOLD["dba_counts"]


def test_dba_tie_case():
    case = GOLD["tie_case"]
    B, cnt = oracle.dba_step(np.array(case["S"], float), [np.array(case["T"], float)], None)
    assert np.allclose(B, np.array(case["dba_sums"], float) / case["dba_counts"], rtol=0,
                       atol=1e-15)
    assert cnt.tolist() == case["dba_counts"]


def test_dba_window_zero_is_the_euclidean_mean():
    g = np.random.default_rng(7)
    X = g.standard_normal((9, 17))
    B = g.standard_normal(17)
    out, cnt = oracle.dba_step(B, X, 0)
    assert np.allclose(out, X.mean(axis=0), rtol=0, atol=1e-14)
    assert np.all(cnt == 9)


def test_dba_of_copies_is_a_fixed_point():
    g = np.random.default_rng(8)
    B = np.round(g.standard_normal(23), 3)
    out, cnt = oracle.dba_step(B, [B.copy() for _ in range(5)], 4)
    assert np.allclose(out, B, rtol=1e-15, atol=0) and np.all(cnt == 5)


def test_dba_against_enumerated_paths():
    """On small integer cases the update is the mean over the enumerated
    optimal path with the tie order (diagonal, then (i-1,j), then (i,j-1))."""
    g = np.random.default_rng(9)
    for _ in range(60):
        lb, n = int(g.integers(1, 5)), int(g.integers(1, 4))
        lens = [int(g.integers(max(1, lb - 2), lb + 3)) for _ in range(n)]
        r = max(abs(lb - L) for L in lens) + int(g.integers(0, 3))
        B = g.integers(0, 3, lb).astype(float)
        X = [g.integers(0, 3, L).astype(float) for L in lens]
        paths = [_enumerated_choice(B, x, r)[0] for x in X]
        want = oracle.dba_of_paths(lb, X, paths)
        got, _ = oracle.dba_step(B, X, r)
        assert np.array_equal(got, want), (B, X, r)


def test_range_helpers_on_the_worked_example():
    """The parity helpers that read GPU path ranges, pinned on the worked
    example's hand-derived path (0-based row ranges)."""
    from parity import column_ranges, range_path_cost_grad, ranges_are_path
    lo = np.array([0, 0, 1, 1, 2, 5])
    hi = np.array([0, 0, 1, 1, 4, 5])
    assert ranges_are_path(lo, hi, 6, 6, 5) and ranges_are_path(lo, hi, 6, 6, 2)
    assert not ranges_are_path(lo, hi, 6, 6, 1)
    clo, chi = column_ranges(lo, hi, 6)
    assert clo.tolist() == [0, 2, 4, 4, 4, 5] and chi.tolist() == [1, 3, 4, 4, 4, 5]
    cost, dS, dT = range_path_cost_grad(S_EX, T_EX, lo, hi, clo, chi)
    assert cost == GOLD["dtw"]
    assert dS.tolist() == GOLD["grad_S"] and dT.tolist() == GOLD["grad_T"]
    bad_lo = lo.copy()
    bad_lo[3] = 3  # skips columns: (3,1) -> (4,3) is not a warping step
    assert not ranges_are_path(bad_lo, np.maximum(hi, bad_lo), 6, 6, 5)
    assert not ranges_are_path(lo[::-1], hi[::-1], 6, 6, 5)
