"""GPU parity of the lower-bound cascade: the per-candidate bounds against the
FP64 oracle, the cascade's fixed-bound distances against the oracle's
threshold contract and against the plain kernels' bits, and the cascade
search against the plain search and the oracle's brute force."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_bounded, assert_close_array, check_nn

pytestmark = pytest.mark.gpu

LB_ABS = 1e-5  # absolute floor for bounds near zero (sums of m float32 terms)


def _cpu(t):
    return t.detach().cpu().numpy()


def _series(m, n, seed, flat=False):
    g = gen.rng(4300, seed)
    x = gen.random_walk(n, g)
    if flat:
        x[n // 3:n // 3 + max(2 * m, 40)] = 2.5  # windows that normalise to all zeros
    return gen.as_f32(gen.random_walk(m, g)), gen.as_f32(x)


# (m, window, n): query lengths 1..7 (LB_Kim levels), ragged staging
# stretches (m > 512), windows 1..64, above 64 (the tiled kernel's cascade)
# and wider than the query
BOUND_CASES = [(1, 1, 300), (2, 1, 300), (5, 2, 400), (6, 3, 400), (7, 64, 500), (40, 4, 2000),
               (128, 13, 3000), (256, 52, 3000), (600, 64, 2500), (60, 100, 1500),
               (300, 100, 3000), (200, 199, 2500), (1000, 500, 3000)]


@pytest.mark.parametrize("m,w,n", BOUND_CASES)
def test_lower_bounds_vs_oracle(m, w, n):
    q32, x32 = _series(m, n, m * 1000 + w, flat=m >= 40)
    kim, eq, ec = (_cpu(t) for t in eap.nn_lower_bounds(torch.from_numpy(q32).cuda(),
                                                        torch.from_numpy(x32).cuda(), w))
    ko, eo, co = oracle.nn_lower_bounds(gen.as_oracle(q32), gen.as_oracle(x32), w,
                                        np.arange(n - m + 1))
    # the LB_Keogh sums add m non-negative float32 terms one after the other:
    # relative error at most (m - 1) 2^-24 from the additions plus a few
    # roundings per term (the recursive-summation bound)
    rel = max(1e-5, (m + 3) * 2.0 ** -24)
    assert_close_array(kim, ko, abs_=LB_ABS, what=f"kim m={m} w={w}")
    assert_close_array(eq, eo, rel=rel, abs_=LB_ABS, what=f"eq m={m} w={w}")
    assert_close_array(ec, co, rel=rel, abs_=LB_ABS, what=f"ec m={m} w={w}")


def test_lower_bounds_window_zero_is_squared_ed():
    """At window 0 both LB_Keogh bounds are the candidate's distance itself."""
    q32, x32 = _series(64, 1500, 7)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    _, eq, ec = (_cpu(t) for t in eap.nn_lower_bounds(q, x, 0))
    d = _cpu(eap.nn_dists(q, x, 0))
    assert_close_array(eq, d, abs_=LB_ABS, what="eq vs ed")
    assert_close_array(ec, d, abs_=LB_ABS, what="ec vs ed")


# (m, window, n): band windows on both sides of the bordered sweep's
# threshold (24), query lengths with a ragged last row group
DIST_CASES = [(64, 6, 3000), (101, 13, 3000), (128, 26, 3000), (250, 52, 3000), (130, 63, 2500),
              (37, 40, 1200), (300, 100, 3000), (150, 149, 2500)]


@pytest.mark.parametrize("ec", [0, 1])
@pytest.mark.parametrize("m,w,n", DIST_CASES)
def test_nn_dists_lb_threshold_contract(m, w, n, ec):
    """Fixed-bound distances with the cascade: the oracle's value where it is
    at most ub, +inf above; wherever the plain kernel keeps a value that the
    cascade keeps too, the bits are the same (the tightened bound never cuts a
    cell of the optimal path of a kept candidate)."""
    q32, x32 = _series(m, n, 50 + m + w, flat=True)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, np.arange(n - m + 1))
    for quant in (0.005, 0.05, 0.3, 1.0):
        ub = float(np.quantile(want, quant)) if quant < 1.0 else math.inf
        (a, st) = _with({"lb_ec": ec}, lambda: eap.nn_dists_lb(q, x, w, ub=ub, stats=True))
        a = _cpu(a)
        b = _cpu(eap.nn_dists(q, x, w, ub=ub))
        assert_bounded(a, want, np.float64(np.float32(ub)), what=f"lb m={m} w={w} q={quant}")
        both = np.isfinite(a) & np.isfinite(b)
        assert np.array_equal(a[both].view(np.uint32), b[both].view(np.uint32)), (m, w, quant)
        only = np.isfinite(a) ^ np.isfinite(b)
        assert np.all(np.abs(np.where(np.isfinite(a), a, b)[only] - ub) <= 1e-5 * abs(ub) + 1e-6)
        skipped = st["pruned_kim"] + st["pruned_keogh_eq"] + st["pruned_keogh_ec"]
        assert st["pruned_recheck"] == 0  # fixed bound: the re-check changes nothing
        assert skipped + st["dtw_candidates"] == n - m + 1
        if math.isinf(ub):
            assert skipped == 0 and np.isfinite(a).all()


# (m, window, n, seed)
SEARCH_CASES = [(128, 13, 20_000, 1), (128, 1, 8_000, 2), (96, 30, 12_000, 3), (256, 52, 30_000, 4),
                (77, 64, 9_000, 5), (200, 26, 25_000, 6), (200, 100, 20_000, 7),
                (150, 149, 15_000, 8)]


def _with(opts, fn):
    old = {k: eap.get_option(k) for k in opts}
    for k, v in opts.items():
        eap.set_option(k, v)
    try:
        return fn()
    finally:
        for k, v in old.items():
            eap.set_option(k, v)


# option sets: default (one pass, no candidate-envelope bound), all three
# bounds, a probe range of K/16 first, a probe of half the offsets
OPTS = [{}, {"lb_ec": 1}, {"lb_probe_div": 16}, {"lb_probe_div": 2, "lb_ec": 1}]


@pytest.mark.parametrize("opts", OPTS, ids=["default", "ec", "probe16", "probe2_ec"])
@pytest.mark.parametrize("m,w,n,seed", SEARCH_CASES)
def test_nn_search_lb_equals_search_and_oracle(m, w, n, seed, opts):
    q32, x32 = _series(m, n, 900 + seed)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    (k, d), st = _with(opts, lambda: eap.nn_search_lb(q, x, w, stats=True))
    kp, dp = eap.nn_search(q, x, w)
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(qo, xo, w)
    check_nn(k, d, ko, do, oracle.nn_dists(qo, xo, w, [k])[0])
    if (k, d) != (kp, dp):  # only a near-tie may differ
        assert abs(d - dp) <= 1e-5 * dp + 1e-6, ((k, d), (kp, dp))
    K = n - m + 1
    assert st["pruned_kim"] + st["pruned_keogh_eq"] + st["pruned_keogh_ec"] + \
        st["pruned_recheck"] + st["dtw_candidates"] == K
    assert 1 <= st["dtw_candidates"] < K
    assert st["problems"] == K and st["lb_ms"] > 0.0
    if not opts.get("lb_ec"):
        assert st["pruned_keogh_ec"] == 0


def test_nn_search_lb_planted_and_c2_windows():
    """C2-shaped series (noisy sinusoids) with a planted scaled copy: found at
    distance 0 at every window; the bounds skip candidates and the DP pass
    evaluates fewer cells than the plain search."""
    q32, x32, windows = gen.c2(n=100_000)
    x32 = gen.plant(x32, q32, 54_321, a=0.7, b=4.0)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    for w in windows:
        (k, d), st = eap.nn_search_lb(q, x, w, stats=True)
        assert k == 54_321 and d <= 1e-5, (w, k, d)
        if w > 0:
            _, sp = eap.nn_search(q, x, w, stats=True)
            assert st["pruned_keogh_eq"] > 0 and st["dtw_candidates"] < x32.size - q32.size + 1
            assert st["cells_evaluated"] < sp["cells_evaluated"], (w, st, sp)


@pytest.mark.parametrize("m,w,n", [(150, 0, 6000), (2100, 2099, 2500)])
def test_nn_search_lb_outside_its_windows_runs_plain_path(m, w, n):
    """Window 0 and windows above 2048 take the plain search: same answer,
    every candidate counted as reaching the DTW."""
    q32, x32 = _series(m, n, 77 + w)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    (k, d), st = eap.nn_search_lb(q, x, w, stats=True)
    assert (k, d) == eap.nn_search(q, x, w)
    assert st["dtw_candidates"] == x32.size - q32.size + 1 and st["pruned_keogh_eq"] == 0


def test_nn_search_lb_nonfinite_and_errors():
    q32, x32 = _series(64, 2000, 99)
    x32[700] = np.nan
    with pytest.raises(eap.EapdtwError):
        eap.nn_search_lb(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 6)
    with pytest.raises(eap.EapdtwError):
        eap.nn_lower_bounds(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 6)
    q32, x32 = _series(2100, 2500, 98)
    with pytest.raises(eap.EapdtwError):  # window 2099 > 2048 after clamping to m - 1
        eap.nn_lower_bounds(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 5000)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("w", [24, 40, 52, 64])
def test_nn_dists_lb_bordered_regression(w, seed):
    """Bordered list sweeps whose per-row bound rises from row to row: a chunk
    dropped from the borders must not re-enter with the values of an older row
    (they are below its cells' true values).  Tight bounds, both bound sets."""
    m, n = 250, 3000
    g = gen.rng(4320, seed * 100 + w)
    x32 = gen.as_f32(gen.random_walk(n, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, np.arange(n - m + 1))
    for quant in (0.02, 0.05, 0.1):
        ub = float(np.quantile(want, quant))
        for ec in (0, 1):
            a = _cpu(_with({"lb_ec": ec}, lambda: eap.nn_dists_lb(q, x, w, ub=ub)))
            assert_bounded(a, want, np.float64(np.float32(ub)),
                           what=f"lb regression w={w} seed={seed} q={quant} ec={ec}")
