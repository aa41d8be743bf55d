"""GPU parity of the batches of uneven pairs (Section 2, Eq. 1-5 with
lS != lT; Section 2.1 window per pair; Section 2.2 bound) and of the DBA
update, against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import (assert_bounded, assert_close_array, close, column_ranges,
                    range_path_cost_grad, ranges_are_path, unpack)

pytestmark = pytest.mark.gpu


def _std(x):
    return gen.standardise(x) if x.size > 1 else x


def _uneven(seed, n, lmax, extra=None):
    """n random-walk pairs, lengths up to lmax (ratio at most 2), windows from
    |lS - lT| up to past the lengths, or up to |lS - lT| + extra."""
    g = np.random.default_rng(seed)
    S, T, W = [], [], []
    for k in range(n):
        ls = int(g.integers(1, lmax + 1))
        lt = int(g.integers(max(1, ls // 2), min(lmax, 2 * ls) + 1))
        hi = max(ls, lt) + 2 if extra is None else abs(ls - lt) + extra
        r = int(g.integers(abs(ls - lt), hi))
        S.append(gen.as_f32(_std(np.cumsum(g.standard_normal(ls)))))
        T.append(gen.as_f32(_std(np.cumsum(g.standard_normal(lt)))))
        W.append(r)
    return S, T, W


def _oracle(S, T, W):
    return np.array([oracle.dtw(gen.as_oracle(s), gen.as_oracle(t), w) for s, t, w in zip(S, T, W)])


def test_uneven_batch_vs_oracle():
    """Every lane class (16 or 64 lanes per pair, 1 to 8 cells per lane)."""
    S, T, W = _uneven(1, 300, 90)
    S2, T2, W2 = _uneven(2, 12, 700, extra=200)
    S, T, W = S + S2, T + T2, W + W2
    d, st = eap.dtw_pairs_batch(S, T, W, stats=True)
    assert_close_array(d.cpu().numpy(), _oracle(S, T, W), what="uneven batch")
    assert st["problems"] == len(S) and st["abandoned"] == 0
    assert st["cells_evaluated"] == st["cells_nominal"] > 0


@pytest.fixture
def wf_lanes():
    """Sets option wf_lanes for one test and restores it."""
    old = eap.get_option("wf_lanes")
    yield lambda v: eap.set_option("wf_lanes", v)
    eap.set_option("wf_lanes", old)


@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_uneven_batch_every_lane_count(wf_lanes, lanes):
    """The same pairs swept with 16, 32 and 64 lanes per pair (each class
    that holds a pair: 1 to 8 cells per lane): distances against the oracle,
    the recorded paths valid and optimal, bounds honoured."""
    wf_lanes(lanes)
    S, T, W = _uneven(11, 160, 140)
    S2, T2, W2 = _uneven(12, 6, 500, extra=300)
    S, T, W = S + S2, T + T2, W + W2
    want = _oracle(S, T, W)
    d = eap.dtw_pairs_batch(S, T, W).cpu().numpy()
    assert_close_array(d, want, what=f"uneven batch, {lanes} lanes")
    g = np.random.default_rng(13)
    ub = gen.as_f32(want * g.choice([0.5, 0.999, 1.001, 2.0], size=want.size))
    db = eap.dtw_pairs_batch(S, T, W, ub=torch.from_numpy(ub)).cpu().numpy()
    assert_bounded(db, want, ub.astype(np.float64), what=f"bound, {lanes} lanes")
    S_pool, T_pool, pairs = eap.pack_pairs(S, T, W)
    rr, cr = eap.dtw_batch_path(S_pool, T_pool, pairs, len(S))
    lo, hi = unpack(rr.cpu().numpy())
    for k in range(len(S)):
        if math.isinf(want[k]):
            continue
        p = pairs[k]
        ls, lt = p.s_len, p.t_len
        sl = slice(p.s_off, p.s_off + ls)
        r = min(W[k], max(ls, lt) - 1)
        assert ranges_are_path(lo[sl], hi[sl], ls, lt, r), (lanes, k)
        clo, chi = column_ranges(lo[sl], hi[sl], lt)
        cost, _, _ = range_path_cost_grad(S[k], T[k], lo[sl], hi[sl], clo, chi, 1.0)
        assert close(cost, want[k]), (lanes, k, cost, want[k])


def test_uneven_edges():
    """No admissible path (|lS - lT| > r: +inf), empty series (Eq. 2-4), a
    single cell, window 0 (squared Euclidean distance) and windows past the
    lengths."""
    g = np.random.default_rng(3)
    a = gen.as_f32(g.standard_normal(10))
    b = gen.as_f32(g.standard_normal(14))
    e = gen.as_f32(np.zeros(0))
    S = [a, a, e, e, a, gen.as_f32([2.0]), a, a]
    T = [b, b, e, b, e, gen.as_f32([-1.0]), a[::-1].copy(), b]
    W = [3, 4, 0, 5, 5, 0, 0, 1000]
    d = eap.dtw_pairs_batch(S, T, W).cpu().numpy()
    assert math.isinf(d[0]) and close(d[1], oracle.dtw(a, b, 4))
    assert d[2] == 0.0 and math.isinf(d[3]) and math.isinf(d[4]) and d[5] == 9.0
    assert close(d[6], float(np.sum((gen.as_oracle(a) - gen.as_oracle(a[::-1])) ** 2)))
    assert close(d[7], oracle.dtw(a, b, None))


def test_uneven_bound_contract():
    S, T, W = _uneven(4, 200, 80)
    exact = _oracle(S, T, W)
    g = np.random.default_rng(5)
    ub = gen.as_f32(exact * g.choice([0.5, 0.999, 1.001, 2.0], size=exact.size))
    ub[::17] = exact[::17]  # the bound equal to the distance: kept
    d, st = eap.dtw_pairs_batch(S, T, W, ub=torch.from_numpy(ub), stats=True)
    assert_bounded(d.cpu().numpy(), exact, ub.astype(np.float64), what="uneven bound")
    assert st["abandoned"] > 0 and st["cells_evaluated"] < st["cells_nominal"]


def test_uneven_non_finite_pair():
    S, T, W = _uneven(6, 10, 40)
    S[4] = S[4].copy()
    S[4][0] = np.nan
    d = eap.dtw_pairs_batch(S, T, W).cpu().numpy()
    assert np.isnan(d[4])
    ok = [k for k in range(10) if k != 4]
    assert_close_array(d[ok], _oracle([S[k] for k in ok], [T[k] for k in ok],
                                      [W[k] for k in ok]), what="finite pairs")


def test_uneven_rejects_bad_pairs():
    a = gen.as_f32(np.ones(10))
    with pytest.raises(eap.EapdtwError):
        eap.dtw_pairs_batch([a], [gen.as_f32(np.ones(9000))], [3])      # too long
    with pytest.raises(eap.EapdtwError):
        eap.dtw_pairs_batch([gen.as_f32(np.ones(600))], [gen.as_f32(np.ones(600))], [599])
    with pytest.raises(eap.EapdtwError):
        eap.dtw_pairs_batch([a], [a], [-1])


def test_uneven_autograd_on_the_gpu_paths():
    """Gradients of the uneven differentiable batch: every pair's path (from
    dtw_batch_path) is a valid warping path in its window whose float64 cost
    is the oracle's DTW, and the gradient is that path's float64 gradient."""
    S, T, W = _uneven(7, 150, 120)
    S_pool, T_pool, pairs = eap.pack_pairs(S, T, W)
    Sp = S_pool.clone().requires_grad_(True)
    Tp = T_pool.clone().requires_grad_(True)
    d = eap.DTWBatchFunction.apply(Sp, Tp, pairs, len(S))
    gout = gen.as_f32(np.random.default_rng(8).uniform(0.5, 2.0, len(S)))
    d.backward(torch.from_numpy(gout).cuda())
    gS, gT = Sp.grad.cpu().numpy(), Tp.grad.cpu().numpy()
    rr, cr = eap.dtw_batch_path(S_pool, T_pool, pairs, len(S))
    lo, hi = unpack(rr.cpu().numpy())
    clo_g, chi_g = unpack(cr.cpu().numpy())
    want = _oracle(S, T, W)
    d = d.detach().cpu().numpy()
    for k in range(len(S)):
        p = pairs[k]
        ls, lt = p.s_len, p.t_len
        sl = slice(p.s_off, p.s_off + ls)
        tl = slice(p.t_off, p.t_off + lt)
        if math.isinf(want[k]):
            assert math.isinf(d[k]) and not gS[sl].any() and not gT[tl].any()
            continue
        r = min(W[k], max(ls, lt) - 1)
        assert ranges_are_path(lo[sl], hi[sl], ls, lt, r), k
        clo, chi = column_ranges(lo[sl], hi[sl], lt)
        assert np.array_equal(clo, clo_g[tl]) and np.array_equal(chi, chi_g[tl]), k
        cost, dS, dT = range_path_cost_grad(S[k], T[k], lo[sl], hi[sl], clo, chi, float(gout[k]))
        assert close(cost, want[k]) and close(float(d[k]), want[k]), (k, cost, d[k], want[k])
        tol = 1e-5 * max(1.0, float(np.max(np.abs(dS)) + np.max(np.abs(dT))))
        assert np.all(np.abs(gS[sl] - dS) <= tol + 1e-5 * np.abs(dS)), k
        assert np.all(np.abs(gT[tl] - dT) <= tol + 1e-5 * np.abs(dT)), k


def test_uneven_recorded_forward_rejects_overlapping_pairs():
    """The record holds the path ranges in the pools' layout, so a forward
    that records (a gradient is wanted) needs disjoint pairs; distances alone
    do not."""
    a = torch.ones(10, device="cuda", requires_grad=True)
    b = torch.ones(12, device="cuda")
    pairs = (eap.Pair * 2)()
    for k in range(2):
        pairs[k].s_off, pairs[k].s_len, pairs[k].t_off, pairs[k].t_len = 0, 10, 0, 12
        pairs[k].window = 5
    with pytest.raises(eap.EapdtwError):
        eap.DTWBatchFunction.apply(a, b, pairs, 2)
    with torch.no_grad():
        d = eap.DTWBatchFunction.apply(a.detach(), b, pairs, 2)
    assert d.tolist() == [0.0, 0.0]


def test_dba_worked_example():
    """The worked example's barycentre update (hand-derived path)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "worked_example.json")))
    B, cnt = eap.dba_step(torch.tensor(gold["S"]), torch.tensor([gold["T"]]), 10, counts=True)
    want = np.array(gold["dba_sums"], float) / np.array(gold["dba_counts"], float)
    assert np.allclose(B.cpu().numpy(), want, rtol=1e-7, atol=0)
    assert cnt.cpu().numpy().tolist() == gold["dba_counts"]


@pytest.mark.parametrize("n,lb,L,w", [(300, 64, 64, 7), (70, 50, 60, 12), (4096, 256, 256, 26)])
def test_dba_step_on_the_gpu_paths(n, lb, L, w):
    """The DBA update equals the float64 average over the GPU's own optimal
    paths; where the paths are the oracle's, it is the oracle's update."""
    g = np.random.default_rng(n + lb)
    X = gen.as_f32(np.stack([gen.standardise(np.cumsum(g.standard_normal(L))) for _ in range(n)]))
    B = gen.as_f32(gen.standardise(np.cumsum(g.standard_normal(lb))))
    out, cnt = eap.dba_step(torch.from_numpy(B), torch.from_numpy(X), w, counts=True)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    S_pool, T_pool, pairs = eap.pack_pairs([B] * n, list(X), w)
    rr, cr = eap.dtw_batch_path(S_pool, T_pool, pairs, n)
    lo, hi = unpack(rr.cpu().numpy().reshape(n, lb))
    s, c = np.zeros(lb), np.zeros(lb)
    X64 = X.astype(np.float64)
    cX = np.concatenate([np.zeros((n, 1)), np.cumsum(X64, axis=1)], axis=1)
    for p in range(n):
        assert ranges_are_path(lo[p], hi[p], lb, L, min(w, max(lb, L) - 1)), p
        s += cX[p, hi[p] + 1] - cX[p, lo[p]]
        c += hi[p] - lo[p] + 1
    assert np.array_equal(cnt, c)
    assert np.allclose(out, s / c, rtol=2e-6, atol=1e-6)
    if n <= 300:
        ob, oc = oracle.dba_step(gen.as_oracle(B), [gen.as_oracle(x) for x in X], w)
        same = np.array_equal(oc, c)
        if same:
            assert np.allclose(out, ob, rtol=2e-6, atol=1e-6)


def test_uneven_batch_at_the_size_limits():
    """The largest pairs a wavefront class holds: series of up to 8,191 points
    whose two lengths sum to at most 16,318 (both sit in one wave's 64 KB of
    LDS), and 512 lane-slots (at most 511 rows active at a step).  Distances and the
    differentiable batch's paths and gradients, against the oracle.  A float32
    DP over a path of up to lS + lT cells rounds at up to ~1e-5 relative per
    2,000 cells, so the distances use that tolerance scaled by the path
    length, and so does the float64 cost of the GPU's own path against the
    optimum."""
    g = np.random.default_rng(77)

    def walk(n):
        return gen.as_f32(_std(np.cumsum(g.standard_normal(n))))

    S = [walk(8191), walk(8191), walk(511), walk(8159), walk(300)]
    T = [walk(8127), walk(500), walk(8191), walk(8159), walk(299)]
    W = [510, 8190, 8190, 20, 299]
    for ls, lt, r in ((8191, 8128, 100), (8159, 8160, 20), (8191, 8127, 511)):
        with pytest.raises(eap.EapdtwError):    # past the LDS or the lane-slots
            eap.dtw_pairs_batch([walk(ls)], [walk(lt)], [r])
    want = _oracle(S, T, W)
    d = eap.dtw_pairs_batch(S, T, W).cpu().numpy()
    for k in range(len(S)):
        rel = 1e-5 * max(1.0, (S[k].size + T[k].size) / 2000.0)
        assert close(float(d[k]), want[k], rel=rel), (k, d[k], want[k])
    S_pool, T_pool, pairs = eap.pack_pairs(S, T, W)
    Sp = S_pool.clone().requires_grad_(True)
    Tp = T_pool.clone().requires_grad_(True)
    dd = eap.DTWBatchFunction.apply(Sp, Tp, pairs, len(S))
    dd.backward(torch.ones_like(dd))
    assert np.array_equal(dd.detach().cpu().numpy(), d), "recorded and distance-only sweeps differ"
    gS, gT = Sp.grad.cpu().numpy(), Tp.grad.cpu().numpy()
    rr, cr = eap.dtw_batch_path(S_pool, T_pool, pairs, len(S))
    lo, hi = unpack(rr.cpu().numpy())
    for k in range(len(S)):
        p = pairs[k]
        ls, lt = p.s_len, p.t_len
        sl = slice(p.s_off, p.s_off + ls)
        tl = slice(p.t_off, p.t_off + lt)
        r = min(W[k], max(ls, lt) - 1)
        assert ranges_are_path(lo[sl], hi[sl], ls, lt, r), k
        clo, chi = column_ranges(lo[sl], hi[sl], lt)
        cost, dS, dT = range_path_cost_grad(S[k], T[k], lo[sl], hi[sl], clo, chi, 1.0)
        rel = 1e-5 * max(1.0, (ls + lt) / 2000.0)
        assert close(cost, want[k], rel=rel), (k, cost, want[k])
        tol = 1e-5 * max(1.0, float(np.max(np.abs(dS)) + np.max(np.abs(dT))))
        assert np.all(np.abs(gS[sl] - dS) <= tol + 1e-5 * np.abs(dS)), k
        assert np.all(np.abs(gT[tl] - dT) <= tol + 1e-5 * np.abs(dT)), k
