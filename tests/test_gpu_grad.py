"""GPU parity of the differentiable batch (forward + backward through
torch.autograd).  Every pair is checked on the GPU's own path: the path the
backward follows (exported by dtw_path) must be a valid warping path in the
window whose float64 cost is the oracle's DTW (Section 2: several optimal paths
may exist, and float32 rounding may pick another one of equal cost), and the
GPU gradient must be that path's float64 gradient.  On integer data, where
float32 is exact, the path must be the oracle's own (its tie order)."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_close_array, check_gpu_paths, unpack

pytestmark = pytest.mark.gpu


def _run(S32, T32, w, gout=None, recompute=False):
    S = torch.from_numpy(S32).cuda().requires_grad_(True)
    T = torch.from_numpy(T32).cuda().requires_grad_(True)
    d = eap.DTWFunction.apply(S, T, w, recompute)
    g = torch.ones_like(d) if gout is None else torch.from_numpy(gout).cuda()
    d.backward(g)
    return d.detach().cpu().numpy(), S.grad.cpu().numpy(), T.grad.cpu().numpy()


def _check(S32, T32, w, gout=None):
    d, gS, gT = _run(S32, T32, w, gout)
    dp, rr, cr = eap.dtw_path(torch.from_numpy(S32), torch.from_numpy(T32), w)
    assert np.array_equal(dp.cpu().numpy(), d), "dtw_path and the forward differ"
    check_gpu_paths(S32, T32, w, d, rr.cpu().numpy(), cr.cpu().numpy(), gS, gT, gout)
    return d, gS, gT


@pytest.mark.parametrize("P,L,w", [(64, 64, 7), (130, 100, 10), (70, 37, 5), (64, 48, 0),
                                   (5, 17, 16), (3, 2, 1), (66, 90, 64), (40, 120, 119),
                                   (17, 300, 200), (9, 700, 300)])
def test_forward_backward_on_the_gpu_path(P, L, w):
    S32, T32, _ = gen.c5(P=P, L=L)
    gout = gen.as_f32(gen.rng(50, P).uniform(0.5, 2.0, P))
    _check(S32, T32, w, gout)


@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("P,L,w", [(70, 64, 7), (33, 100, 40), (12, 300, 200)])
def test_every_lane_count(P, L, w, lanes):
    """Distances, paths and gradients with 16, 32 and 64 lanes per pair."""
    old = eap.get_option("wf_lanes")
    eap.set_option("wf_lanes", lanes)
    try:
        S32, T32, _ = gen.c5(P=P, L=L)
        gout = gen.as_f32(gen.rng(52, P).uniform(0.5, 2.0, P))
        d, _, _ = _check(S32, T32, w, gout)
        with torch.no_grad():
            d0 = eap.DTWFunction.apply(torch.from_numpy(S32).cuda(), torch.from_numpy(T32).cuda(),
                                       w, False).cpu().numpy()
        assert np.array_equal(d0, d), "distance-only and recorded sweeps differ"
        want = np.array([oracle.dtw(S32[p].astype(float), T32[p].astype(float), w)
                         for p in range(P)])
        assert_close_array(d, want, what=f"{lanes} lanes")
    finally:
        eap.set_option("wf_lanes", old)


def test_integer_data_follows_the_oracle_tie_order():
    """Small integers: float32 arithmetic is exact, ties are exact, and the
    GPU's path must be the oracle's (diagonal, then (i-1,j), then (i,j-1))."""
    g = np.random.default_rng(31)
    for L, w in ((9, 3), (16, 15), (33, 4), (70, 70)):
        S32 = g.integers(0, 3, (64, L)).astype(np.float32)
        T32 = g.integers(0, 3, (64, L)).astype(np.float32)
        d, rr, cr = eap.dtw_path(torch.from_numpy(S32), torch.from_numpy(T32), w)
        lo, hi = unpack(rr.cpu().numpy())
        for p in range(64):
            od, _, _, opath, _ = oracle.dtw_grad(S32[p].astype(float), T32[p].astype(float), w)
            mine = sorted((i + 1, j + 1) for i in range(L) for j in range(lo[p, i], hi[p, i] + 1))
            assert mine == sorted(opath), (L, w, p)
            assert float(d[p]) == od


def test_recompute_equals_record():
    S32, T32, _ = gen.c5(P=100, L=80)
    a = _run(S32, T32, 9, recompute=False)
    b = _run(S32, T32, 9, recompute=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_single_cell():
    d, gS, gT = _run(gen.as_f32([[1.5]]), gen.as_f32([[-0.5]]), 0)
    assert d[0] == 4.0 and gS[0, 0] == 4.0 and gT[0, 0] == -4.0


def test_window_zero_closed_form():
    S32, T32 = gen.random_pairs(64, 50, seed=77)
    d, gS, gT = _run(S32, T32, 0)
    diff = gen.as_oracle(S32) - gen.as_oracle(T32)
    np.testing.assert_allclose(gS, 2 * diff, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(gT, -2 * diff, rtol=1e-6, atol=1e-6)


def test_identical_series_zero_gradient():
    S32, _ = gen.random_pairs(64, 40, seed=78)
    d, gS, gT = _run(S32, S32.copy(), 6)
    assert not d.any() and not gS.any() and not gT.any()


def test_non_finite_pair_gives_nan_and_leaves_the_others():
    S32, T32, _ = gen.c5(P=20, L=30)
    S32[3, 7] = np.nan
    T32[11, 0] = np.inf
    d, gS, gT = _run(S32, T32, 4)
    for p in (3, 11):
        assert np.isnan(d[p]) and np.isnan(gS[p]).all() and np.isnan(gT[p]).all()
    ok = [p for p in range(20) if p not in (3, 11)]
    want = oracle.dtw_pairs(gen.as_oracle(S32[ok]), gen.as_oracle(T32[ok]), 4, np.arange(18),
                            np.arange(18))
    assert_close_array(d[ok], want, what="finite pairs")
    assert np.isfinite(gS[ok]).all() and np.isfinite(gT[ok]).all()


def test_central_finite_differences():
    """FP64 central differences of the oracle DTW are exact for a fixed path;
    compare the GPU gradient to them on coordinates whose perturbation keeps
    the oracle's optimal path (where the oracle's path is the GPU's)."""
    S32, T32, _ = gen.c5(P=8, L=40)
    w = 4
    d, gS, gT = _run(S32, T32, w)
    _, rr, _ = eap.dtw_path(torch.from_numpy(S32), torch.from_numpy(T32), w)
    lo, hi = unpack(rr.cpu().numpy())
    h = 1e-4
    checked = 0
    for p in range(8):
        S, T = gen.as_oracle(S32[p]), gen.as_oracle(T32[p])
        _, _, _, path, _ = oracle.dtw_grad(S, T, w)
        mine = sorted((i + 1, j + 1) for i in range(40) for j in range(lo[p, i], hi[p, i] + 1))
        if mine != sorted(path):
            continue
        for which, base, grad in (("S", S, gS[p]), ("T", T, gT[p])):
            for k in range(0, 40, 3):
                xp, xm = base.copy(), base.copy()
                xp[k] += h
                xm[k] -= h
                if which == "S":
                    fp, _, _, pp, _ = oracle.dtw_grad(xp, T, w)
                    fm, _, _, pm, _ = oracle.dtw_grad(xm, T, w)
                else:
                    fp, _, _, pp, _ = oracle.dtw_grad(S, xp, w)
                    fm, _, _, pm, _ = oracle.dtw_grad(S, xm, w)
                if pp != path or pm != path:
                    continue
                fd = (fp - fm) / (2 * h)
                assert abs(grad[k] - fd) <= 1e-5 * max(1.0, abs(fd)), (p, which, k, grad[k], fd)
                checked += 1
    assert checked > 50


def test_ckpt_bytes():
    lib = eap._lib.load()
    # a status word per pair and the path ranges (one word per row and per
    # column); the code words stay in LDS at these sizes
    for P, L, w in ((4096, 256, 26), (10, 256, 100), (7, 200, 100)):
        b = lib.eapdtw_dtw_ckpt_bytes(P, L, w)
        assert P * (1 + 2 * L) * 4 <= b < P * (1 + 2 * L) * 4 + 3 * 256, (P, L, w, b)
    # 300 rows active at once: 512 lane-slots, whose codes (38 chunks of 16
    # steps) do not fit in LDS and stay in the record
    b = lib.eapdtw_dtw_ckpt_bytes(7, 300, 299)
    assert b == 256 + 2 * 8448 + 7 * 38 * 512 * 4, b
    assert lib.eapdtw_dtw_ckpt_bytes(10, 600, 599) == -1   # 600 rows active at once
    assert lib.eapdtw_dtw_ckpt_bytes(10, 9000, 3) == -1    # longer than 8191
    # both series of a pair in one wave's 64 KB of LDS: 2 len + 66 <= 16384
    assert lib.eapdtw_dtw_ckpt_bytes(10, 8159, 3) > 0
    assert lib.eapdtw_dtw_ckpt_bytes(10, 8160, 3) == -1


def test_kernel_class_follows_the_lanes_option():
    """4,096 pairs of length 256, window 26 (28 rows active at once): 32
    lane-slots per pair; by default two pairs per wave, each lane one row, the
    codes kept in LDS; option wf_lanes = 16 takes two rows per lane."""
    old = eap.get_option("wf_lanes")
    try:
        eap.set_option("wf_lanes", 0)
        assert eap.dtw_kernel_class(4096, 256, 26, True) == {"lanes": 32, "slots": 1,
                                                              "codes_in_lds": True}
        assert eap.dtw_kernel_class(4096, 256, 26, False)["lanes"] == 32
        eap.set_option("wf_lanes", 16)
        assert eap.dtw_kernel_class(4096, 256, 26, True) == {"lanes": 16, "slots": 2,
                                                              "codes_in_lds": True}
        # 8,192 pairs give two waves per SIMD with four pairs per wave
        eap.set_option("wf_lanes", 0)
        assert eap.dtw_kernel_class(8192, 256, 26, False) == {"lanes": 16, "slots": 2,
                                                              "codes_in_lds": False}
        assert not eap.dtw_kernel_class(7, 300, 299, True)["codes_in_lds"]
    finally:
        eap.set_option("wf_lanes", old)


@pytest.mark.parametrize("lanes", [0, 16])
def test_c5_full_size(lanes):
    """4,096 warped pairs of length 256, window 26: every pair's distance,
    path and gradient (the default class, and 16 lanes per pair)."""
    old = eap.get_option("wf_lanes")
    eap.set_option("wf_lanes", lanes)
    try:
        S32, T32, w = gen.c5()
        gout = gen.as_f32(gen.rng(51, S32.shape[0]).uniform(0.5, 2.0, S32.shape[0]))
        _check(S32, T32, w, gout)
    finally:
        eap.set_option("wf_lanes", old)


def test_fwd_bwd_replayed_from_a_captured_graph():
    """The recorded forward and the backward through the C ABI, captured once
    as a HIP graph (no memset nodes) and replayed several times with eager
    work and synchronisations between the replays: every replay gives the
    eager distances and gradients bit for bit."""
    import ctypes
    S32, T32, w = gen.c5(P=512, L=200)
    P, L = S32.shape
    S, T = torch.from_numpy(S32).cuda(), torch.from_numpy(T32).cuda()
    ctx = eap.context(0)
    lib, h, p = ctx._lib, ctx.handle, eap._ptr
    rec = torch.empty(int(lib.eapdtw_dtw_ckpt_bytes(P, L, w)), device="cuda", dtype=torch.uint8)
    out = torch.empty(P, device="cuda")
    gout = torch.from_numpy(gen.as_f32(gen.rng(53, P).uniform(0.5, 2.0, P))).cuda()
    gS, gT = torch.empty_like(S), torch.empty_like(T)

    def step():
        ctx.check(lib.eapdtw_dtw_fwd(h, p(S), p(T), P, L, w, p(out), ctypes.c_void_p(rec.data_ptr())))
        ctx.check(lib.eapdtw_dtw_bwd(h, p(S), p(T), P, L, w, ctypes.c_void_p(rec.data_ptr()),
                                     p(gout), p(gS), p(gT)))

    ctx.bind_stream()
    step()
    torch.cuda.synchronize()
    want = (out.clone(), gS.clone(), gT.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.bind_stream()
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(graph):
            ctx.bind_stream()
            step()
    finally:
        ctx.bind_stream()
    for k in range(4):
        out.fill_(-1.0)
        gS.zero_()
        gT.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want[0]) and torch.equal(gS, want[1]) and torch.equal(gT, want[2]), k
        # eager work between the replays
        d = eap.DTWFunction.apply(S, T, w)
        assert torch.equal(d, want[0])
        torch.cuda.synchronize()
