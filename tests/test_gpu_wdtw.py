"""GPU parity of the weighted-DTW search (an elastic distance with DTW's
recurrence, cost w(|i-j|) (a-b)^2) against the FP64 oracle: fixed-bound
distances of every candidate (threshold contract) and the search."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_bounded, assert_close_array, check_nn

pytestmark = pytest.mark.gpu


def _cpu(t):
    return t.detach().cpu().numpy()


# (m, window, g): window 0, narrow, bordered (>= 24) and the whole query,
# ragged row groups, weights from flat (g = 0) to steep; windows above 64 (the
# tiled kernel with the weights in LDS: banded tiles, and whole-query tiles)
CASES = [(64, 0, 0.1), (101, 13, 0.05), (128, 26, 0.25), (250, 52, 0.02), (37, 40, 1.0),
         (96, 30, 0.0), (300, 100, 0.05), (150, 149, 0.1), (200, 65, 0.0)]


@pytest.mark.parametrize("m,w,g", CASES)
def test_nn_dists_w_threshold_contract(m, w, g):
    gg = gen.rng(4600, m * 100 + w)
    x32 = gen.as_f32(gen.random_walk(2500, gg))
    x32[900:900 + 2 * m] = 1.0  # flat stretch: windows normalise to zeros
    q32 = gen.as_f32(gen.random_walk(m, gg))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    want = oracle.nn_dists_w(gen.as_oracle(q32), gen.as_oracle(x32), w, g, np.arange(x32.size - m + 1))
    assert_close_array(_cpu(eap.nn_dists_w(q, x, w, g)), want, what=f"wdtw m={m} w={w} g={g}")
    for quant in (0.01, 0.3):
        ub = float(np.quantile(want, quant))
        a = _cpu(eap.nn_dists_w(q, x, w, g, ub=ub))
        assert_bounded(a, want, np.float64(np.float32(ub)), what=f"wdtw bounded m={m} w={w}")


@pytest.mark.parametrize("m,w,g,n", [(128, 13, 0.1, 20_000), (256, 52, 0.05, 30_000),
                                     (77, 0, 0.3, 9_000), (200, 26, 0.15, 25_000),
                                     (200, 100, 0.05, 12_000), (120, 119, 0.2, 8_000)])
def test_nn_search_w_vs_oracle(m, w, g, n):
    gg = gen.rng(4601, m + w)
    q32, x32 = gen.as_f32(gen.random_walk(m, gg)), gen.as_f32(gen.random_walk(n, gg))
    k, d = eap.nn_search_w(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w, g)
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search_w(qo, xo, w, g)
    check_nn(k, d, ko, do, oracle.nn_dists_w(qo, xo, w, g, [k])[0])


def test_wdtw_flat_weights_half_dtw_and_planted():
    """g = 0 makes every weight 1/2: half the DTW distance; a planted copy is
    found at distance 0."""
    gg = gen.rng(4602)
    q32, x32 = gen.as_f32(gen.random_walk(80, gg)), gen.as_f32(gen.random_walk(4000, gg))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    a = _cpu(eap.nn_dists_w(q, x, 8, 0.0)).astype(np.float64)
    b = _cpu(eap.nn_dists(q, x, 8)).astype(np.float64)
    np.testing.assert_allclose(a, 0.5 * b, rtol=2e-6, atol=1e-6)
    x32 = gen.plant(x32, q32, 1717, a=2.0, b=-1.0)
    k, d = eap.nn_search_w(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 8, 0.2)
    assert k == 1717 and d <= 1e-5


def test_wdtw_errors():
    gg = gen.rng(4603)
    q = torch.from_numpy(gen.as_f32(gen.random_walk(300, gg))).cuda()
    x = torch.from_numpy(gen.as_f32(gen.random_walk(3000, gg))).cuda()
    with pytest.raises(eap.EapdtwError):
        eap.nn_search_w(q, x, 10, math.inf)
    q = torch.from_numpy(gen.as_f32(gen.random_walk(5000, gg))).cuda()
    x = torch.from_numpy(gen.as_f32(gen.random_walk(6000, gg))).cuda()
    with pytest.raises(eap.EapdtwError):  # window 4999 > 4095 after clamping to m - 1
        eap.nn_search_w(q, x, 5000, 0.1)


def test_wdtw_force_wide_keeps_band_windows():
    """Windows up to 64 take the band kernels even with option force_wide
    (the tiled kernel's weighted form serves the windows above them)."""
    gg = gen.rng(4604)
    q = torch.from_numpy(gen.as_f32(gen.random_walk(90, gg))).cuda()
    x = torch.from_numpy(gen.as_f32(gen.random_walk(3000, gg))).cuda()
    want = eap.nn_search_w(q, x, 20, 0.1)
    eap.set_option("force_wide", 1)
    try:
        assert eap.nn_search_w(q, x, 20, 0.1) == want
    finally:
        eap.set_option("force_wide", 0)
