"""GPU parity of the lane-refill band search against the wave-synchronous
band kernels (same cells, same bits: identical answers) and the FP64 oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import check_nn

pytestmark = pytest.mark.gpu


def _search(q, x, w, lanes):
    old = eap.get_option("lanes")
    eap.set_option("lanes", lanes)
    try:
        return eap.nn_search(q, x, w, stats=True)
    finally:
        eap.set_option("lanes", old)


# (m, window, series length): ranges of 512 candidates with a ragged last one,
# a series shorter than one range, windows wider than the query, m = 4
CASES = [(128, 13, 20_000), (256, 52, 40_000), (64, 1, 3_000), (100, 64, 9_000),
         (4, 2, 700), (40, 100, 1_000), (512, 26, 30_000), (96, 7, 515)]


@pytest.mark.parametrize("m,w,n", CASES)
def test_lanes_equal_wave_synchronous(m, w, n):
    g = gen.rng(4200, m * 1000 + w)
    x32 = gen.as_f32(gen.random_walk(n, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    (ka, da), sa = _search(q, x, w, 1)
    (kb, db), _ = _search(q, x, w, 0)
    assert (ka, da) == (kb, db)
    assert sa["problems"] == n - m + 1
    assert 0 < sa["cells_evaluated"] <= sa["cells_computed"]
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(qo, xo, w)
    check_nn(ka, da, ko, do, oracle.nn_dists(qo, xo, w, [ka])[0])


def test_lanes_c2_cut_and_planted():
    q32, x32, windows = gen.c2(n=100_000)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    for w in windows[1:]:
        assert _search(q, x, w, 1)[0] == _search(q, x, w, 0)[0]
    xp = gen.plant(x32, q32, 54_321, a=2.5, b=-1.0)
    (k, d), _ = _search(q, torch.from_numpy(xp).cuda(), 26, 1)
    assert k == 54_321 and d <= 1e-6
