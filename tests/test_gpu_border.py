"""GPU parity of the bordered band search (each row group swept only between
its pruning borders) against the whole-band sweep and the FP64 oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_bounded, check_nn

pytestmark = pytest.mark.gpu


def _cpu(t):
    return t.detach().cpu().numpy()


def _with_border(flag, fn):
    old = eap.get_option("border")
    eap.set_option("border", flag)
    try:
        return fn()
    finally:
        eap.set_option("border", old)


# (m, window): bands of 7 to 17 diagonal chunks (the bordered sweep serves
# windows from 24 on), query lengths that leave a ragged last row group,
# windows wider than the query
CASES = [(25, 24), (33, 30), (96, 24), (96, 40), (128, 52), (130, 63), (250, 26), (257, 64),
         (40, 100)]


@pytest.mark.parametrize("m,w", CASES)
def test_border_nn_dists_bitwise(m, w):
    """Every distance at most the bound has the same bits with and without
    the borders; every other candidate reads +inf in both."""
    g = gen.rng(3100, m * 1000 + w)
    x32 = gen.as_f32(gen.random_walk(2500, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    ks = np.arange(x32.size - m + 1)
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, ks)
    for ub in (float(np.quantile(want, 0.01)), float(np.quantile(want, 0.3)),
               float(want.max()), float("inf")):
        a = _cpu(_with_border(1, lambda: eap.nn_dists(q, x, w, ub=ub)))
        b = _cpu(_with_border(0, lambda: eap.nn_dists(q, x, w, ub=ub)))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (m, w, ub)
        assert_bounded(a, want, np.float64(np.float32(ub)), what=f"border m={m} w={w} ub={ub}")


@pytest.mark.parametrize("w", [24, 26, 52, 64])
def test_border_search_equals_whole_band(w):
    q32, x32, _ = gen.c2(n=60_000)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    (ka, da), sa = _with_border(1, lambda: eap.nn_search(q, x, w, stats=True))
    (kb, db), sb = _with_border(0, lambda: eap.nn_search(q, x, w, stats=True))
    assert (ka, da) == (kb, db)
    assert 0 < sa["cells_evaluated"] <= sa["cells_computed"]
    if w >= 26:
        assert sa["cells_computed"] < sb["cells_computed"]
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(qo, xo, w)
    check_nn(ka, da, ko, do, oracle.nn_dists(qo, xo, w, [ka])[0])


def test_border_planted_match_and_flat_windows():
    """A planted exact copy (distance 0, every cell on the diagonal live) and
    flat stretches of the series (windows normalised to all zeros)."""
    g = gen.rng(3101)
    q32 = gen.as_f32(gen.random_walk(200, g))
    x = gen.random_walk(20_000, g)
    x[5000:5600] = 3.0
    x32 = gen.plant(gen.as_f32(x), q32, 12_345, a=1.5, b=-2.0)
    k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), 48)
    assert k == 12_345 and d <= 1e-6
    ub = 50.0
    a = _cpu(_with_border(1, lambda: eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), 48, ub=ub)))
    b = _cpu(_with_border(0, lambda: eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), 48, ub=ub)))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
