"""GPU parity of the window-0 (squared Euclidean) search kernel against the
band kernel at window 0 (same bits) and the FP64 oracle."""
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


def _with_ed(flag, fn):
    old = eap.get_option("ed")
    eap.set_option("ed", flag)
    try:
        return fn()
    finally:
        eap.set_option("ed", old)


# query lengths: shorter than a check block, ragged blocks, more than one
# staged stretch of 512 rows
@pytest.mark.parametrize("m", [1, 5, 16, 37, 256, 700, 1100])
def test_ed_nn_dists_bitwise_and_oracle(m):
    g = gen.rng(3200, m)
    x32 = gen.as_f32(gen.random_walk(3000, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    ks = np.arange(x32.size - m + 1)
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), 0, ks)
    a = _cpu(_with_ed(1, lambda: eap.nn_dists(q, x, 0)))
    assert_close_array(a, want, what=f"ed m={m}")
    for ub in (float(np.quantile(want, 0.02)), float(np.quantile(want, 0.5)), float("inf")):
        a = _cpu(_with_ed(1, lambda: eap.nn_dists(q, x, 0, ub=ub)))
        b = _cpu(_with_ed(0, lambda: eap.nn_dists(q, x, 0, ub=ub)))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (m, ub)
        assert_bounded(a, want, np.float64(np.float32(ub)), what=f"ed bounded m={m}")


@pytest.mark.parametrize("w", [0, 13, 52])
def test_ed_seeding_and_search_equal(w):
    """Window-0 searches, and the window-0 seeding pass of wider searches,
    give the same answer with either kernel."""
    q32, x32, _ = gen.c2(n=40_000)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    ra = _with_ed(1, lambda: eap.nn_search(q, x, w))
    rb = _with_ed(0, lambda: eap.nn_search(q, x, w))
    assert ra == rb
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(qo, xo, w)
    check_nn(ra[0], ra[1], ko, do, oracle.nn_dists(qo, xo, w, [ra[0]])[0])
