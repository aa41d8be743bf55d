"""GPU parity of the batched uneven search (one persistent launch, replayed
from a captured hipGraph) against the FP64 oracle and the single-query search."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import check_nn, close

pytestmark = pytest.mark.gpu


def _queries(nq, mlo, mhi, rlo, rhi, seed):
    g = gen.rng(1000, seed)
    qs = []
    for _ in range(nq):
        m = int(g.integers(mlo, mhi + 1))
        ratio = float(g.uniform(rlo, rhi))
        qs.append((gen.as_f32(gen.random_walk(m, g)), gen.window_from_ratio(ratio, m)))
    return qs


def test_batch_vs_oracle_small():
    x32 = gen.as_f32(gen.random_walk(3000, gen.rng(1001)))
    qs = _queries(12, 16, 220, 0.0, 0.4, 1)
    qs.append((gen.as_f32(np.arange(40, dtype=np.float64) ** 1.5), 0))
    res = eap.nn_search_batch([(torch.from_numpy(q), w) for q, w in qs], torch.from_numpy(x32))
    x = gen.as_oracle(x32)
    for (q32, w), (k, d) in zip(qs, res):
        q = gen.as_oracle(q32)
        ko, do = oracle.nn_search(q, x, w)
        at = oracle.nn_dists(q, x, w, [k])[0]
        check_nn(k, d, ko, do, at)


@pytest.mark.parametrize("graph", [1, 0])
def test_batch_equals_single_query_search(graph):
    """Same float32 recurrence cell by cell: the batched results equal the
    single-query results exactly."""
    x32 = gen.as_f32(gen.random_walk(40_000, gen.rng(1002)))
    qs = _queries(20, 64, 700, 0.05, 0.20, 2)
    xt = torch.from_numpy(x32).cuda()
    qt = [(torch.from_numpy(q).cuda(), w) for q, w in qs]
    eap.set_option("graph", graph)
    try:
        res = eap.nn_search_batch(qt, xt)
    finally:
        eap.set_option("graph", 1)
    for (q, w), (k, d) in zip(qt, res):
        ks, ds = eap.nn_search(q, xt, w)
        assert (k, d) == (ks, ds), (q.numel(), w, k, d, ks, ds)


def test_graph_replays_are_identical():
    """Replays of the captured graph, with eager work and synchronisations in
    between, give the eager result every time."""
    x32 = gen.as_f32(gen.random_walk(20_000, gen.rng(1003)))
    qs = _queries(9, 32, 400, 0.05, 0.20, 3)
    xt = torch.from_numpy(x32).cuda()
    qt = [(torch.from_numpy(q).cuda(), w) for q, w in qs]
    eap.set_option("graph", 0)
    try:
        eager = eap.nn_search_batch(qt, xt)
    finally:
        eap.set_option("graph", 1)
    for rep in range(4):
        got = eap.nn_search_batch(qt, xt)
        assert got == eager, rep
        # unrelated eager work between replays
        eap.nn_search(qt[0][0], xt, qt[0][1])
        torch.cuda.synchronize()


def test_batch_knobs_do_not_change_results():
    x32 = gen.as_f32(gen.random_walk(15_000, gen.rng(1004)))
    qs = _queries(7, 50, 300, 0.05, 0.2, 4)
    xt = torch.from_numpy(x32).cuda()
    qt = [(torch.from_numpy(q).cuda(), w) for q, w in qs]
    base = eap.nn_search_batch(qt, xt)
    for key, val in (("batch_chunk", 1), ("batch_grid", 64), ("check_interval", 7), ("seed", 0),
                     ("batch_seed_stride", 1), ("batch_branches", 1), ("batch_branches", 8)):
        old = eap.get_option(key)
        eap.set_option(key, val)
        try:
            assert eap.nn_search_batch(qt, xt) == base, key
        finally:
            eap.set_option(key, old)


@pytest.mark.parametrize("graph", [0, 1])
def test_band_launch_branches(graph):
    """Band-window queries spread over 1-8 concurrent streams, with and
    without tiled-window queries beside them, in a graph or eagerly: the same
    answers as one search per query."""
    g = gen.rng(1006)
    x32 = gen.as_f32(gen.random_walk(60_000, g))
    q = gen.as_f32(gen.random_walk(128, g))
    wide = gen.as_f32(gen.random_walk(300, g))
    xt = torch.from_numpy(x32).cuda()
    qt = torch.from_numpy(q).cuda()
    band_only = [(qt, w) for w in (0, 13, 26, 52, 5)]
    mixed = band_only + [(torch.from_numpy(wide).cuda(), 120)]
    want = {id(b): [eap.nn_search(t, xt, w) for t, w in b] for b in (band_only, mixed)}
    old_g, old_b = eap.get_option("graph"), eap.get_option("batch_branches")
    eap.set_option("graph", graph)
    try:
        for nb in (1, 2, 3, 4, 8):
            eap.set_option("batch_branches", nb)
            for b in (band_only, mixed):
                for _ in range(2):
                    assert eap.nn_search_batch(b, xt) == want[id(b)], (nb, len(b))
    finally:
        eap.set_option("graph", old_g)
        eap.set_option("batch_branches", old_b)
    # on a caller's stream other than the default one (forked from and joined
    # back to it); the answers are read after that stream alone is synchronised
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for b in (band_only, mixed):
            assert eap.nn_search_batch(b, xt) == want[id(b)], len(b)
    side.synchronize()
    with pytest.raises(eap.EapdtwError):
        eap.set_option("batch_branches", 0)
    with pytest.raises(eap.EapdtwError):
        eap.set_option("batch_branches", 9)


def test_batch_stats_and_validation():
    x32 = gen.as_f32(gen.random_walk(5000, gen.rng(1005)))
    qs = _queries(5, 30, 200, 0.05, 0.2, 5)
    res, st = eap.nn_search_batch([(torch.from_numpy(q), w) for q, w in qs],
                                  torch.from_numpy(x32), stats=True)
    assert st["problems"] == sum(x32.size - q.size + 1 for q, _ in qs)
    assert 0 < st["cells_evaluated"] <= st["cells_computed"]
    with pytest.raises(eap.EapdtwError):
        eap.nn_search_batch([(torch.ones(10), -1)], torch.from_numpy(x32))
    with pytest.raises(eap.EapdtwError):
        eap.nn_search_batch([(torch.ones(10000), 3)], torch.from_numpy(x32))
    assert eap.nn_search_batch([], torch.from_numpy(x32)) == []
