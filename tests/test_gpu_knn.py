"""GPU parity of the k-nearest-neighbour search against the FP64 oracle's
plain definition (every distance, then a lexicographic sort)."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import close

pytestmark = pytest.mark.gpu


def _check(res, q32, x32, w, k):
    qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
    want = oracle.knn_search(qo, xo, w, k)
    K = x32.size - q32.size + 1
    assert len(res) == k
    got = [(o, d) for o, d in res if o >= 0]
    assert len(got) == min(k, K)
    assert all(o == -1 and math.isinf(d) for o, d in res[len(got):])
    offs = [o for o, _ in got]
    assert len(set(offs)) == len(offs)
    # ascending (distance, offset) order
    assert all((got[i][1], got[i][0]) < (got[i + 1][1], got[i + 1][0]) for i in range(len(got) - 1))
    at = oracle.nn_dists(qo, xo, w, offs)
    for i, ((o, d), (wo, wd)) in enumerate(zip(got, want)):
        assert close(d, at[i]), (i, o, d, at[i])  # the reported distance is the offset's
        assert close(d, wd), (i, d, wd)             # the i-th best, to the tolerance
        if o != wo:  # a near-tie swapped places
            assert abs(at[i] - wd) <= 1e-5 * wd + 1e-6, (i, o, wo, at[i], wd)


# (m, window, n, k): window 0, narrow and bordered windows, windows past 64
# (tiled kernel, banded and whole-query), k = 1 and 64, ragged row groups
CASES = [(64, 0, 3000, 5), (128, 13, 20_000, 10), (96, 30, 8000, 64), (37, 6, 5000, 1),
         (200, 52, 12_000, 16), (150, 64, 6000, 33), (150, 100, 6000, 12), (90, 89, 4000, 64),
         (300, 65, 5000, 7)]


@pytest.mark.parametrize("m,w,n,k", CASES)
def test_knn_vs_oracle(m, w, n, k):
    g = gen.rng(4400, m * 100 + w)
    q32, x32 = gen.as_f32(gen.random_walk(m, g)), gen.as_f32(gen.random_walk(n, g))
    res, st = eap.knn_search(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w, k,
                             stats=True)
    _check(res, q32, x32, w, k)
    assert st["problems"] == n - m + 1


def test_knn_one_is_nn_search():
    q32, x32, _ = gen.c2(n=80_000)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    for w in (0, 13, 26):
        (res,) = eap.knn_search(q, x, w, 1)
        assert res == eap.nn_search(q, x, w)


def test_knn_periodic_ties_and_planted():
    """Exactly repeated windows tie bit for bit: the smaller offsets come first.
    Planted copies come before everything else."""
    pattern = gen.random_walk(40, gen.rng(4401))
    x32 = gen.as_f32(np.tile(pattern, 50))
    q32 = gen.as_f32(np.asarray(x32[7:7 + 32], dtype=np.float64) + 0.01 * gen.rng(4402).standard_normal(32))
    res = eap.knn_search(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 4, 8)
    assert [o for o, _ in res] == [7 + 40 * j for j in range(8)]
    assert len({d for _, d in res}) == 1
    _check(res, q32, x32, 4, 8)
    g = gen.rng(4403)
    q = gen.random_walk(64, g)
    x = gen.random_walk(30_000, g)
    x32 = gen.plant(gen.plant(x, q, 12_000, a=3.0, b=1.0), q, 25_000, a=0.5, b=-2.0)
    q32 = gen.as_f32(q)
    res = eap.knn_search(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 6, 5)
    assert [o for o, _ in res[:2]] == [12_000, 25_000] and res[1][1] <= 1e-5
    _check(res, q32, x32, 6, 5)


def test_knn_fewer_offsets_than_k_and_errors():
    g = gen.rng(4404)
    q32, x32 = gen.as_f32(gen.random_walk(10, g)), gen.as_f32(gen.random_walk(14, g))
    res = eap.knn_search(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), 2, 8)
    _check(res, q32, x32, 2, 8)
    q32, x32 = gen.as_f32(gen.random_walk(300, g)), gen.as_f32(gen.random_walk(2000, g))
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    for bad_k in (0, 65):
        with pytest.raises(eap.EapdtwError):
            eap.knn_search(q, x, 10, bad_k)


def test_knn_many_ties_multi_tile_selection():
    """A long periodic series: 6,000 windows per phase tie bit for bit, so
    the words at or below the final bound span several 4,096-word sort tiles
    and the k best must be carried from tile to tile (smaller offsets first
    among the equal distances)."""
    pattern = gen.random_walk(20, gen.rng(4405))
    x32 = gen.as_f32(np.tile(pattern, 6000))
    q32 = gen.as_f32(np.asarray(x32[3:3 + 40], dtype=np.float64)
                     + 0.05 * gen.rng(4406).standard_normal(40))
    for w, k in ((0, 64), (4, 17), (6, 1)):
        res = eap.knn_search(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w, k)
        offs = [o for o, _ in res]
        ds = [d for _, d in res]
        # the best phase repeats every 20 points: offsets 3, 23, 43, ... all at one distance
        assert offs == [3 + 20 * j for j in range(k)], (w, offs[:5])
        assert len(set(ds)) == 1
        qo, xo = gen.as_oracle(q32), gen.as_oracle(x32)
        assert close(ds[0], oracle.nn_dists(qo, xo, w, [3])[0])


def _batch_queries(seed, n_queries, mlo, mhi, rlo, rhi):
    g = gen.rng(seed)
    out = []
    for _ in range(n_queries):
        m = int(g.integers(mlo, mhi + 1))
        w = int(np.ceil(float(g.uniform(rlo, rhi)) * m))
        out.append((gen.as_f32(gen.random_walk(m, g)), w))
    return out


@pytest.mark.parametrize("k", [1, 7, 64])
def test_knn_batch_equals_single_queries(k):
    """The batched search with a top-k bound per query: every query's k best
    (offset, distance) pairs are the single-query k-NN search's, bit for bit
    (band windows on concurrent streams, windows past 64 in the persistent
    tiled launch, window 0, a query with fewer offsets than k), and
    k = 1 is the batched nearest-neighbour search."""
    x32 = gen.as_f32(gen.random_walk(60_000, gen.rng(4500)))
    qs = _batch_queries(4501, 10, 40, 400, 0.0, 0.4)
    qs.append((gen.as_f32(gen.random_walk(90, gen.rng(4502))), 0))
    qs.append((gen.as_f32(gen.random_walk(300, gen.rng(4503))), 299))
    qs.append((x32[-60:].copy(), 5))
    xs = gen.as_f32(gen.random_walk(1000, gen.rng(4504)))
    x = torch.from_numpy(x32).cuda()
    tq = [(torch.from_numpy(q).cuda(), w) for q, w in qs]
    for graph in (1, 0):
        eap.set_option("graph", graph)
        try:
            got, st = eap.knn_search_batch(tq, x, k, stats=True)
            again = eap.knn_search_batch(tq, x, k)
        finally:
            eap.set_option("graph", 1)
        assert again == got
        for (q, w), res in zip(tq, got):
            assert res == eap.knn_search(q, x, w, k), (q.numel(), w, k)
        assert st["problems"] == sum(x.numel() - q.numel() + 1 for q, _ in tq)
    if k == 1:
        assert [r[0] for r in got] == eap.nn_search_batch(tq, x)
    # fewer offsets than k, and the oracle's definition on a short series
    small = [(torch.from_numpy(q).cuda(), min(w, 60)) for q, w in qs[:4]]
    small.append((torch.from_numpy(gen.as_f32(gen.random_walk(995, gen.rng(4506)))).cuda(), 3))
    got = eap.knn_search_batch(small, torch.from_numpy(xs).cuda(), k)
    for (q, w), res in zip(small, got):
        _check(res, q.cpu().numpy(), xs, w, k)


def test_knn_batch_rejects_bad_k():
    x = torch.from_numpy(gen.as_f32(gen.random_walk(500, gen.rng(4505)))).cuda()
    q = x[:50].clone()
    for k in (0, 65):
        with pytest.raises(eap.EapdtwError):
            eap.knn_search_batch([(q, 5)], x, k)


# k-NN behind the lower-bound cascade: the same cases (windows 0 and above 2048
# take the plain path, reported as every candidate reaching the DTW), plus
# noisy sinusoids where most candidates are skipped
@pytest.mark.parametrize("m,w,n,k", CASES)
def test_knn_lb_vs_oracle(m, w, n, k):
    g = gen.rng(4410, m * 100 + w)
    q32, x32 = gen.as_f32(gen.random_walk(m, g)), gen.as_f32(gen.random_walk(n, g))
    res, st = eap.knn_search_lb(torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w, k,
                                stats=True)
    _check(res, q32, x32, w, k)
    K = n - m + 1
    assert st["pruned_kim"] + st["pruned_keogh_eq"] + st["pruned_keogh_ec"] + \
        st["pruned_recheck"] + st["dtw_candidates"] == K
    if w == 0:
        assert st["dtw_candidates"] == K
    else:
        assert min(k, K) <= st["dtw_candidates"] <= K


@pytest.mark.parametrize("m,w,k", [(128, 13, 10), (128, 40, 16), (256, 100, 5), (200, 150, 20)])
def test_knn_lb_sinusoid_prunes(m, w, k):
    q32, x32, _ = gen.c2(n=20_000, m=m)
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    res, st = eap.knn_search_lb(q, x, w, k, stats=True)
    _check(res, q32, x32, w, k)
    assert st["dtw_candidates"] < x32.size - m + 1
    plain = eap.knn_search(q, x, w, k)
    assert [d for _, d in res] == pytest.approx([d for _, d in plain], rel=1e-5, abs=1e-6)


def test_knn_lb_bad_k():
    q = torch.zeros(16, device="cuda")
    x = torch.arange(100, dtype=torch.float32, device="cuda")
    for k in (0, 65):
        with pytest.raises(eap.EapdtwError):
            eap.knn_search_lb(q, x, 3, k)
