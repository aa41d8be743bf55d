"""GPU parity of the leave-one-out nearest neighbour (NN1) over a set of
series: against the FP64 oracle on small sets, and at the all-pairs
workload's full size against the minima of the GPU's own all-pairs matrix
(same kernel arithmetic: the same bits) plus sampled oracle rows."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import close

pytestmark = pytest.mark.gpu


def _check(idx, dist, X32, w, rows=None):
    Xo = gen.as_oracle(X32)
    N = X32.shape[0]
    rows = range(N) if rows is None else rows
    if len(rows) == N:
        oj, od = oracle.nn1(Xo, w)
    for i in rows:
        others = np.array([j for j in range(N) if j != i])
        if len(rows) == N:
            ref_j, ref_d = int(oj[i]), float(od[i])
        else:
            ds = oracle.dtw_pairs(Xo, Xo, w, np.full(others.size, i), others)
            ref_j, ref_d = int(others[np.argmin(ds)]), float(ds.min())
        assert close(dist[i], ref_d), (i, dist[i], ref_d)
        if idx[i] != ref_j:  # a near-tie: the reported neighbour's distance is the minimum
            at = oracle.dtw_pairs(Xo, Xo, w, [i], [int(idx[i])])[0]
            assert abs(at - ref_d) <= 1e-5 * ref_d + 1e-6, (i, idx[i], ref_j, at, ref_d)


# (N, len, window): sets that span several 64-series blocks with a ragged
# last one, band and whole-series windows
@pytest.mark.parametrize("N,L,w", [(150, 48, 5), (130, 64, 63), (70, 100, 20), (200, 32, 0)])
def test_nn1_vs_oracle(N, L, w):
    X = np.stack([gen.standardise(gen.random_walk(L, gen.rng(4500, N * 10 + i))) for i in range(N)])
    X32 = gen.as_f32(X)
    X32[N // 2] = X32[3]  # a duplicate: each other's neighbour at distance 0
    idx, dist = eap.nn1(torch.from_numpy(X32).cuda(), w)
    assert idx[3] == N // 2 and idx[N // 2] == 3 and dist[3] == 0.0
    _check(idx, dist, X32, w)


def test_nn1_full_size_against_all_pairs():
    """2,000 standardised random walks of 512, whole-series window: NN1 equals
    the row/column minima of the all-pairs matrix bit for bit, and a sample of
    rows equals the oracle's; far fewer cells than all pairs."""
    X, w = gen.c3()
    Xt = torch.from_numpy(X).cuda()
    (idx, dist), st = eap.nn1(Xt, w, stats=True)
    D, sp = eap.pairwise(Xt, w, stats=True)
    D = D.cpu().numpy()
    N = X.shape[0]
    M = np.full((N, N), np.inf, dtype=np.float32)
    iu = np.triu_indices(N, 1)
    M[iu] = D
    M.T[iu] = D
    ref_j = np.argmin(M, axis=1)  # first index among equal minima
    assert np.array_equal(dist.astype(np.float32), M[np.arange(N), ref_j])
    assert np.array_equal(idx, ref_j)
    _check(idx, dist, X, w, rows=[0, 777, 1999])
    assert st["cells_evaluated"] < 0.5 * sp["cells_evaluated"]


@pytest.mark.parametrize("nq,nr,L,w", [(40, 150, 48, 5), (70, 65, 64, 63), (3, 200, 100, 20),
                                       (64, 64, 32, 0)])
def test_nn1_ref_vs_oracle(nq, nr, L, w):
    g = gen.rng(4501, nq + nr + w)
    Q = gen.as_f32(np.stack([gen.standardise(gen.random_walk(L, g)) for _ in range(nq)]))
    R = gen.as_f32(np.stack([gen.standardise(gen.random_walk(L, g)) for _ in range(nr)]))
    R[nr // 2] = Q[1]  # a copy of a test series: its neighbour at distance 0
    idx, dist = eap.nn1_ref(torch.from_numpy(Q).cuda(), torch.from_numpy(R).cuda(), w)
    assert idx[1] == nr // 2 and dist[1] == 0.0
    oj, od = oracle.nn1_ref(gen.as_oracle(Q), gen.as_oracle(R), w)
    for i in range(nq):
        assert close(dist[i], od[i]), (i, dist[i], od[i])
        if idx[i] != oj[i]:
            at = oracle.dtw_pairs(gen.as_oracle(Q), gen.as_oracle(R), w, [i], [int(idx[i])])[0]
            assert abs(at - od[i]) <= 1e-5 * od[i] + 1e-6, (i, idx[i], oj[i])


def test_nn1_ref_matches_leave_one_out_split():
    """The C3 set split into 1,500 reference and 500 test series: every test
    series' neighbour equals the minimum of the GPU's own all-pairs distances
    between the two parts (same kernel arithmetic: the same bits)."""
    X, w = gen.c3()
    Xt = torch.from_numpy(X).cuda()
    (idx, dist), st = eap.nn1_ref(Xt[1500:], Xt[:1500], w, stats=True)
    D = eap.pairwise(Xt, w).cpu().numpy()
    N = X.shape[0]
    for t in (0, 123, 499):
        i = 1500 + t
        ds = np.array([D[eap.pairwise_index(N, j, i)] for j in range(1500)])
        j = int(np.argmin(ds))
        assert idx[t] == j and np.float32(dist[t]) == ds[j], (t, idx[t], j, dist[t], ds[j])
    assert st["problems"] == 500 * 1500
