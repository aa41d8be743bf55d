"""GPU parity of the wide-window (tiled) kernels against the FP64 oracle:
windows wider than the register band, unconstrained DTW, all-pairs."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2010_05371_amd as eap
from parity import assert_bounded, assert_close_array, check_nn, close

pytestmark = pytest.mark.gpu


def _cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture
def force_wide():
    eap.set_option("force_wide", 1)
    yield
    eap.set_option("force_wide", 0)


@pytest.mark.parametrize("L,w", [(150, 65), (150, 100), (150, 149), (300, 200), (97, 500),
                                 (64, 64), (33, 32), (700, 90)])
def test_wide_pairs_plain(L, w):
    P = 70
    X, Y = gen.random_pairs(P, L, seed=L + w)
    got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), w))
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    assert_close_array(got, want, what=f"wide pairs L={L} w={w}")


@pytest.mark.parametrize("w", [0, 1, 2, 3, 6, 7, 8, 13, 26, 40])
def test_forced_wide_matches_oracle_for_narrow_windows(force_wide, w):
    P, L = 130, 45
    X, Y = gen.random_pairs(P, L, seed=500 + w)
    got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), w))
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    assert_close_array(got, want, what=f"forced wide w={w}")


@pytest.mark.parametrize("w", [5, 26, 90])
def test_band_and_wide_agree_bitwise(w):
    """Both kernels evaluate the same float32 recurrence cell by cell."""
    P, L = 64, 120
    X, Y = gen.random_pairs(P, L, seed=600 + w)
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    eap.set_option("force_wide", 1)
    try:
        wide = _cpu(eap.dtw_pairs(Xt, Yt, w))
    finally:
        eap.set_option("force_wide", 0)
    if w <= 64:
        band = _cpu(eap.dtw_pairs(Xt, Yt, w))
        assert np.array_equal(band.view(np.uint32), wide.view(np.uint32))
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    assert_close_array(wide, want)


@pytest.mark.parametrize("w", [80, 299])
def test_wide_pairs_bounded_and_bitwise(w):
    P, L = 128, 300
    X, Y = gen.random_pairs(P, L, seed=700 + w)
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    exact = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    plain = _cpu(eap.dtw_pairs(Xt, Yt, w))
    tied = _cpu(eap.dtw_pairs(Xt, Yt, w, ub=torch.from_numpy(plain.copy())))
    assert np.array_equal(tied.view(np.uint32), plain.view(np.uint32))
    ed = _cpu(eap.dtw_pairs(Xt, Yt, w, ub="ed"))
    assert np.array_equal(ed.view(np.uint32), plain.view(np.uint32))
    ub = (exact * np.random.default_rng(w).uniform(0.6, 1.4, P)).astype(np.float32)
    got = _cpu(eap.dtw_pairs(Xt, Yt, w, ub=torch.from_numpy(ub)))
    assert_bounded(got, exact, ub.astype(np.float64))


@pytest.mark.parametrize("lS,lT,w", [(300, 250, 80), (250, 300, 120), (400, 400, 399), (90, 150, 70)])
def test_wide_single_pair_unequal(lS, lT, w):
    g = np.random.default_rng(lS + 3 * lT + w)
    S = gen.as_f32(np.cumsum(g.standard_normal(lS)))
    T = gen.as_f32(np.cumsum(g.standard_normal(lT)))
    got = eap.dtw(S, T, w)
    want = oracle.dtw(gen.as_oracle(S), gen.as_oracle(T), w)
    assert close(got, want), (got, want)
    assert eap.dtw(S, T, w, ub=got) == got
    assert eap.dtw(S, T, w, ub=float(np.nextafter(np.float32(got), np.float32(0)))) == math.inf


@pytest.mark.parametrize("N,L,w", [(130, 64, 63), (70, 150, 149), (66, 120, 30), (65, 90, 70),
                                   (3, 17, 16), (2, 5, 4)])
def test_pairwise(N, L, w):
    X = gen.as_f32(np.stack([gen.standardise(gen.random_walk(L, gen.rng(800, N * 1000 + i)))
                             for i in range(N)]))
    got = _cpu(eap.pairwise(torch.from_numpy(X), w))
    ia, ib = np.triu_indices(N, 1)
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(X), w, ia, ib)
    assert got.size == N * (N - 1) // 2
    assert_close_array(got, want, what=f"pairwise N={N} L={L} w={w}")
    # DTW <= squared Euclidean distance (the bound of Section 2.3 never binds)
    ed = np.sum((gen.as_oracle(X)[ia] - gen.as_oracle(X)[ib]) ** 2, axis=1)
    assert np.all(got <= ed * (1 + 1e-6))
    k = eap.pairwise_index(N, 0, N - 1)
    assert close(float(got[k]), float(want[k]))


@pytest.mark.parametrize("m,w,n", [(300, 100, 2500), (200, 199, 1500), (257, 65, 3000)])
def test_wide_nn_search(m, w, n):
    g = gen.rng(900, m + w)
    x32 = gen.as_f32(gen.random_walk(n, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    (k, d), st = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), w, stats=True)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(q, x, w)
    at = oracle.nn_dists(q, x, w, [k])[0]
    check_nn(k, d, ko, do, at)
    assert st["cells_evaluated"] <= st["cells_computed"]


def test_wide_nn_dists(force_wide):
    q32, x32, _ = gen.c1(n=1500, m=100)
    ks = np.arange(x32.size - q32.size + 1)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    for w in (10, 70):
        want = oracle.nn_dists(q, x, w, ks)
        got = _cpu(eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), w))
        assert_close_array(got, want, what=f"wide nn_dists w={w}")
        ub = float(np.quantile(want, 0.1))
        got = _cpu(eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), w, ub=ub))
        assert_bounded(got, want, np.float64(np.float32(ub)))


def test_wide_nn_search_planted(force_wide):
    q32, x32, w = gen.c1(n=4000, m=128)
    xp = gen.plant(x32, q32, 2222, a=3.0, b=1.0)
    k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(xp), 40)
    assert k == 2222 and d <= 1e-6


@pytest.mark.parametrize("rows", [32, 64])
def test_whole_window_tile_heights(rows):
    """Whole-matrix windows under every tile height of the tiled kernel (option
    wide_rows): pairs with ragged last tiles, all pairs, NN1 and the search,
    against the oracle and bit for bit against the default height."""
    L, w = 150, 149                       # 150 = 2 x 64 + 22 = 4 x 32 + 22: ragged last tiles
    P = 70
    X, Y = gen.random_pairs(P, L, seed=4242)
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    N = 67
    Z = gen.as_f32(np.stack([gen.standardise(gen.random_walk(L, gen.rng(801, i))) for i in range(N)]))
    ia, ib = np.triu_indices(N, 1)
    want_pw = oracle.dtw_pairs(gen.as_oracle(Z), gen.as_oracle(Z), w, ia, ib)
    g = gen.rng(902, rows)
    x32 = gen.as_f32(gen.random_walk(1200, g))
    q32 = gen.as_f32(gen.random_walk(97, g))
    ko, do = oracle.nn_search(gen.as_oracle(q32), gen.as_oracle(x32), 96)
    base = None
    for opt in (0, rows):
        eap.set_option("wide_rows", opt)
        try:
            got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), w))
            pw = _cpu(eap.pairwise(torch.from_numpy(Z), w))
            idx, dist = eap.nn1(torch.from_numpy(Z), w)
            k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), 96)
        finally:
            eap.set_option("wide_rows", 0)
        assert_close_array(got, want, what=f"pairs rows={opt}")
        assert_close_array(pw, want_pw, what=f"pairwise rows={opt}")
        check_nn(k, d, ko, do, oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), 96, [k])[0])
        cur = (got, pw, np.asarray(idx), np.asarray(dist), k, d)
        if base is None:
            base = cur
        else:
            for a, b in zip(base[:4], cur[:4]):
                assert np.array_equal(a, b)
            assert base[4:] == cur[4:]


@pytest.mark.parametrize("m,w,n", [(2048, 300, 3000), (1500, 1499, 1500), (1024, 65, 1090)])
def test_wide_search_long_queries(m, w, n):
    """Long queries through the tiled kernel: many tiles per candidate, a
    single candidate (n = m), and a ragged last block of candidates."""
    g = gen.rng(903, m + w)
    x32 = gen.as_f32(gen.random_walk(n, g))
    q32 = gen.as_f32(gen.random_walk(m, g))
    k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), w)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(q, x, w)
    # a DP over ~2m cells in float32: the tolerance scales with the path length
    rel = 1e-5 * max(1.0, 2 * m / 2000.0)
    check_nn(k, d, ko, do, oracle.nn_dists(q, x, w, [k])[0], rel=rel)
