"""GPU parity of the band-in-registers kernels against the FP64 oracle,
called through the C ABI (windows up to 64)."""
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


# ----------------------------------------------------------------------------- exposed steps

@pytest.mark.parametrize("m", [1, 7, 64, 128, 1024])
def test_window_stats(m):
    x32 = gen.as_f32(gen.random_walk(5000 + 37, gen.rng(200, m)) * 3.0 + 1000.0)
    mu, sd = eap.window_stats(torch.from_numpy(x32), m)
    omu, osd = oracle.window_stats(gen.as_oracle(x32), m)
    np.testing.assert_allclose(_cpu(mu), omu, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(_cpu(sd), osd, rtol=1e-8, atol=1e-9)


def test_window_stats_flat_window_is_zero():
    x = np.concatenate([np.linspace(0, 5, 100), np.full(40, 2.5), np.linspace(5, 0, 100)])
    mu, sd = eap.window_stats(torch.from_numpy(gen.as_f32(x)), 32)
    assert float(_cpu(sd)[104]) == 0.0


def _step_plateaus():
    """A random walk, then a plateau at 1000 with noise of sd 1e-3 (variance
    1e-12 of the mean square: normalised), a constant plateau at 500 (flat),
    a plateau at 200 with noise of sd 1e-2 (normalised) and one at 200 with
    float32-rounding-level noise (a few ulps of 200: flat)."""
    g = np.random.default_rng(7)
    ulp = float(np.spacing(np.float32(200.0)))
    parts = [np.cumsum(g.standard_normal(700)), 1000.0 + 1e-3 * g.standard_normal(600),
             np.full(500, 500.0), 200.0 + 1e-2 * g.standard_normal(600),
             200.0 + ulp * g.integers(-1, 2, 600)]
    return gen.as_f32(np.concatenate(parts))


def test_flat_rule_on_step_plateaus():
    """Flat windows (variance at most 1e-14 of the window's mean square) are
    the oracle's: the same windows get sigma 0, the others the oracle's
    statistics; the search distances of every offset follow."""
    x32 = _step_plateaus()
    m, w = 64, 6
    mu, sd = eap.window_stats(torch.from_numpy(x32), m)
    omu, osd = oracle.window_stats(gen.as_oracle(x32), m)
    sd, mu = _cpu(sd), _cpu(mu)
    np.testing.assert_array_equal(sd == 0.0, osd == 0.0)
    assert (osd == 0.0).sum() > 500 and (osd > 0.0).sum() > 1500
    np.testing.assert_allclose(mu, omu, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(sd, osd, rtol=1e-6, atol=0)
    q32 = gen.as_f32(np.cumsum(np.random.default_rng(8).standard_normal(m)))
    d = _cpu(eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), w))
    offs = np.arange(x32.size - m + 1)
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, offs)
    assert_close_array(d, want, what="step plateaus")


@pytest.mark.parametrize("m", [1, 5, 256, 1000])
def test_znorm(m):
    x32 = gen.as_f32(gen.random_walk(m, gen.rng(201, m)) + 50.0)
    z = _cpu(eap.znorm(torch.from_numpy(x32)))
    np.testing.assert_allclose(z, oracle.znorm(gen.as_oracle(x32)), rtol=0, atol=2e-6)


# ----------------------------------------------------------------------------- single pair

@pytest.mark.parametrize("lS,lT,w", [(1, 1, 0), (6, 6, 6), (37, 37, 0), (37, 37, 5), (100, 90, 12),
                                     (90, 100, 12), (200, 200, 64), (64, 64, 200), (33, 40, 7)])
def test_dtw_single_pair(lS, lT, w):
    g = np.random.default_rng(lS * 1000 + lT * 10 + w)
    S = gen.as_f32(g.standard_normal(lS))
    T = gen.as_f32(g.standard_normal(lT))
    got = eap.dtw(torch.from_numpy(S), torch.from_numpy(T), w)
    want = oracle.dtw(gen.as_oracle(S), gen.as_oracle(T), w)
    assert close(got, want), (got, want)


def test_dtw_worked_example():
    S = [3, 1, 4, 4, 1, 1]
    T = [1, 3, 2, 1, 2, 2]
    assert eap.dtw(S, T, 6) == 9.0
    assert eap.dtw(S, T, 6, ub=9.0) == 9.0
    assert eap.dtw(S, T, 6, ub=6.0) == math.inf
    assert eap.dtw(S, T, 0) == 23.0
    assert eap.dtw(S, T, 1) == oracle.dtw(S, T, 1)


def test_dtw_edge_cases():
    e = torch.zeros(0)
    assert eap.dtw(e, e, 3) == 0.0
    assert eap.dtw([1.0], e, 3) == math.inf
    assert eap.dtw(np.ones(5), np.ones(9), 3) == math.inf   # no admissible path
    assert eap.dtw(np.ones(5), np.ones(8), 3) == 0.0
    assert eap.dtw([1.0, 2.0], [1.0, 2.0], 1, ub=-1.0) == math.inf
    with pytest.raises(eap.EapdtwError):
        eap.dtw([1.0], [1.0], -1)
    with pytest.raises(eap.EapdtwError):
        eap.dtw([1.0], [1.0], 0, ub=float("nan"))


def test_dtw_bound_is_strict_and_ties_are_kept():
    g = np.random.default_rng(9)
    S, T = gen.as_f32(g.standard_normal(50)), gen.as_f32(g.standard_normal(50))
    d = eap.dtw(S, T, 10)
    assert eap.dtw(S, T, 10, ub=d) == d                      # tie kept
    assert eap.dtw(S, T, 10, ub=float(np.nextafter(np.float32(d), np.float32(0)))) == math.inf
    assert eap.dtw(S, T, 10, ub=math.inf) == d


# ----------------------------------------------------------------------------- pairs

@pytest.mark.parametrize("w", [0, 1, 3, 13, 26, 52, 64])
@pytest.mark.parametrize("P,L", [(1, 9), (130, 37), (64, 128)])
def test_dtw_pairs_plain(w, P, L):
    X, Y = gen.random_pairs(P, L, seed=w * 7 + P)
    got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), w))
    want = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    assert_close_array(got, want, what=f"pairs w={w}")


@pytest.mark.parametrize("w", [2, 26])
def test_dtw_pairs_bounded_contract(w):
    P, L = 200, 60
    X, Y = gen.random_pairs(P, L, seed=300 + w)
    exact = oracle.dtw_pairs(gen.as_oracle(X), gen.as_oracle(Y), w, np.arange(P), np.arange(P))
    g = np.random.default_rng(w)
    ub = exact * g.uniform(0.5, 1.5, P)
    ub[:5] = exact[:5]           # ties (kept up to float32 rounding)
    ub[5:8] = -1.0
    got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), w,
                             ub=torch.from_numpy(ub.astype(np.float32))))
    assert_bounded(got, exact, ub.astype(np.float32).astype(np.float64), what="bounded pairs")


def test_pruned_equals_unpruned_bitwise():
    """A kept result is bit-identical to the unbounded float32 recurrence."""
    P, L, w = 256, 80, 13
    X, Y = gen.random_pairs(P, L, seed=401)
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    plain = _cpu(eap.dtw_pairs(Xt, Yt, w))
    ub_tie = torch.from_numpy(plain.copy())
    tied = _cpu(eap.dtw_pairs(Xt, Yt, w, ub=ub_tie))
    assert np.array_equal(tied.view(np.uint32), plain.view(np.uint32))
    loose = _cpu(eap.dtw_pairs(Xt, Yt, w, ub=torch.from_numpy(plain * 1.5)))
    assert np.array_equal(loose.view(np.uint32), plain.view(np.uint32))
    ed = _cpu(eap.dtw_pairs(Xt, Yt, w, ub="ed"))
    assert np.array_equal(ed.view(np.uint32), plain.view(np.uint32))


def test_ed_mode_window_zero_is_exact_ed():
    P, L = 70, 33
    X, Y = gen.random_pairs(P, L, seed=402)
    got = _cpu(eap.dtw_pairs(torch.from_numpy(X), torch.from_numpy(Y), 0, ub="ed"))
    want = np.sum((gen.as_oracle(X) - gen.as_oracle(Y)) ** 2, axis=1)
    assert_close_array(got, want, what="window 0")


# ----------------------------------------------------------------------------- search

@pytest.mark.parametrize("w", [0, 5, 13, 40, 64])
def test_nn_dists_unbounded(w):
    q32, x32, _ = gen.c1(n=3000, m=96)
    d = _cpu(eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), w))
    ks = np.arange(x32.size - q32.size + 1)
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, ks)
    assert_close_array(d, want, what=f"nn_dists w={w}")


def test_nn_dists_bounded_contract():
    q32, x32, w = gen.c1(n=4000, m=128)
    ks = np.arange(x32.size - q32.size + 1)
    want = oracle.nn_dists(gen.as_oracle(q32), gen.as_oracle(x32), w, ks)
    ub = float(np.quantile(want, 0.05))
    d = _cpu(eap.nn_dists(torch.from_numpy(q32), torch.from_numpy(x32), w, ub=ub))
    assert_bounded(d, want, np.float64(np.float32(ub)), what="bounded nn_dists")


@pytest.mark.parametrize("seed_opt", [0, 1])
@pytest.mark.parametrize("interval", [1, 1000])
def test_nn_search_c1_full(seed_opt, interval):
    """C1 at full size: 19,873 candidates; the brute-force oracle is the definition."""
    q32, x32, w = gen.c1()
    old_interval = eap.get_option("check_interval")
    eap.set_option("seed", seed_opt)
    eap.set_option("check_interval", interval)
    try:
        (k, d), st = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), w, stats=True)
    finally:
        eap.set_option("seed", 1)
        eap.set_option("check_interval", old_interval)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(q, x, w)
    at = oracle.nn_dists(q, x, w, [k])[0]
    check_nn(k, d, ko, do, at)
    assert st["problems"] == x32.size - q32.size + 1
    assert st["cells_evaluated"] <= st["cells_computed"]
    assert st["cells_nominal"] == (x32.size - q32.size + 1) * sum(
        min(127, i + w) - max(0, i - w) + 1 for i in range(128))


@pytest.mark.parametrize("w", [0, 13, 26, 52])
def test_nn_search_c2_cut(w):
    """C2 generator, 20,000-point cut, every window of the config."""
    q32, x32, _ = gen.c2(n=20_000)
    k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), w)
    q, x = gen.as_oracle(q32), gen.as_oracle(x32)
    ko, do = oracle.nn_search(q, x, w)
    at = oracle.nn_dists(q, x, w, [k])[0]
    check_nn(k, d, ko, do, at)


def test_nn_search_planted_copy_and_ties():
    q32, x32, w = gen.c1(n=5000, m=64)
    xp = gen.plant(x32, q32, 3001, a=0.5, b=7.0)
    xp = gen.plant(xp, q32, 1200, a=2.0, b=-3.0)
    k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(xp), w)
    assert k == 1200 and d <= 1e-6


def test_nn_search_ragged_and_small():
    g = np.random.default_rng(17)
    for n, m, w in ((10, 10, 3), (11, 10, 0), (200, 3, 1), (129, 65, 64), (64 * 3 + 5, 40, 9)):
        x32 = gen.as_f32(np.cumsum(g.standard_normal(n)))
        q32 = gen.as_f32(np.cumsum(g.standard_normal(m)))
        k, d = eap.nn_search(torch.from_numpy(q32), torch.from_numpy(x32), w)
        q, x = gen.as_oracle(q32), gen.as_oracle(x32)
        ko, do = oracle.nn_search(q, x, w)
        at = oracle.nn_dists(q, x, w, [k])[0]
        check_nn(k, d, ko, do, at)


def test_nn_search_rejects_bad_input():
    x = torch.ones(100)
    with pytest.raises(eap.EapdtwError):
        eap.nn_search(torch.ones(0), x, 3)
    with pytest.raises(eap.EapdtwError):
        eap.nn_search(torch.ones(200), x, 3)
    with pytest.raises(eap.EapdtwError):
        eap.nn_search(torch.ones(10), x, -2)
    bad = torch.arange(100, dtype=torch.float32)
    bad[50] = float("nan")
    with pytest.raises(eap.EapdtwError) as e:
        eap.nn_search(torch.arange(10, dtype=torch.float32), bad, 2)
    assert "ENONFINITE" in str(e.value)


def test_seeded_search_keeps_the_true_minimum():
    """The seeding workgroup normalises its candidates with the search's own
    64-offset block statistics, so its bound never falls below the search's
    own distance of the best candidate: with seeding on, every search returns
    a valid offset and the same answer, bit for bit, as without seeding (small
    windows, where the seeding window equals the search window)."""
    g = np.random.default_rng(2024)
    cases = []
    for _ in range(60):
        m = int(g.integers(8, 80))
        n = int(g.integers(m + 1, 3000))
        w = int(g.integers(0, 9))
        x32 = gen.as_f32(np.cumsum(g.standard_normal(n)) * float(g.uniform(0.1, 100)))
        q32 = gen.as_f32(np.cumsum(g.standard_normal(m)))
        cases.append((torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w))
    try:
        eap.set_option("seed", 0)
        plain = [eap.nn_search(q, x, w) for q, x, w in cases]
        eap.set_option("seed", 1)
        seeded = [eap.nn_search(q, x, w) for q, x, w in cases]
    finally:
        eap.set_option("seed", 1)
    for (q, x, w), p, s in zip(cases, plain, seeded):
        assert s[0] >= 0 and s == p, (q.numel(), x.numel(), w, p, s)
