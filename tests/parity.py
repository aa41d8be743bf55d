"""Shared tolerance rules of the GPU parity tests.

The GPU recurrence runs in float32; the oracle in float64 on the same float32
inputs.  A float32 DTW over at most ~2,000 path cells stays within 1e-5
relative of the float64 value (its error is a few ulps per accumulated cell);
near zero an absolute floor of 1e-6 applies (exact-copy candidates).
"""
import math

import numpy as np

REL = 1e-5
ABS = 1e-6


def close(gpu: float, ref: float, rel: float = REL, abs_: float = ABS) -> bool:
    if math.isinf(ref) or math.isinf(gpu):
        return math.isinf(ref) and math.isinf(gpu)
    return abs(gpu - ref) <= max(abs_, rel * abs(ref))


def assert_close_array(gpu, ref, rel: float = REL, abs_: float = ABS, what: str = ""):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape
    inf_g, inf_r = np.isinf(gpu), np.isinf(ref)
    assert np.array_equal(inf_g, inf_r), f"{what}: infinity pattern differs at {np.nonzero(inf_g != inf_r)[0][:10]}"
    fin = ~inf_r
    err = np.abs(gpu[fin] - ref[fin])
    tol = np.maximum(abs_, rel * np.abs(ref[fin]))
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches; worst rel "
                           f"{float(np.max(err / np.maximum(np.abs(ref[fin]), 1e-300))):.3e}")


def assert_bounded(gpu, exact, ub, rel: float = REL, abs_: float = ABS, what: str = ""):
    """Threshold contract: exact value where exact <= ub, +inf where exact > ub;
    within the tolerance band around ub either outcome is accepted."""
    gpu = np.asarray(gpu, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    ub = np.broadcast_to(np.asarray(ub, dtype=np.float64), exact.shape)
    band = np.abs(exact - ub) <= np.maximum(abs_, rel * np.abs(ub))
    for k in range(exact.size):
        e, g, u = exact.flat[k], gpu.flat[k], ub.flat[k]
        if band.flat[k]:
            assert math.isinf(g) or close(g, e, rel, abs_), (what, k, g, e, u)
        elif e <= u:
            assert close(g, e, rel, abs_), (what, k, g, e, u)
        else:
            assert math.isinf(g), (what, k, g, e, u)


def check_nn(gpu_off: int, gpu_dist: float, oracle_off: int, oracle_dist: float,
             oracle_at_gpu: float, rel: float = REL, abs_: float = ABS):
    """Best offset bit-exact except on ties within tolerance; distance within tolerance."""
    assert close(gpu_dist, oracle_at_gpu, rel, abs_), (gpu_off, gpu_dist, oracle_at_gpu)
    if gpu_off != oracle_off:
        assert abs(oracle_at_gpu - oracle_dist) <= max(abs_, rel * abs(oracle_dist)), (
            f"offset {gpu_off} vs {oracle_off}: {oracle_at_gpu} vs {oracle_dist}")


# --------------------------------------------------------------------------
# Warping paths reported by the GPU as per-row / per-column ranges (packed
# lo | hi << 16, 0-based), checked on their own terms: a valid warping path
# in the window (Section 2, 2.1), its float64 cost against the oracle's DTW,
# and the gradient of that path's cost.

def unpack(rng):
    r = np.asarray(rng).astype(np.int64) & 0xFFFFFFFF
    return r & 0xFFFF, r >> 16


def ranges_are_path(lo, hi, ls: int, lt: int, r: int) -> bool:
    """Row ranges [lo[i], hi[i]] of one pair describe a warping path from
    (0,0) to (ls-1, lt-1) with |i - j| <= r on every cell."""
    lo, hi = np.asarray(lo[:ls]), np.asarray(hi[:ls])
    if lo[0] != 0 or hi[-1] != lt - 1 or np.any(lo > hi) or np.any(hi > lt - 1):
        return False
    # the next row starts where the previous one ended (vertical step) or one after
    if ls > 1 and not np.all((lo[1:] == hi[:-1]) | (lo[1:] == hi[:-1] + 1)):
        return False
    i = np.arange(ls)
    return bool(np.all(lo >= i - r) and np.all(hi <= i + r))


def column_ranges(lo, hi, lt: int):
    """Column ranges implied by the row ranges of a monotone path: column j
    holds the rows from the first whose range reaches j to the last whose
    range starts at or before j."""
    j = np.arange(lt)
    clo = np.searchsorted(np.asarray(hi), j, side="left")
    chi = np.searchsorted(np.asarray(lo), j, side="right") - 1
    return clo.astype(np.int64), chi.astype(np.int64)


def range_path_cost_grad(S, T, lo, hi, clo, chi, gout: float = 1.0):
    """float64 cost and gradient of the path with row ranges lo..hi and column
    ranges clo..chi: cost = sum (S(i)-T(j))^2, dS(i) = 2g sum_j (S(i)-T(j)),
    dT(j) = -2g sum_i (S(i)-T(j)) over the path cells."""
    S = np.asarray(S, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    cT = np.concatenate([[0.0], np.cumsum(T)])
    cT2 = np.concatenate([[0.0], np.cumsum(T * T)])
    cS = np.concatenate([[0.0], np.cumsum(S)])
    n = (hi - lo + 1).astype(np.float64)
    sT = cT[hi + 1] - cT[lo]
    sT2 = cT2[hi + 1] - cT2[lo]
    cost = float(np.sum(n * S * S - 2.0 * S * sT + sT2))
    dS = 2.0 * gout * (n * S - sT)
    m = (chi - clo + 1).astype(np.float64)
    dT = -2.0 * gout * ((cS[chi + 1] - cS[clo]) - m * T)
    return cost, dS, dT


def check_gpu_paths(S32, T32, w, d_gpu, rowrng, colrng, gS=None, gT=None, gout=None,
                    grad_rel: float = 1e-5, grad_abs: float = 1e-5):
    """For every pair: the GPU's ranges form a valid warping path in the window,
    its column ranges agree with its row ranges, the path's float64 cost is the
    oracle's DTW within the distance tolerance (so the path is optimal up to
    float32 rounding), the GPU distance matches, and the GPU gradient (if
    given) is the float64 gradient of that path."""
    import oracle

    S64, T64 = np.asarray(S32, np.float64), np.asarray(T32, np.float64)
    P, L = S64.shape
    r = min(int(w), L - 1)
    lo, hi = unpack(rowrng)
    clo_g, chi_g = unpack(colrng)
    want = oracle.dtw_pairs(S64, T64, w, np.arange(P), np.arange(P))
    for p in range(P):
        assert ranges_are_path(lo[p], hi[p], L, L, r), f"pair {p}: not a warping path"
        clo, chi = column_ranges(lo[p], hi[p], L)
        assert np.array_equal(clo, clo_g[p]) and np.array_equal(chi, chi_g[p]), (
            f"pair {p}: column ranges disagree with row ranges")
        g = 1.0 if gout is None else float(gout[p])
        cost, dS, dT = range_path_cost_grad(S64[p], T64[p], lo[p], hi[p], clo, chi, g)
        assert close(cost, want[p]), (p, cost, want[p])
        assert close(float(d_gpu[p]), want[p]), (p, float(d_gpu[p]), want[p])
        scale = float(np.max(np.abs(dS)) + np.max(np.abs(dT)))
        tol = grad_abs * max(1.0, scale)
        if gS is not None:
            assert np.all(np.abs(gS[p] - dS) <= tol + grad_rel * np.abs(dS)), (p, "dS")
        if gT is not None:
            assert np.all(np.abs(gT[p] - dT) <= tol + grad_rel * np.abs(dT)), (p, "dT")
