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
