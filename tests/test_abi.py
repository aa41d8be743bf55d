"""The C-ABI library loads and exports every symbol include/eapdtw.h declares;
host-side behaviour that needs no GPU (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_2010_05371_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eapdtw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eapdtw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("eapdtw_dtw", "eapdtw_nn_search", "eapdtw_nn_search_batch", "eapdtw_dtw_pairs",
                 "eapdtw_pairwise", "eapdtw_dtw_fwd", "eapdtw_dtw_bwd", "eapdtw_create",
                 "eapdtw_destroy", "eapdtw_last_error", "eapdtw_nn_search_lb", "eapdtw_nn_dists_lb",
                 "eapdtw_nn_lower_bounds", "eapdtw_knn_search", "eapdtw_nn1", "eapdtw_nn_search_w",
                 "eapdtw_nn_dists_w"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and they are real exported C symbols
    raw = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_functions():
        assert ctypes.cast(getattr(raw, n), ctypes.c_void_p).value


def test_version():
    assert b"gfx950" in _lib.load().eapdtw_version()


def test_null_context_is_einval():
    lib = _lib.load()
    out = ctypes.c_double()
    assert lib.eapdtw_dtw(None, None, 0, None, 0, 0, 0.0, ctypes.byref(out), None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_set_option(None, b"seed", 1) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_nn_search(None, None, 1, None, 1, 0, None, None, None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_nn_search_lb(None, None, 1, None, 1, 0, None, None, None, None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_knn_search(None, None, 1, None, 1, 0, 1, None, None, None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_nn1(None, None, 2, 4, 0, None, None, None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_nn_search_w(None, None, 1, None, 1, 0, 0.1, None, None, None) == _lib.EAPDTW_EINVAL


def test_create_rejects_null_out():
    lib = _lib.load()
    assert lib.eapdtw_create(0, None, None) == _lib.EAPDTW_EINVAL
    assert lib.eapdtw_last_error(None)


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be visible: ENODEV is only checked without one")
def test_create_without_device_is_enodev():
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.eapdtw_create(0, None, ctypes.byref(h))
    assert rc == _lib.EAPDTW_ENODEV
    assert not h.value
    assert lib.eapdtw_last_error(None)


def test_ckpt_bytes_is_host_arithmetic():
    lib = _lib.load()
    assert lib.eapdtw_dtw_ckpt_bytes(-1, 10, 2) < 0


def test_record_sizes_follow_the_size_limits():
    """The wavefront batches' limits, decided on the host: at most 511 rows
    active at once (512 lane-slots), and a pair's two series in one wave's
    64 KB of LDS (s_len + t_len + 66 <= 16384 floats)."""
    lib = _lib.load()
    assert lib.eapdtw_dtw_ckpt_bytes(10, 8159, 3) > 0
    assert lib.eapdtw_dtw_ckpt_bytes(10, 8160, 3) == -1
    assert lib.eapdtw_dtw_ckpt_bytes(10, 600, 510) > 0
    assert lib.eapdtw_dtw_ckpt_bytes(10, 600, 511) == -1

    def rec(ls, lt, r):
        p = (_lib.Pair * 1)()
        p[0].s_off, p[0].s_len, p[0].t_off, p[0].t_len, p[0].window = 0, ls, 0, lt, r
        return lib.eapdtw_dtw_batch_record_bytes(p, 1)
    assert rec(8191, 8127, 510) > 0 and rec(8191, 500, 8190) > 0
    assert rec(8191, 8128, 100) < 0 and rec(8191, 8127, 511) < 0 and rec(8192, 10, 9000) < 0


def test_xcd_block_mapping_is_a_bijection():
    """The dispatch-index to logical-block map of the search kernels (runs of
    64 consecutive logical blocks dealt to the eight XCDs in turn) permutes
    [0, n) for any n, and dispatch b of a whole round lands on XCD b % 8."""
    def xcd_block(b, n, run=64):
        rnd = 8 * run
        if b >= n // rnd * rnd:
            return b
        x, j = b % 8, b // 8
        return (j // run) * rnd + x * run + j % run
    for n in list(range(1, 70)) + [511, 512, 513, 1953, 4097, 31250]:
        assert sorted(xcd_block(b, n) for b in range(n)) == list(range(n)), n
    n = 31250
    for b in range(0, n // 512 * 512, 97):
        assert (xcd_block(b, n) // 64) % 8 == b % 8


def test_tune_bucket():
    """Autotuning buckets: 32 x bit length of m + window class."""
    import paper_2010_05371_amd as eap
    assert eap.tune_bucket(256, 0) == 9 * 32
    assert eap.tune_bucket(256, 13) == 9 * 32 + 4
    assert eap.tune_bucket(256, 52) == 9 * 32 + 6
    assert eap.tune_bucket(256, 64) == 9 * 32 + 7
    assert eap.tune_bucket(256, 65) == 9 * 32 + 8 + 7
    assert eap.tune_bucket(256, 255) == eap.tune_bucket(256, 10_000) == 9 * 32 + 31
    assert eap.tune_bucket(512, 100) == 10 * 32 + 8 + 7
    assert eap.tune_bucket(0, 3) == -1 and eap.tune_bucket(5, -1) == -1
