"""The launch log (option "log", environment variable EAPDTW_LOG): one stderr
line per kernel choice naming the kernel and its launch shape, nothing when
off, and no change to any result."""
import ctypes
import os

import numpy as np
import pytest
import torch

import gen
import paper_2010_05371_amd as eap

pytestmark = pytest.mark.gpu


@pytest.fixture
def logging_on():
    eap.set_option("log", 1)
    try:
        yield
    finally:
        eap.set_option("log", 0)


def _lines(err: str):
    return [ln for ln in err.splitlines() if ln.startswith("[eapdtw] ")]


def test_search_logs_its_kernel(capfd, logging_on):
    q32, x32, w = gen.c1()
    q, x = torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda()
    got = eap.nn_search(q, x, w)
    torch.cuda.synchronize()
    lines = _lines(capfd.readouterr().err)
    assert any(f"search m={q.numel()} r={w}: nn_band_kernel<{w}," in ln for ln in lines), lines
    assert any(ln.startswith("[eapdtw] search seeding:") for ln in lines), lines
    eap.set_option("log", 0)
    assert eap.nn_search(q, x, w) == got
    torch.cuda.synchronize()
    assert _lines(capfd.readouterr().err) == []


def test_wide_pairs_and_wavefront_batches_log(capfd, logging_on):
    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.standard_normal((70, 150)).astype(np.float32)).cuda()
    eap.pairwise(X, 149)
    # forward with a record and backward through the C ABI on this thread's
    # context (the options belong to a context; autograd's backward runs on
    # another thread, with that thread's own context)
    P, L, w = 64, 96, 9
    S = torch.from_numpy(rng.standard_normal((P, L)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((P, L)).astype(np.float32)).cuda()
    c = eap.context(0)
    c.bind_stream()
    lib, h, p = c._lib, c.handle, eap._ptr
    rec = torch.empty(int(lib.eapdtw_dtw_ckpt_bytes(P, L, w)), device="cuda", dtype=torch.uint8)
    out, gout = torch.empty(P, device="cuda"), torch.ones(P, device="cuda")
    gS, gT = torch.empty_like(S), torch.empty_like(T)
    c.check(lib.eapdtw_dtw_fwd(h, p(S), p(T), P, L, w, p(out), ctypes.c_void_p(rec.data_ptr())))
    c.check(lib.eapdtw_dtw_bwd(h, p(S), p(T), P, L, w, ctypes.c_void_p(rec.data_ptr()), p(gout),
                               p(gS), p(gT)))
    torch.cuda.synchronize()
    lines = _lines(capfd.readouterr().err)
    assert any("pairwise rows 70 x 70 columns of length 150" in ln and "wide_kernel<64,pairwise>" in ln
               for ln in lines), lines
    assert any("wf_fwd_kernel<" in ln for ln in lines), lines
    assert any(ln.startswith("[eapdtw] wf_grad_kernel 64 pairs") for ln in lines), lines


def test_environment_variable_sets_the_option():
    old = os.environ.get("EAPDTW_LOG")
    try:
        os.environ["EAPDTW_LOG"] = "1"
        assert eap.Context(0).get_option("log") == 1
        os.environ["EAPDTW_LOG"] = "0"
        assert eap.Context(0).get_option("log") == 0
    finally:
        if old is None:
            os.environ.pop("EAPDTW_LOG", None)
        else:
            os.environ["EAPDTW_LOG"] = old
