"""Error paths of the C ABI that need a context (forced from the host through
test hooks, so no kernel faults): ENOMEM when the scratch would exceed the
context's limit, and a reported device fault that poisons the context
(EPOISONED afterwards) while other contexts keep working."""
import ctypes

import pytest
import torch

import gen
import paper_2010_05371_amd as eap
from paper_2010_05371_amd import _lib

pytestmark = pytest.mark.gpu


def _search(ctx, q, x, w, bind=True):
    if bind:
        ctx.bind_stream()
    off, dist = ctypes.c_int64(), ctypes.c_double()
    rc = ctx._lib.eapdtw_nn_search(ctx.handle, eap._ptr(q), q.numel(), eap._ptr(x), x.numel(),
                                   int(w), ctypes.byref(off), ctypes.byref(dist), None)
    return rc, (off.value, dist.value)


@pytest.fixture(scope="module")
def c1():
    q32, x32, w = gen.c1()
    return torch.from_numpy(q32).cuda(), torch.from_numpy(x32).cuda(), w


def test_scratch_limit_gives_enomem(c1):
    q, x, w = c1
    want = eap.nn_search(q, x, w)
    ctx = eap.Context(0)
    ctx.set_option("scratch_limit", 4096)
    rc, _ = _search(ctx, q, x, w)
    assert rc == _lib.EAPDTW_ENOMEM
    assert b"scratch_limit" in ctx._lib.eapdtw_last_error(ctx.handle)
    ctx.set_option("scratch_limit", 0)
    rc, got = _search(ctx, q, x, w)
    assert rc == 0 and got == want


def test_injected_fault_poisons_only_its_context(c1):
    q, x, w = c1
    want = eap.nn_search(q, x, w)
    ctx = eap.Context(0)
    assert _search(ctx, q, x, w) == (0, want)
    ctx.set_option("inject_fault", 1)
    rc, _ = _search(ctx, q, x, w, bind=False)   # the next call reports the fault
    assert rc == _lib.EAPDTW_EDEVICE
    for _ in range(2):
        rc, _ = _search(ctx, q, x, w, bind=False)
        assert rc == _lib.EAPDTW_EPOISONED
    with pytest.raises(eap.EapdtwError) as e:
        ctx.check(ctx._lib.eapdtw_dtw_pairs_batch(ctx.handle, None, 0, None, 0, None, 0, None,
                                                  None, None))
    assert e.value.code == _lib.EAPDTW_EPOISONED
    other = eap.Context(0)
    assert _search(other, q, x, w) == (0, want)
    assert eap.nn_search(q, x, w) == want
