"""bg_me2_noalloc (the allocation-free variant of bg_me2, for callers that
cannot allocate) called through the C ABI: its results equal bg_me2's bit
for bit on two calls in a row, the second with fewer events, for every mode
that uses a workspace (colour-ordered with the FP32 check, the persistent
n = 7 kernel, colour-dressed); device memory is unchanged across its calls;
sizes beyond its maximum and the colour-sampled mode are refused."""
import ctypes

import numpy as np
import pytest

from bg_inputs import make_events

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_06507_amd import api as a
    return a


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _noalloc(api, ctx, mom, hel, col, mode, precision, out):
    from paper_2106_06507_amd._lib import check, lib
    r = api._request(mom, hel, col, mode, precision, out)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().bg_me2_noalloc(ctx.handle, ctypes.byref(r), stream), "bg_me2_noalloc")
    return out


CASES = [("cobg", 6, "fp64", 5000, 1237), ("cobg", 6, "fp32", 20000, 3001),
         ("cobg", 7, "fp32", 3000, 517), ("cobg", 7, "fp64", 1000, 33),
         ("cdbg", 8, "fp32", 60000, 7001), ("cdbg", 9, "fp64", 20000, 999),
         ("lc", 5, "fp32", 4000, 100), ("auto", 8, "fp64", 9000, 64)]


@pytest.mark.parametrize("mode,n,precision,E1,E2", CASES)
def test_noalloc_equals_me2(api, mode, n, precision, E1, E2):
    ctx = api.default_context()
    for k, E in enumerate((E1, E2)):
        ev = make_events(n, E, seed=9300 + 10 * n + k, cuts=True, sample_hel=True,
                         sample_col=True)
        mom, hel = _dev(ev["mom"]), _dev(ev["hel"])
        col = _dev(ev["col"]) if mode in ("cdbg", "auto") else None
        ref = api.me2(mom, hel, col, mode=mode, precision=precision, ctx=ctx)
        out = torch.full((E,), -1.0, dtype=torch.float64, device="cuda")
        _noalloc(api, ctx, mom, hel, col, mode, precision, out)
        torch.cuda.synchronize()
        print(f"noalloc {mode} n={n} {precision} E={E}: equal {torch.equal(out, ref)}", flush=True)
        assert torch.equal(out, ref), (mode, n, precision, E)


def test_noalloc_allocates_nothing(api):
    ctx = api.default_context()
    ev = make_events(7, 4000, seed=9400, cuts=True, sample_hel=True)
    mom, hel = _dev(ev["mom"]), _dev(ev["hel"])
    out = torch.empty(4000, dtype=torch.float64, device="cuda")
    _noalloc(api, ctx, mom, hel, None, "cobg", "fp32", out)  # first launch of each kernel
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        _noalloc(api, ctx, mom, hel, None, "cobg", "fp32", out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_refuses(api):
    from paper_2106_06507_amd._lib import (BG_ERANGE, BG_EUNSUPPORTED, bg_request, lib)
    ctx = api.default_context()
    ev = make_events(6, 16, seed=9401, cuts=True, sample_hel=True, sample_col=True)
    mom, hel, col = _dev(ev["mom"]), _dev(ev["hel"]), _dev(ev["col"])
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = api._request(mom, hel, col, "comc", "fp64", out)
    assert lib().bg_me2_noalloc(ctx.handle, ctypes.byref(r), stream) == BG_EUNSUPPORTED
    # colour-ordered n = 8 runs through a chunk workspace that grows
    ev8 = make_events(8, 16, seed=9402, cuts=True, sample_hel=True)
    r8 = api._request(_dev(ev8["mom"]), _dev(ev8["hel"]), None, "cobg", "fp64", out)
    assert lib().bg_me2_noalloc(ctx.handle, ctypes.byref(r8), stream) == BG_EUNSUPPORTED
    # beyond the maximum: refused before anything is read or launched
    big = bg_request()
    big.n, big.mode, big.precision, big.flags = 6, 0, 0, 0
    big.n_events = (1 << 22) + 1
    big.mom, big.hel, big.me2 = mom.data_ptr(), hel.data_ptr(), out.data_ptr()
    assert lib().bg_me2_noalloc(ctx.handle, ctypes.byref(big), stream) == BG_ERANGE
