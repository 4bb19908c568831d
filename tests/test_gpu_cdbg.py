"""GPU parity of the colour-dressed path against the oracle.

For one colour-flow assignment and helicity configuration per event the GPU
returns |A|^2 of eq. color_decomposition_colorflow computed with the
dressed recursion; the oracle evaluates the same amplitude with its own
dressed recursion (itself pinned to the brute-force sum over orderings), in
long double for the reference.  Assignments whose edges j_k -> i_k do not
close into one circuit must give exactly 0.  Per event, on events whose
helicity configuration does not vanish identically:
  * FP64: |got - ref| <= max(1e-12 |ref|, 12 (n - 2) u m) with m = 2 |A| m_A
    and m_A the magnitude of the flow amplitude written as the sum of the
    colour-ordered amplitudes whose chain closes (oracle.conditioning; the
    same running error bound as the colour-ordered path), the median
    relative error below 1e-13, and p99 and max within 10x those of the
    FP64 oracle's own dressed recursion (helpers.fp64_comparable);
  * FP32 (checked, FP64 re-evaluation of listed events): every event within
    FP32_MAX = 3e-4 and the median below 1e-6; p99 <= 1e-5 is asserted on
    2^18-event samples in test_gpu_fp32_check.
"""
import numpy as np
import pytest

from bg_inputs import make_events, workload
from oracle import cdbg as ocdbg
from oracle.conditioning import flow_amplitude_magnitude
from oracle.numeric import extended
from tests.helpers import U64, fp64_comparable, mhv_helicities, nonvanishing, valid_colours

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_MAX = 3e-4


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_06507_amd import api as a
    return a


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(*a):
    print(*a, flush=True)


def _reference(mom, hel, col):
    """|A|^2 from the oracle's dressed recursion in long double (float64)."""
    return (np.abs(ocdbg.flow_amplitude(extended(mom), hel, col)) ** 2).astype(np.float64)


def _check(got, ref, mom, hel, col, precision, label):
    """Per-event bars of the module docstring; ref is the long-double |A|^2."""
    n = mom.shape[0]
    # exclude identically vanishing helicity configurations and flows whose
    # amplitude cancels exactly (e.g. all gluons of one colour: U(1) decoupling);
    # both sides return rounding noise there
    typical = np.median(np.abs(ref[nonvanishing(hel)])) if nonvanishing(hel).any() else 0.0
    nz = nonvanishing(hel) & (np.abs(ref) > 1e-8 * typical)
    assert np.all(np.abs(got[~nz]) < 1e-6 * typical + 1e-300)
    d = np.abs(got - ref)
    rel = d[nz] / np.abs(ref[nz])
    _say(f"  {label} {precision}: events {nz.sum()} rel err median {np.median(rel):.2e} "
         f"p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}")
    if precision == "fp64":
        o64 = np.abs(ocdbg.flow_amplitude(mom, hel, col)) ** 2
        orel = np.abs(o64 - ref)[nz] / np.abs(ref[nz])
        _say(f"  FP64 oracle's own error: p99 {np.percentile(orel, 99):.2e} max {orel.max():.2e}")
        assert np.median(rel) < 1e-13
        assert fp64_comparable(rel, orel)
        # the conditioning term only for the events above 1e-12 (it is costly)
        over = np.nonzero(nz & (d > 1e-12 * np.abs(ref)))[0]
        if over.size:
            _, mA = flow_amplitude_magnitude(mom[:, :, over], hel[:, over], col[:, :, over])
            allow = 12 * (n - 2) * U64 * 2.0 * np.sqrt(ref[over]) * mA
            _say(f"  {over.size} events above 1e-12: max |d| / allowance {np.max(d[over] / allow):.2e}")
            assert np.all(d[over] <= allow)
    else:
        assert np.median(rel) < 1e-6
        assert rel.max() <= FP32_MAX


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_valid_flows_match_oracle(api, n, precision):
    E = {4: 130, 5: 130, 6: 100, 7: 64, 8: 48, 9: 40}[n]
    ev = make_events(n, E, seed=5000 + n, cuts=True)
    col = valid_colours(n, E, np.random.default_rng(50 + n))
    _say(f"bg_me2 cdbg {precision} n={n} E={E}")
    got = api.me2(_dev(ev["mom"]), _dev(ev["hel"]), _dev(col), mode="cdbg",
                  precision=precision).cpu().numpy()
    ref = _reference(ev["mom"], ev["hel"], col)
    _check(got, ref, ev["mom"], ev["hel"], col, precision, f"n={n}")


def test_sampled_flows_zero_when_invalid(api):
    n = 6
    E = 600
    ev = make_events(n, E, seed=5100, cuts=True, sample_col=True)
    valid = ocdbg.is_valid_flow(ev["col"])
    _say(f"bg_me2 cdbg sampled colours n={n} E={E} valid={valid.sum()}")
    got = api.me2(_dev(ev["mom"]), _dev(ev["hel"]), _dev(ev["col"]), mode="cdbg").cpu().numpy()
    assert np.all(got[~valid] == 0.0)
    idx = np.nonzero(valid)[0]
    m, h, c = ev["mom"][:, :, idx], ev["hel"][:, idx], ev["col"][:, :, idx]
    _check(got[idx], _reference(m, h, c), m, h, c, "fp64", "sampled")


def test_auto_mode_and_determinism(api):
    n = 8
    ev = make_events(n, 2000, seed=5200, cuts=True, sample_col=True)
    m, h, c = _dev(ev["mom"]), _dev(ev["hel"]), _dev(ev["col"])
    a = api.me2(m, h, c, mode="auto", precision="fp32")
    b = api.me2(m, h, c, mode="cdbg", precision="fp32")
    assert torch.equal(a, b)


def test_full_size_gg_6g_sampled(api):
    """2^20 gg -> 6g events with sampled colours and helicities at the
    benchmark launch shape; valid events are checked against the oracle on a
    sample, invalid ones must be exactly zero."""
    ev = workload("gg_6g_n8_colour")
    mom, hel, col = ev["mom"], ev["hel"], ev["col"]
    E = mom.shape[2]
    _say(f"bg_me2 cdbg full size n=8 E={E}")
    dm, dh, dc = _dev(mom), _dev(hel), _dev(col)
    g64 = api.me2(dm, dh, dc, mode="cdbg", precision="fp64").cpu().numpy()
    g32 = api.me2(dm, dh, dc, mode="cdbg", precision="fp32").cpu().numpy()
    frac = (g64 != 0.0).mean()
    _say(f"  non-zero fraction {frac:.4f}")
    assert 0.03 < frac < 0.06
    # zero patterns of the two precisions agree, except flows whose amplitude
    # cancels to rounding (one side may return an exact 0, the other noise)
    typical = np.median(np.abs(g64[g64 != 0.0]))
    noise = (np.abs(g64) < 1e-8 * typical) & (np.abs(g32) < 1e-8 * typical)
    assert np.array_equal((g64 == 0.0) | noise, (g32 == 0.0) | noise)
    # on a sample, against the oracle's classification: no closed colour
    # circuit -> exactly 0 in both precisions; closed circuits non-zero
    rng = np.random.default_rng(9)
    smp = np.sort(rng.choice(E, 20000, replace=False))
    valid = ocdbg.is_valid_flow(col[:, :, smp])
    assert np.all(g64[smp][~valid] == 0.0) and np.all(g32[smp][~valid] == 0.0)
    assert (g64[smp][valid] != 0.0).mean() > 0.99
    nonzero = g64 != 0.0
    idx = np.sort(rng.choice(np.nonzero(nonzero)[0], 10, replace=False))
    m, h, c = mom[:, :, idx], hel[:, idx], col[:, :, idx]
    ref = _reference(m, h, c)
    _check(g64[idx], ref, m, h, c, "fp64", "full")
    _check(g32[idx], ref, m, h, c, "fp32", "full")


@pytest.mark.parametrize("n", [4, 6, 8, 9])
def test_single_event(api, n):
    """One event per call (a grid of one block) on a closed colour flow."""
    ev = make_events(n, 1, seed=5300 + n, cuts=True)
    col = valid_colours(n, 1, np.random.default_rng(53 + n))
    hel = mhv_helicities(n, 1, np.random.default_rng(54 + n))
    ref = _reference(ev["mom"], hel, col)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        got = api.me2(_dev(ev["mom"]), _dev(hel), _dev(col), mode="cdbg", precision=prec).cpu().numpy()
        assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (prec, got[0], ref[0])
