"""GPU parity of the colour-ordered path against the FP64 oracle.

Error statistics.  For one sampled helicity configuration per event two
relative errors are used:
  * per-event:      |got - ref| / |ref|;
  * scale-relative: |got - ref| / S_e, S_e = helicity-averaged |M|^2 of the
    event (the scale of the sampled estimator 2^n |M|^2_h).
Configurations whose |M|^2 is suppressed by 1e-8..1e-11 against S_e amplify
input rounding (the problem's conditioning, ~1e3 at the 99th percentile for
n = 6), so the per-event error of any FP32 evaluation has a long tail.
Bars: FP64 path scale-relative max <= 1e-12 and per-event median <= 1e-13;
FP32 path scale-relative max <= 1e-5 and per-event median <= 1e-5.
Configurations that vanish identically at tree level (all helicities equal
but at most one) are checked against rounding level instead.
"""
import numpy as np
import pytest

from bg_inputs import make_events, workload
from oracle import cobg as ocobg
from oracle import me2 as ome2
from tests.helpers import nonvanishing, helicity_scale, mhv_helicities

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_ME2_RTOL = 1e-12
FP32_ME2_RTOL = 1e-5


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_06507_amd import api as a
    return a


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _events(n, E, seed):
    ev = make_events(n, E, seed=seed, cuts=True, sample_hel=True)
    return ev["mom"], ev["hel"]


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_amplitudes_fp64_match_oracle(api, n):
    E = 200 if n < 7 else 136  # several 64-lane tiles and a ragged tail
    mom, hel = _events(n, E, 3000 + n)
    _say(f"bg_currents fp64 n={n} E={E}")
    amp = api.currents(_dev(mom), _dev(hel), "fp64").cpu().numpy()
    got = amp[0] + 1j * amp[1]
    ref = ocobg.partial_amplitudes(mom, hel)
    nz = nonvanishing(hel)
    scale = np.max(np.abs(ref), axis=0)
    err = np.max(np.abs(got - ref), axis=0) / scale
    assert np.max(err[nz]) < 1e-11, np.max(err[nz])
    # vanishing helicity configurations: rounding level relative to the batch
    typical = np.median(scale[nz])
    assert np.max(np.abs(got[:, ~nz]), initial=0.0) < 1e-10 * typical


def _check_sampled(got, ref, scale, nz, precision):
    rel = (np.abs(got - ref) / np.abs(ref))[nz]
    srel = (np.abs(got - ref) / scale)[nz]
    _say(f"  per-event rel err median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} "
         f"max {rel.max():.2e}; scale-relative max {srel.max():.2e}")
    if precision == "fp64":
        assert srel.max() < FP64_ME2_RTOL
        assert np.median(rel) < 1e-13
    else:
        assert srel.max() < FP32_ME2_RTOL
        assert np.median(rel) < FP32_ME2_RTOL


@pytest.mark.parametrize("n", [4, 5, 6, 7])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_me2_match_oracle(api, n, precision):
    E = 200 if n < 7 else 40
    mom, hel = _events(n, E, 3100 + n)
    _say(f"bg_me2 {precision} n={n} E={E}")
    got = api.me2(_dev(mom), _dev(hel), precision=precision).cpu().numpy()
    ref = ome2.me2_cobg(mom, hel)
    nz = nonvanishing(hel)
    zero_tol = 1e-20 if precision == "fp64" else 1e-8
    assert np.max(np.abs(got[~nz]), initial=0.0) < zero_tol * np.median(np.abs(ref[nz]))
    _check_sampled(got, ref, helicity_scale(mom), nz, precision)


def test_helicity_sum_gg_gg(api):
    """gg -> gg, all 16 helicities summed, 1024 points without cuts."""
    ev = workload("gg_gg_n4_sumhel")
    mom = ev["mom"]
    _say("bg_me2 n=4 helicity sum E=1024")
    got = api.me2(_dev(mom), None).cpu().numpy()
    ref = ome2.me2_cobg(mom, None)
    assert np.max(np.abs(got - ref) / ref) < FP64_ME2_RTOL


@pytest.mark.parametrize("n", [5, 6])
def test_helicity_sum_fused(api, n):
    """Helicity-summed |M|^2 (all 2^n configurations inside the fused kernel)."""
    E = 40 if n == 5 else 12
    mom, _ = _events(n, E, 3150 + n)
    _say(f"bg_me2 helicity sum n={n} E={E}")
    got = api.me2(_dev(mom), None).cpu().numpy()
    ref = ome2.me2_cobg(mom, None)
    assert np.max(np.abs(got - ref) / ref) < FP64_ME2_RTOL


@pytest.mark.parametrize("n", [4, 5, 6, 7])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_equals_two_stage(api, n, precision):
    """bg_me2 (recursion and colour sum in one kernel) against bg_currents
    followed by bg_color_contract (amplitudes through memory, matrix cores at
    n = 6): the same recursion, colour sums in a different order.  In FP64
    the two agree to rounding of the sums; in FP32 the compiler may fuse a
    product into a different multiply-add in the two kernels, so they agree
    to FP32 rounding amplified by the event's cancellations."""
    E = 1000 if n < 7 else 200
    mom, hel = _events(n, E, 3180 + n)
    dm, dh = _dev(mom), _dev(hel)
    _say(f"fused vs two-stage {precision} n={n} E={E}")
    fused = api.me2(dm, dh, precision=precision).cpu().numpy()
    two = api.color_contract(api.currents(dm, dh, precision), n).cpu().numpy()
    nz = nonvanishing(hel)
    rel = np.abs(fused - two)[nz] / np.abs(two[nz])
    _say(f"  max rel {rel.max():.2e} median {np.median(rel):.2e}")
    if precision == "fp64":
        assert rel.max() < 1e-12
    else:
        assert np.median(rel) < 1e-6 and rel.max() < 1e-4


@pytest.mark.parametrize("n", [5, 6])
def test_contraction_matches_oracle(api, n):
    """bg_color_contract on oracle amplitudes (matrix cores at n = 6)."""
    E = 300
    mom, hel = _events(n, E, 3200 + n)
    hel = np.where(nonvanishing(hel)[None, :], hel, np.array([[-1], [-1]] + [[1]] * (n - 2)))
    hel = hel.astype(np.int8)
    A = ocobg.partial_amplitudes(mom, hel)
    amp = np.stack([A.real, A.imag])
    _say(f"bg_color_contract n={n} E={E}")
    got = api.color_contract(_dev(amp), n).cpu().numpy()
    ref = ome2.me2_cobg(mom, hel)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-13
    # accumulate mode adds onto the output
    out = _dev(np.ones(E))
    api.color_contract(_dev(amp), n, out=out, accumulate=True)
    assert np.max(np.abs(out.cpu().numpy() - 1.0 - ref) / np.abs(1.0 + ref)) < 1e-13


def test_empty_batch(api):
    mom = torch.zeros((6, 4, 0), dtype=torch.float64, device="cuda")
    hel = torch.zeros((6, 0), dtype=torch.int8, device="cuda")
    assert api.me2(mom, hel).numel() == 0
    assert api.currents(mom, hel).shape == (2, 24, 0)


def test_single_event_and_tail(api):
    for E in (1, 63, 65):
        mom, hel = _events(6, E, 3300 + E)
        got = api.me2(_dev(mom), _dev(hel)).cpu().numpy()
        ref = ome2.me2_cobg(mom, hel)
        nz = nonvanishing(hel)
        srel = (np.abs(got - ref) / helicity_scale(mom))[nz]
        assert np.max(srel, initial=0.0) < FP64_ME2_RTOL


def test_bitwise_deterministic(api):
    mom, hel = _events(6, 4096, 3400)
    a = api.me2(_dev(mom), _dev(hel), precision="fp32")
    b = api.me2(_dev(mom), _dev(hel), precision="fp32")
    assert torch.equal(a, b)


def test_full_size_gg_4g_sampled(api):
    """2^20 events of gg -> 4g at the benchmark launch shape; 256 sampled
    events are recomputed by the oracle."""
    ev = workload("gg_4g_n6")
    mom, hel = ev["mom"], ev["hel"]
    E = mom.shape[2]
    _say(f"bg_me2 full size n=6 E={E}")
    dm, dh = _dev(mom), _dev(hel)
    g64 = api.me2(dm, dh, precision="fp64").cpu().numpy()
    g32 = api.me2(dm, dh, precision="fp32").cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(E, 126, replace=False))
    idx = np.concatenate([idx, [0, E - 1]])
    m, h = mom[:, :, idx], hel[:, idx]
    ref = ome2.me2_cobg(m, h)
    nz = nonvanishing(h)
    scale = helicity_scale(m)
    _check_sampled(g64[idx], ref, scale, nz, "fp64")
    _check_sampled(g32[idx], ref, scale, nz, "fp32")
    assert np.all(np.isfinite(g64)) and np.all(np.isfinite(g32))


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_single_event(api, n):
    """One event per call: a single partial tile (and for n = 7 a single
    queue entry), helicity-summed and sampled."""
    mom, hel = _events(n, 1, 3300 + n)
    hel = mhv_helicities(n, 1, np.random.default_rng(33 + n))
    dm = _dev(mom)
    for h in (hel, None):
        ref = ome2.me2_cobg(mom, h)
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-4)):
            got = api.me2(dm, None if h is None else _dev(h), precision=prec).cpu().numpy()
            assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (prec, h is None, got[0], ref[0])
