"""GPU parity of the colour-ordered path against the oracle.

Reference: the oracle evaluated in long double (64-bit significand), whose
agreement with a 40-digit evaluation is pinned on the CPU.  Per event:
  * FP64 path: |got - ref| <= max(1e-12 |ref|, 12 (n - 2) u m) for every
    event (helpers.fp64_allowance: m is the event's magnitude, so the second
    term is the running error bound of any FP64 evaluation order; rigorous
    but loose), the median relative error below 1e-14 (or ten times the FP64
    oracle's own median where that is larger), and the p99 and max
    of the relative errors within 10x those of the FP64 oracle on the same
    events (helpers.fp64_comparable: two FP64 evaluations of the same
    conditioned function);
  * FP32 path (FP32 recursion, FP64 re-evaluation of the events its error
    bound lists): every event within FP32_MAX = 3e-4 and the median below
    1e-6 here; the p99 <= 1e-5 bar is asserted on 2^18-event samples in
    test_gpu_fp32_check.
Configurations that vanish identically at tree level (all helicities equal
but at most one) are checked against rounding level instead.
"""
import numpy as np
import pytest

from bg_inputs import make_events, workload
from oracle import cobg as ocobg
from oracle import me2 as ome2
from tests.helpers import (U64, colour_matrix_n8, fp64_allowance, fp64_comparable, mhv_helicities,
                           nonvanishing, reference_cobg)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_ME2_RTOL = 1e-12
FP32_MAX = 3e-4


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


def _check_sampled(got, mom, hel, precision, C=None):
    """Per-event bars against the long-double reference (module docstring)."""
    n = mom.shape[0]
    ref, mag, o64 = reference_cobg(mom, hel, with_oracle_fp64=True, C=C)
    nz = nonvanishing(hel)
    d = np.abs(got - ref)
    rel = (d / np.abs(ref))[nz]
    orel = (np.abs(o64 - ref) / np.abs(ref))[nz]
    _say(f"  per-event rel err median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} "
         f"max {rel.max():.2e}")
    if precision == "fp64":
        allow = fp64_allowance(n, ref, mag)
        worst = np.max((d / allow)[nz])
        _say(f"  max |d| / allowance {worst:.2f}; events needing the conditioning term: "
             f"{np.mean((d > 1e-12 * np.abs(ref))[nz]):.1%}")
        _say(f"  FP64 oracle's own error: p99 {np.percentile(orel, 99):.2e} max {orel.max():.2e}")
        assert worst <= 1.0
        # median: 1e-14, or ten times the FP64 oracle's own median where that
        # is larger (n = 8: 720 orderings, more roundings per event)
        assert np.median(rel) < max(1e-14, 10 * np.median(orel))
        assert fp64_comparable(rel, orel)
    else:
        assert rel.max() <= FP32_MAX
        assert np.median(rel) < 1e-6
    return ref


@pytest.mark.parametrize("n", [4, 5, 6, 7])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_me2_match_oracle(api, n, precision):
    E = 200 if n < 7 else 40
    mom, hel = _events(n, E, 3100 + n)
    _say(f"bg_me2 {precision} n={n} E={E}")
    got = api.me2(_dev(mom), _dev(hel), precision=precision).cpu().numpy()
    ref = _check_sampled(got, mom, hel, precision)
    nz = nonvanishing(hel)
    zero_tol = 1e-20 if precision == "fp64" else 1e-8
    assert np.max(np.abs(got[~nz]), initial=0.0) < zero_tol * np.median(np.abs(ref[nz]))


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


@pytest.mark.parametrize("n", [4, 5, 6])
def test_helicity_sum_split_equals_fused(api, n):
    """Helicity-summed FP64 requests of up to 16384 events run one block per
    (tile, configuration) and add the configurations afterwards; larger ones
    run the configurations in turn in the fused kernel.  Same operations in
    the same order: the first events agree bit for bit, ragged tail included."""
    E_big, E_small = 16500, 1001
    ev = make_events(n, E_big, seed=9600 + n, cuts=True)
    big = api.me2(_dev(ev["mom"]), None, precision="fp64").cpu().numpy()
    small = api.me2(_dev(np.ascontiguousarray(ev["mom"][:, :, :E_small])), None,
                    precision="fp64").cpu().numpy()
    _say(f"helicity-sum split n={n}: {E_small} events against the fused kernel's {E_big}")
    assert np.array_equal(small, big[:E_small])


@pytest.mark.parametrize("n", [4, 5, 6, 7])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_equals_two_stage(api, n, precision):
    """bg_me2 (recursion and colour sum in one kernel) against bg_currents
    followed by bg_color_contract (amplitudes through memory, matrix cores at
    n = 6, 7; at n = 7 in FP64 one straight path per ordering with 1/P^2 from
    prefix sums instead of the walk's subset table): colour sums in a
    different order.  In FP64 the two agree within twice the running error
    bound; in FP32 the compiler may fuse a product into a different
    multiply-add in the two kernels, so they agree to FP32 rounding amplified
    by the event's cancellations."""
    E = 1000 if n < 7 else 200
    mom, hel = _events(n, E, 3180 + n)
    dm, dh = _dev(mom), _dev(hel)
    _say(f"fused vs two-stage {precision} n={n} E={E}")
    # the two-stage path has no FP32 check: compare the plain FP32 recursions
    fprec = "fp32_unchecked" if precision == "fp32" else precision
    fused = api.me2(dm, dh, precision=fprec).cpu().numpy()
    two = api.color_contract(api.currents(dm, dh, precision), n).cpu().numpy()
    nz = nonvanishing(hel)
    rel = np.abs(fused - two)[nz] / np.abs(two[nz])
    _say(f"  max rel {rel.max():.2e} median {np.median(rel):.2e}")
    if precision == "fp64":
        # both sides are FP64 evaluations within the running error bound
        # 12 (n - 2) u m of the exact value (helpers.fp64_allowance), so they
        # differ by at most twice it; checked on the events above 1e-12
        assert np.median(rel) < 1e-14
        d = np.abs(fused - two)
        over = np.nonzero(nz & (d > 1e-12 * np.abs(two)))[0]
        if over.size:
            from oracle.conditioning import me2_cobg_magnitude
            _, mag = me2_cobg_magnitude(mom[:, :, over], hel[:, over])
            _say(f"  {over.size} events above 1e-12: max |d| / (2 x bound) "
                 f"{np.max(d[over] / (2 * 12 * (n - 2) * U64 * mag)):.2e}")
            assert np.all(d[over] <= 2 * 12 * (n - 2) * U64 * mag)
    else:
        assert np.median(rel) < 1e-6 and rel.max() < 1e-4


@pytest.mark.parametrize("n", [5, 6, 7])
def test_contraction_matches_oracle(api, n):
    """bg_color_contract on oracle amplitudes (VALU at n = 5, matrix cores at
    n = 6 and 7); 300 events: several event tiles and a ragged tail."""
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
        ref, mag = reference_cobg(mom, hel)
        nz = nonvanishing(hel)
        assert np.all((np.abs(got - ref) <= fp64_allowance(6, ref, mag))[nz])


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
    _check_sampled(g64[idx], m, h, "fp64")
    _check_sampled(g32[idx], m, h, "fp32")
    assert np.all(np.isfinite(g64)) and np.all(np.isfinite(g32))
    # FP32 against FP64 on every event of the launch
    nz = nonvanishing(hel)
    rel = np.abs(g32 - g64)[nz] / np.abs(g64[nz])
    _say(f"  fp32 vs fp64, all {nz.sum()} non-vanishing events: median {np.median(rel):.2e} "
         f"p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}")
    assert np.percentile(rel, 99) <= 1e-5 and rel.max() <= FP32_MAX


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_single_event(api, n):
    """One event per call: a single partial tile (and for n = 7 a single
    queue entry), helicity-summed and sampled."""
    mom, hel = _events(n, 1, 3300 + n)
    hel = mhv_helicities(n, 1, np.random.default_rng(33 + n))
    dm = _dev(mom)
    for h in (hel, None):
        ref = ome2.me2_cobg(mom, h)
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
            got = api.me2(dm, None if h is None else _dev(h), precision=prec).cpu().numpy()
            assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (prec, h is None, got[0], ref[0])


# ---------------------------------------------------------------------------
# full colour at n = 8 (K = 720, colour matrix held as its first row)

@pytest.fixture(scope="module")
def c8():
    return colour_matrix_n8()


def test_full_colour_n8_match_oracle(api, c8):
    """n = 8, one helicity per event, 40 events (two blocks of the recursion
    with a ragged tail; one full and one partial event block of the
    contraction): bg_currents against the oracle's 720 amplitudes, bg_me2
    (recursion, then the colour sum through the relabelled first row of C)
    against the long-double reference with the per-event bars of the module
    docstring, and bg_color_contract on the oracle's own amplitudes against
    the oracle's contraction with the full C(8)."""
    n, E = 8, 40
    mom, hel = _events(n, E, 3800)
    dm, dh = _dev(mom), _dev(hel)
    nz = nonvanishing(hel)
    _say(f"bg_currents fp64 n=8 E={E}")
    amp = api.currents(dm, dh, "fp64").cpu().numpy()
    A = ocobg.partial_amplitudes(mom, hel)
    scale = np.max(np.abs(A), axis=0)
    err = np.max(np.abs(amp[0] + 1j * amp[1] - A), axis=0) / scale
    _say(f"  amplitudes: max err / max |A| {np.max(err[nz]):.2e}")
    assert np.max(err[nz]) < 1e-11
    _say(f"bg_me2 cobg fp64 n=8 E={E}")
    got = api.me2(dm, dh, mode="cobg").cpu().numpy()
    ref = _check_sampled(got, mom, hel, "fp64", C=c8)
    assert np.max(np.abs(got[~nz]), initial=0.0) < 1e-20 * np.median(np.abs(ref[nz]))
    _say(f"bg_color_contract n=8 E={E} on oracle amplitudes")
    con = api.color_contract(_dev(np.stack([A.real, A.imag])), n).cpu().numpy()
    refc = ome2.contract(A, c8)
    rel = np.abs(con - refc)[nz] / np.abs(refc[nz])
    _say(f"  contraction rel err max {rel.max():.2e}")
    assert rel.max() < 1e-12
    out = _dev(np.full(E, 2.0))
    api.color_contract(_dev(np.stack([A.real, A.imag])), n, out=out, accumulate=True)
    assert np.array_equal(out.cpu().numpy(), 2.0 + con)


def test_full_colour_n8_chunks_sampled(api, c8):
    """2^17 + 2^16 + 37 events: two chunks of the n = 8 two-stage path (the
    second one ragged), 8 sampled non-vanishing events against the oracle
    with the per-event bars; the two-stage calls give the same values."""
    n, E = 8, (1 << 17) + (1 << 16) + 37
    mom, hel = _events(n, E, 3810)
    dm, dh = _dev(mom), _dev(hel)
    _say(f"bg_me2 cobg fp64 n=8 E={E}")
    got = api.me2(dm, dh, mode="cobg").cpu().numpy()
    assert np.all(np.isfinite(got))
    ok = np.nonzero(nonvanishing(hel))[0]
    idx = np.sort(np.concatenate([np.random.default_rng(12).choice(ok[ok < (1 << 17)], 4, replace=False),
                                  np.random.default_rng(13).choice(ok[ok >= (1 << 17)], 4, replace=False)]))
    _check_sampled(got[idx], np.ascontiguousarray(mom[:, :, idx]), np.ascontiguousarray(hel[:, idx]),
                   "fp64", C=c8)
    head = slice(E - 3000, E)
    m2, h2 = _dev(np.ascontiguousarray(mom[:, :, head])), _dev(np.ascontiguousarray(hel[:, head]))
    two = api.color_contract(api.currents(m2, h2), n).cpu().numpy()
    assert np.array_equal(two, got[head])


def test_full_colour_n8_helicity_sum(api):
    """hel = NULL at n = 8 sums the 256 configurations (accumulated through
    the contraction); equal to the sum of the per-configuration results
    within rounding of the different summation order; configurations are
    checked against the oracle above."""
    n, E = 8, 5
    mom, _ = _events(n, E, 3820)
    dm = _dev(mom)
    _say(f"bg_me2 cobg n=8 helicity sum E={E}")
    tot = api.me2(dm, None, mode="cobg").cpu().numpy()
    acc = np.zeros(E)
    for h in range(256):
        hel = np.array([[1 if (h >> (n - 1 - i)) & 1 == 0 else -1] * E for i in range(n)], dtype=np.int8)
        acc += api.me2(dm, _dev(hel), mode="cobg").cpu().numpy()
    assert np.max(np.abs(tot - acc) / acc) < 1e-12


def test_full_colour_n8_fp32_unsupported(api):
    """Colour-ordered n = 8 runs in FP64 only (the FP32 recursion has no
    accuracy check there): refused, not silently degraded."""
    mom, hel = _events(8, 4, 3830)
    with pytest.raises(RuntimeError):
        api.me2(_dev(mom), _dev(hel), mode="cobg", precision="fp32")


def test_helicity_sum_n7_two_stage(api):
    """hel = NULL at n = 7: FP64 runs the two-stage path once per helicity
    configuration (accumulated), equal to the sum of the 128 per-
    configuration results within rounding of the summation order; the
    checked FP32 helicity sum (fused, listed events again in two FP64 stages)
    within the FP32 bars of the module docstring."""
    n, E = 7, 6
    mom, _ = _events(n, E, 3840)
    dm = _dev(mom)
    _say(f"bg_me2 cobg n=7 helicity sum E={E}")
    tot = api.me2(dm, None).cpu().numpy()
    acc = np.zeros(E)
    for h in range(1 << n):
        hel = np.array([[1 if (h >> (n - 1 - i)) & 1 == 0 else -1] * E for i in range(n)], dtype=np.int8)
        acc += api.me2(dm, _dev(hel)).cpu().numpy()
    assert np.max(np.abs(tot - acc) / acc) < 1e-12
    t32 = api.me2(dm, None, precision="fp32").cpu().numpy()
    rel = np.abs(t32 - tot) / tot
    _say(f"  fp32 helicity sum rel err max {rel.max():.2e}")
    assert rel.max() <= FP32_MAX
    default = api.fp32_check(n)
    try:
        api.fp32_check(n, 0.0)
        all64 = api.me2(dm, None, precision="fp32").cpu().numpy()
    finally:
        api.fp32_check(n, default)
    assert np.array_equal(all64, tot)
