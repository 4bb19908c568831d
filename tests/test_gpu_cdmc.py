"""GPU parity of continuous colour / real-polarization sampling.

The GPU returns A^2 for real polarizations e(phi) and colour vectors
(eta, etabar) per event (dressed recursion, all arithmetic real); the
oracle evaluates the same amplitude with its dressed recursion over
external colour matrices etabar eta^T (pinned on the CPU to the colour-flow
limit, exact phi and colour quadratures and the Ward identity).  A^2 is a
continuous function of the sampled variables that passes through zero and
spreads over many decades, so per-event relative errors are taken on events
above 1e-3 of the median, and every event's error is also held to a bar
relative to the largest A^2 of the sample.  Bars: FP64 1e-12 median / 1e-9
max relative, 1e-11 of the largest; FP32 1e-5 median / 1e-2 max relative,
1e-4 of the largest.
"""
import numpy as np
import pytest

from bg_inputs import make_events, continuous_states
from oracle import cdmc as ocdmc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BARS = {"fp64": (1e-12, 1e-9, 1e-11), "fp32": (1e-5, 1e-2, 1e-4)}


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


def _check(got, ref, precision, label):
    med = np.median(np.abs(ref))
    big = np.abs(ref) > 1e-3 * med
    rel = np.abs(got - ref)[big] / np.abs(ref[big])
    scale = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  {label} {precision}: events {big.sum()}/{ref.size} rel err median {np.median(rel):.2e} "
         f"max {rel.max():.2e}; max |d| / max A^2 {scale:.2e}")
    m, mx, sc = BARS[precision]
    assert np.median(rel) < m
    assert rel.max() < mx
    assert scale < sc


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_matches_oracle(api, n, precision):
    E = {4: 96, 5: 96, 6: 40, 7: 24, 8: 12}[n]
    ev = make_events(n, E, seed=8000 + n, cuts=True)
    phi, eta = continuous_states(n, E, 80 + n)
    _say(f"bg_me2_continuous {precision} n={n} E={E}")
    got = api.me2_continuous(_dev(ev["mom"]), _dev(phi), _dev(eta), precision=precision).cpu().numpy()
    ref = ocdmc.me2_continuous(ev["mom"], phi, eta)
    _check(got, ref, precision, f"n={n}")


def test_n9_few_events(api):
    n, E = 9, 6
    ev = make_events(n, E, seed=8009, cuts=True)
    phi, eta = continuous_states(n, E, 89)
    _say(f"bg_me2_continuous n=9 E={E}")
    m, p, h = _dev(ev["mom"]), _dev(phi), _dev(eta)
    ref = ocdmc.me2_continuous(ev["mom"], phi, eta)
    for prec in ("fp64", "fp32"):
        got = api.me2_continuous(m, p, h, precision=prec).cpu().numpy()
        _check(got, ref, prec, "n=9")


@pytest.mark.parametrize("n", [6, 9])
def test_fp32_vs_fp64_many_events(api, n):
    E = 4096 if n == 6 else 1024
    ev = make_events(n, E, seed=8100 + n, cuts=True)
    phi, eta = continuous_states(n, E, 81 + n)
    m, p, h = _dev(ev["mom"]), _dev(phi), _dev(eta)
    _say(f"bg_me2_continuous fp32 vs fp64 n={n} E={E}")
    a = api.me2_continuous(m, p, h, precision="fp64").cpu().numpy()
    b = api.me2_continuous(m, p, h, precision="fp32").cpu().numpy()
    med = np.median(a)
    big = a > 1e-3 * med
    rel = np.abs(a - b)[big] / a[big]
    top = np.max(np.abs(a - b)) / np.max(a)
    _say(f"  median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max |d| / max A^2 {top:.2e}")
    assert np.median(rel) < 1e-5 and np.percentile(rel, 99) < 1e-3
    assert top < 1e-4
    again = api.me2_continuous(m, p, h, precision="fp32").cpu().numpy()
    assert np.array_equal(b, again)


def test_estimator_normalisation(api):
    """9^n times the mean of A^2 over uniform angles and sphere vectors at one
    phase-space point approaches the colour- and helicity-summed |M|^2 of the
    colour-ordered path (n = 6, 2^18 samples, 5 sigma)."""
    n, S = 6, 1 << 18
    ev = make_events(n, 1, seed=8200, cuts=True)
    mom1 = _dev(ev["mom"])
    ref = api.me2(mom1, None, precision="fp64").cpu().numpy()[0]
    phi, eta = continuous_states(n, S, 82)
    mom = _dev(np.repeat(ev["mom"], S, axis=2))
    w = 9.0 ** n * api.me2_continuous(mom, _dev(phi), _dev(eta)).cpu().numpy()
    mean, err = w.mean(), w.std() / np.sqrt(S)
    _say(f"  estimate {mean:.6e} +- {err:.2e} vs summed {ref:.6e}")
    assert abs(mean - ref) < 5 * err


def test_bad_shapes(api):
    ev = make_events(5, 8, seed=8300, cuts=True)
    phi, eta = continuous_states(5, 8, 83)
    with pytest.raises(ValueError):
        api.me2_continuous(_dev(ev["mom"]), _dev(phi[:4]), _dev(eta))
    out = api.me2_continuous(_dev(ev["mom"][:, :, :0]), _dev(phi[:, :0]), _dev(eta[..., :0]))
    assert out.numel() == 0


def test_device_variables_match_host_generator(api):
    """bg_generate_continuous draws the same variables as the host generator
    (same keyed stream and draw layout): angles exactly, unit vectors to a
    few units in the last place of the angle (the two sides' cos and sin
    differ by that); a resumed range equals the tail of a full one."""
    n, E, seed = 7, 5000, 2106
    phi_d, eta_d = api.generate_continuous(n, E, seed, first_event=0)
    phi_h, eta_h = continuous_states(n, E, seed)
    assert np.array_equal(phi_d.cpu().numpy(), phi_h)
    assert np.max(np.abs(eta_d.cpu().numpy() - eta_h)) < 1e-14
    phi_r, eta_r = api.generate_continuous(n, 1000, seed, first_event=4000)
    assert torch.equal(phi_r, phi_d[:, 4000:])
    assert torch.equal(eta_r, eta_d[..., 4000:])
    # feeding the device variables to the evaluation gives the host-input result
    ev = make_events(n, 64, seed=8400, cuts=True)
    m = _dev(ev["mom"])
    a = api.me2_continuous(m, phi_d[:, :64].contiguous(), eta_d[..., :64].contiguous()).cpu().numpy()
    b = api.me2_continuous(m, _dev(phi_h[:, :64]), _dev(eta_h[..., :64])).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9])
def test_single_event(api, n):
    """One event per call (grid of one workgroup), every multiplicity."""
    ev = make_events(n, 1, seed=8500 + n, cuts=True)
    phi, eta = continuous_states(n, 1, 85 + n)
    ref = ocdmc.me2_continuous(ev["mom"], phi, eta)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-3)):
        got = api.me2_continuous(_dev(ev["mom"]), _dev(phi), _dev(eta), precision=prec).cpu().numpy()
        assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (prec, got[0], ref[0])


def test_generate_continuous_edges(api):
    from paper_2106_06507_amd._lib import BGError
    phi, eta = api.generate_continuous(5, 0, 1)
    assert phi.shape == (5, 0) and eta.shape == (2, 5, 3, 0)
    with pytest.raises(BGError):
        api.generate_continuous(3, 10, 1)
