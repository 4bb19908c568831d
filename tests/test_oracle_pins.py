"""Pins of the FP64 oracle against closed forms and identities (CPU only).

Each test names what fixes the expected value: a textbook closed form, an
identity of the paper, or a brute-force evaluation of a definition.
"""
import itertools
import math

import numpy as np
import pytest

from bg_inputs import make_events
from oracle import cobg, color, me2, polarization
from oracle.cobg import G_S, momenta_list, external_currents, ordered_amplitude
from oracle.lorentz import mdot
from tests.helpers import mhv_helicities, sij, mink

RNG_SEED = 20260101


def _events(n, E, seed, cuts=True):
    return make_events(n, E, seed=seed, cuts=cuts, sample_hel=True)


# --------------------------------------------------------------------------
# polarization vectors: eq. tensor_axial and eq. helicity_axial (Section 2.1)
# --------------------------------------------------------------------------
def test_polarization_transverse_normalised_complete():
    ev = _events(6, 64, 11)
    mom = ev["mom"]
    for i in range(6):
        p = [mom[i, mu] for mu in range(4)]
        k = [np.sign(p[0]) * p[mu] for mu in range(4)]
        q = polarization.gauge_vector(p)
        assert np.max(np.abs(mdot(q, q)) / q[0] ** 2) < 1e-14  # light-like
        ep = polarization.external_current(p, np.ones(64))
        em = polarization.external_current(p, -np.ones(64))
        scale = np.abs(k[0])
        for e in (ep, em):
            assert np.max(np.abs(mdot(e, k)) / scale) < 1e-14
            assert np.max(np.abs(mdot(e, q)) / scale) < 1e-14
            assert np.max(np.abs(mdot(e, [np.conj(x) for x in e]) + 1.0)) < 1e-14
            assert np.max(np.abs(mdot(e, e))) < 1e-14  # helicity states are null
            assert np.max(np.abs(np.array(e))) <= 1.0 + 1e-15
        # eq. helicity_axial: sum_lambda eps eps^dagger = P(k, q) (both indices up)
        P = polarization.projector(k, q)
        for a in range(4):
            for b in range(4):
                s = ep[a] * np.conj(ep[b]) + em[a] * np.conj(em[b])
                assert np.max(np.abs(s - P[a][b])) < 1e-13


def test_polarization_helicity_sign_along_z():
    # k along +z: (e1, e2, z) right-handed, so eps^+ = (e1 + i e2)/sqrt2 ~ (x + i y)
    # carries J_z = +1.
    p = [np.array([1.0]), np.array([0.0]), np.array([0.0]), np.array([1.0])]
    e1, e2 = polarization.basis(p)
    cross_z = e1[1][0] * e2[2][0] - e1[2][0] * e2[1][0]
    assert cross_z == pytest.approx(1.0, abs=1e-14)
    assert abs(e1[0][0]) == 0.0 and abs(e2[0][0]) == 0.0


# --------------------------------------------------------------------------
# colour-ordered amplitudes (Section 2.3, eq. cobg, eq. cobg_full_amplitude)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_parke_taylor_magnitude(n):
    """|A(1..n)|^2 = g^(2(n-2)) s_jl^4 / prod |s_i,i+1| for two negative helicities."""
    E = 24
    ev = _events(n, E, 100 + n)
    mom = ev["mom"]
    rng = np.random.default_rng(RNG_SEED + n)
    hel = mhv_helicities(n, E, rng)
    for order in [tuple(range(n)), tuple(rng.permutation(n))]:
        a = cobg.amplitude_of(mom, hel, order)
        jl = [np.nonzero(hel[:, e] < 0)[0] for e in range(E)]
        num = np.array([sij(mom[:, :, e:e + 1], j, l)[0] ** 4 for e, (j, l) in enumerate(jl)])
        den = 1.0
        for k in range(n):
            den = den * np.abs(sij(mom, order[k], order[(k + 1) % n]))
        pt = G_S ** (2 * (n - 2)) * num / den
        np.testing.assert_allclose(np.abs(a) ** 2, pt, rtol=1e-8)
        # the conjugate configuration (two positive helicities) has the same magnitude
        b = cobg.amplitude_of(mom, -hel, order)
        np.testing.assert_allclose(np.abs(b) ** 2, pt, rtol=1e-8)


@pytest.mark.parametrize("n", [5, 6])
def test_vanishing_helicity_configurations(n):
    """All-plus and one-minus tree amplitudes vanish (relative to the MHV scale)."""
    E = 16
    mom = _events(n, E, 200 + n)["mom"]
    rng = np.random.default_rng(3)
    ref = np.abs(cobg.amplitude_of(mom, mhv_helicities(n, E, rng), tuple(range(n))))
    allp = np.ones((n, E))
    onem = np.ones((n, E))
    onem[2] = -1
    for h in (allp, onem, -allp, -onem):
        a = np.abs(cobg.amplitude_of(mom, h, tuple(range(n))))
        assert np.max(a / ref) < 1e-10


@pytest.mark.parametrize("n", [5, 6, 7])
def test_cyclicity_reflection(n):
    E = 16
    ev = _events(n, E, 300 + n)
    mom, hel = ev["mom"], ev["hel"]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    base = tuple(range(n))
    a = ordered_amplitude(ps, eps, base)
    scale = np.max(np.abs(a))
    for r in range(1, n):
        b = ordered_amplitude(ps, eps, base[r:] + base[:r])
        assert np.max(np.abs(a - b)) / scale < 1e-9
    rev = ordered_amplitude(ps, eps, tuple(reversed(base)))
    assert np.max(np.abs(rev - (-1) ** n * a)) / scale < 1e-9


@pytest.mark.parametrize("n", [5, 6, 7])
def test_u1_decoupling(n):
    """Sum over insertions of gluon 1 into the cyclic order of 2..n vanishes."""
    E = 16
    mom = _events(n, E, 400 + n)["mom"]
    hel = mhv_helicities(n, E, np.random.default_rng(n))
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    rest = list(range(1, n))
    tot = 0.0
    scale = 0.0
    for p in range(n - 1):
        a = ordered_amplitude(ps, eps, tuple(rest[:p] + [0] + rest[p:]))
        tot = tot + a
        scale = np.maximum(scale, np.abs(a))
    assert np.max(np.abs(tot) / scale) < 1e-9


def _shuffles(a, b):
    if not a:
        return [tuple(b)]
    if not b:
        return [tuple(a)]
    return [(a[0],) + s for s in _shuffles(a[1:], b)] + [(b[0],) + s for s in _shuffles(a, b[1:])]


@pytest.mark.parametrize("split", [1, 2, 3])
def test_kleiss_kuijf(split):
    """A(1, alpha, n, beta) = (-1)^|beta| sum_{s in alpha ⧢ beta^T} A(1, s, n)."""
    n = 7
    E = 12
    mom = _events(n, E, 500 + split)["mom"]
    hel = mhv_helicities(n, E, np.random.default_rng(split))
    hel[:, ::2] = np.random.default_rng(99).choice([-1, 1], size=(n, (E + 1) // 2))
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    mid = list(range(1, n - 1))
    alpha, beta = mid[:split], mid[split:]
    lhs = ordered_amplitude(ps, eps, (0,) + tuple(alpha) + (n - 1,) + tuple(beta))
    rhs = 0.0
    for s in _shuffles(alpha, list(reversed(beta))):
        rhs = rhs + ordered_amplitude(ps, eps, (0,) + s + (n - 1,))
    rhs = (-1) ** len(beta) * rhs
    scale = np.maximum(np.abs(lhs), 1e-300)
    ok = np.abs(lhs) > 1e-8 * np.max(np.abs(lhs))
    assert np.max((np.abs(lhs - rhs) / scale)[ok]) < 1e-9


@pytest.mark.parametrize("n", [4, 5, 6])
def test_gauge_invariance(n):
    """Replacing any polarization by its momentum gives a vanishing amplitude."""
    E = 16
    ev = _events(n, E, 600 + n)
    mom, hel = ev["mom"], ev["hel"]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    order = tuple(range(n))
    ref = np.abs(ordered_amplitude(ps, eps, order))
    ref = np.maximum(ref, np.max(ref) * 1e-3)
    for i in range(n):
        e2 = list(eps)
        e2[i] = [ps[i][mu].astype(np.complex128) / np.abs(ps[i][0]) for mu in range(4)]
        a = ordered_amplitude(ps, e2, order)
        assert np.max(np.abs(a) / ref) < 1e-9, i


@pytest.mark.parametrize("n", [5, 6, 7])
def test_tensor_form_equals_explicit_v4(n):
    """eq. cobg_tensor / cobg_tensor_current reproduce the explicit V4 recursion."""
    E = 8
    ev = _events(n, E, 700 + n)
    a = cobg.partial_amplitudes(ev["mom"], ev["hel"])
    b = cobg.partial_amplitudes(ev["mom"], ev["hel"], tensor=True)
    assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-13


@pytest.mark.parametrize("n", [5, 6])
def test_gauge_vector_independence(n):
    """|A|^2 is the same in the radiation gauge and in light-cone gauges with a
    fixed gauge vector (eq. tensor_axial holds for any light-like k)."""
    E = 16
    ev = _events(n, E, 800 + n)
    mom, hel = ev["mom"], ev["hel"]
    ps = momenta_list(mom)
    a1 = np.abs(cobg.partial_amplitudes(mom, hel))
    for q, r in (((1.0, 2 / 7, 3 / 7, 6 / 7), (0.0, 3 / 7, -6 / 7, 2 / 7)),
                 ((1.0, -6 / 7, 2 / 7, 3 / 7), (0.0, 3 / 7, 6 / 7, 2 / 7))):
        fn = lambda p, q=q, r=r: polarization.basis_lightcone(p, list(q), list(r))
        eps = [polarization.external_current(ps[i], hel[i], basis_fn=fn) for i in range(n)]
        a2 = np.abs(np.array([ordered_amplitude(ps, eps, o) for o in cobg.ddm_orderings(n)]))
        assert np.max(np.abs(a1 - a2)) / np.max(a1) < 1e-9


# --------------------------------------------------------------------------
# colour matrix and assembly (Section 2.2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [4, 5, 6])
def test_colour_matrix_exact_equals_gellmann(n):
    """Exact trace-word evaluation equals eq. color_coefficient_adjoint with
    explicit Gell-Mann F matrices."""
    Ce = color.color_matrix(n).astype(np.float64)
    Cg = color.color_matrix_gellmann(n)
    assert np.max(np.abs(Ce - Cg)) < 1e-9 * np.max(Ce)


def test_projection_identity():
    """F^a_bc T^a_ij T^b_kl T^c_mn = d_il d_kn d_mj - d_in d_kj d_ml (Section 2.3)."""
    F = color.adjoint_F()
    T = color.gellmann_generators()
    lhs = np.einsum("abc,aij,bkl,cmn->ijklmn", F, T, T, T)
    d = np.eye(3)
    rhs = np.einsum("il,kn,mj->ijklmn", d, d, d) - np.einsum("in,kj,ml->ijklmn", d, d, d)
    assert np.max(np.abs(lhs - rhs)) < 1e-14


@pytest.mark.parametrize("n", [4, 5, 6])
def test_colour_matrix_symmetries(n):
    C = color.color_matrix(n)
    assert np.array_equal(C, C.T)
    assert np.all(np.linalg.eigvalsh(C.astype(float)) > 0)
    assert np.array_equal(C, color.color_matrix(n, relabel=True))
    # diagonal: sum_a |(F..F)_{a1 an}|^2 = C_A^(n-2) (N^2-1) with the adjoint
    # Casimir C_A = 2N in the Tr(T^a T^b) = delta^ab normalisation
    assert np.all(np.diag(C) == 6 ** (n - 2) * 8)


@pytest.mark.parametrize("n", [4, 5])
def test_leading_colour_formula_exact_at_low_n(n):
    """Section 3.1 leading-colour formula has no 1/N^2 terms for n = 4, 5."""
    E = 12
    mom = _events(n, E, 900 + n)["mom"]
    hel = mhv_helicities(n, E, np.random.default_rng(n))
    full = me2.me2_cobg(mom, hel)
    lc = me2.me2_leading_colour(mom, hel)
    np.testing.assert_allclose(full, lc, rtol=1e-11)


def test_gg_gg_closed_form():
    """Colour- and helicity-summed gg -> gg: 4 g^4 N^2(N^2-1)(s^4+t^4+u^4)(s^2+t^2+u^2)/(s t u)^2
    = 256 x (9/2) g^4 (3 - tu/s^2 - su/t^2 - st/u^2) at N = 3 (textbook)."""
    ev = make_events(4, 64, seed=1234, cuts=False, sample_hel=False)
    mom = ev["mom"]
    m = me2.me2_cobg(mom, None)
    s, t = sij(mom, 0, 1), sij(mom, 0, 2)
    u = sij(mom, 0, 3)
    f1 = 4 * G_S ** 4 * 9 * 8 * (s ** 4 + t ** 4 + u ** 4) * (s ** 2 + t ** 2 + u ** 2) / (s * t * u) ** 2
    f2 = 1152 * G_S ** 4 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
    np.testing.assert_allclose(m, f1, rtol=1e-11)
    np.testing.assert_allclose(m, f2, rtol=1e-11)


def test_five_gluon_closed_form():
    """n = 5: |M|^2 = N^3 (N^2-1) g^6 sum over MHV and anti-MHV helicities of
    sum_{rho in S_4} s_jl^4 / prod |s_i,i+1| (Parke-Taylor, leading colour exact)."""
    n = 5
    E = 8
    mom = make_events(n, E, seed=55, cuts=True, sample_hel=False)["mom"]
    m = me2.me2_cobg(mom, None)
    ref = 0.0
    for h in itertools.product((1, -1), repeat=n):
        neg = [i for i in range(n) if h[i] < 0]
        pos = [i for i in range(n) if h[i] > 0]
        pair = neg if len(neg) == 2 else (pos if len(pos) == 2 else None)
        if pair is None:
            continue
        num = sij(mom, pair[0], pair[1]) ** 4
        for rho in itertools.permutations(range(1, n)):
            o = (0,) + rho
            den = 1.0
            for k in range(n):
                den = den * np.abs(sij(mom, o[k], o[(k + 1) % n]))
            ref = ref + num / den
    ref = 27 * 8 * G_S ** 6 * ref
    np.testing.assert_allclose(m, ref, rtol=1e-10)
