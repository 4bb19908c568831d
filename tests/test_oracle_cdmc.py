"""Pins of the oracle's continuous colour / polarization sampling (CPU only).

The amplitude with real polarizations e(phi) and colour vectors (eta,
etabar) must reduce to the colour-flow amplitude for basis vectors and
complex helicity currents; average to the helicity sum over phi (exactly on
a three-point grid per gluon, since |A|^2 is a trigonometric polynomial of
degree 2 in each phi); average to the colour sum over the colour vectors
(exactly on any orthonormal basis per vector, since |A|^2 is quadratic in
each vector and E[eta eta^T] = 1/3); be real; and obey the Ward identity.
"""
import itertools

import numpy as np
import pytest

from bg_inputs import make_events
from oracle import cdbg, cdmc, me2
from oracle.cobg import external_currents, momenta_list
from oracle.lorentz import mdot
from tests.helpers import valid_colours, mhv_helicities


def _rand_unit(rng, shape):
    v = rng.normal(size=(3,) + shape)
    return v / np.linalg.norm(v, axis=0)


def _eta(n, E, rng):
    return np.stack([_rand_unit(rng, (n, E)).transpose(1, 0, 2),
                     _rand_unit(rng, (n, E)).transpose(1, 0, 2)])


@pytest.mark.parametrize("n", [4, 5, 6])
def test_flow_limit(n):
    """Basis vectors eta = e_i, etabar = e_j and helicity currents give the
    colour-flow amplitude (itself pinned to the literal sum over orderings)."""
    E = 10
    ev = make_events(n, E, seed=2000 + n, cuts=True)
    col = valid_colours(n, E, np.random.default_rng(20 + n))
    eye = np.eye(3)
    eta = np.stack([eye[col[0]].transpose(0, 2, 1), eye[col[1]].transpose(0, 2, 1)])  # [2][n][3][E]
    ps = momenta_list(ev["mom"])
    eps = external_currents(ps, ev["hel"])
    a = cdmc.amplitude_general(ps, eps, cdmc.colour_matrices(eta), eta[0, n - 1], eta[1, n - 1])
    ref = cdbg.flow_amplitude(ev["mom"], ev["hel"], col)
    assert np.max(np.abs(a - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [4, 5, 6])
def test_real_and_ward(n):
    """All-real inputs give a real amplitude; replacing one polarization by
    its gluon's momentum gives zero (current conservation)."""
    E = 12
    rng = np.random.default_rng(2100 + n)
    ev = make_events(n, E, seed=2100 + n, cuts=True)
    phi = rng.uniform(0.0, 2 * np.pi, (n, E))
    eta = _eta(n, E, rng)
    a = cdmc.continuous_amplitude(ev["mom"], phi, eta)
    assert np.all(np.imag(a) == 0.0)
    ps = momenta_list(ev["mom"])
    eps = cdmc.real_polarizations(ps, phi)
    for k in (0, n // 2, n - 1):
        e2 = list(eps)
        e2[k] = ps[k]
        w = cdmc.amplitude_general(ps, e2, cdmc.colour_matrices(eta), eta[0, n - 1], eta[1, n - 1])
        # the momentum has size sqrt(s)/n ~ 1e2 against |e| = sqrt2
        assert np.max(np.abs(w)) < 1e-11 * 1e2 * np.max(np.abs(a))


def test_real_polarization_vectors():
    """e(phi) is transverse, e.e = -2, and sqrt2 e1, sqrt2 e2 at phi = 0, pi/2."""
    ev = make_events(5, 20, seed=2200, cuts=True)
    ps = momenta_list(ev["mom"])
    rng = np.random.default_rng(1)
    phi = rng.uniform(0.0, 2 * np.pi, (5, 20))
    for k, e in enumerate(cdmc.real_polarizations(ps, phi)):
        np.testing.assert_allclose(mdot(e, e), -2.0, rtol=1e-13)
        assert np.max(np.abs(mdot(e, ps[k]))) < 1e-12 * 1e3


@pytest.mark.parametrize("n", [4, 5])
def test_phi_average_is_helicity_sum(n):
    """mean of A(e(phi))^2 over phi_k in {0, 2pi/3, 4pi/3}^n equals
    sum over helicities of |A_h|^2 for the same colour vectors."""
    rng = np.random.default_rng(2300 + n)
    ev = make_events(n, 3, seed=2300 + n, cuts=True)
    eta1 = _eta(n, 3, rng)
    grid = np.array(list(itertools.product(range(3), repeat=n)), dtype=float).T * (2 * np.pi / 3)
    hels = np.array(list(itertools.product((1, -1), repeat=n)), dtype=np.int8).T
    for e in range(3):
        G = grid.shape[1]
        mom = np.repeat(ev["mom"][:, :, e:e + 1], G, axis=2)
        eta = np.repeat(eta1[..., e:e + 1], G, axis=-1)
        avg = np.mean(cdmc.me2_continuous(mom, grid, eta))
        H = hels.shape[1]
        momh = np.repeat(ev["mom"][:, :, e:e + 1], H, axis=2)
        etah = np.repeat(eta1[..., e:e + 1], H, axis=-1)
        ps = momenta_list(momh)
        eps = external_currents(ps, hels)
        ah = cdmc.amplitude_general(ps, eps, cdmc.colour_matrices(etah), etah[0, n - 1], etah[1, n - 1])
        np.testing.assert_allclose(avg, np.sum(np.abs(ah) ** 2), rtol=1e-11)


def test_colour_average_is_colour_sum():
    """9^n times the mean of |A_h|^2 over a rotated orthonormal basis for
    every eta and etabar equals the colour-summed |M_h|^2 of the
    colour-ordered decomposition with the exact colour matrix."""
    n = 4
    rng = np.random.default_rng(2400)
    ev = make_events(n, 2, seed=2400, cuts=True)
    hel = mhv_helicities(n, 2, rng)
    ref = me2.me2_cobg(ev["mom"], hel)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))  # columns: a rotated basis
    idx = np.array(list(itertools.product(range(3), repeat=2 * n))).T  # [2n][9^n]
    G = idx.shape[1]
    eta = np.stack([q[:, idx[0::2]].transpose(1, 0, 2), q[:, idx[1::2]].transpose(1, 0, 2)])
    for e in range(2):
        mom = np.repeat(ev["mom"][:, :, e:e + 1], G, axis=2)
        h = np.repeat(hel[:, e:e + 1], G, axis=1)
        ps = momenta_list(mom)
        eps = external_currents(ps, h)
        a = cdmc.amplitude_general(ps, eps, cdmc.colour_matrices(eta), eta[0, n - 1], eta[1, n - 1])
        est = cdmc.COLOUR_WEIGHT ** n * np.mean(np.abs(a) ** 2)
        np.testing.assert_allclose(est, ref[e], rtol=1e-11)


def test_tensor_form_equals_explicit_v4():
    n = 5
    rng = np.random.default_rng(2500)
    ev = make_events(n, 6, seed=2500, cuts=True)
    phi = rng.uniform(0.0, 2 * np.pi, (n, 6))
    eta = _eta(n, 6, rng)
    a = cdmc.continuous_amplitude(ev["mom"], phi, eta, tensor=True)
    b = cdmc.continuous_amplitude(ev["mom"], phi, eta, tensor=False)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_sphere_vectors_uniform():
    """eq. color_angles with uniform cos(theta) and phi: unit vectors with
    second moments 1/3 (Monte Carlo, 4 sigma)."""
    rng = np.random.default_rng(2600)
    v = cdmc.sphere_vector(rng.uniform(size=200000), rng.uniform(size=200000))
    np.testing.assert_allclose(np.linalg.norm(v, axis=0), 1.0, rtol=1e-14)
    m = v @ v.T / v.shape[1]
    assert np.max(np.abs(m - np.eye(3) / 3)) < 4 * np.sqrt(0.1 / 200000) * 3


def test_estimator_monte_carlo():
    """9^n E[A^2] over uniform phi and sphere vectors approaches the colour-
    and helicity-summed |M|^2 (n = 4, 40000 samples, 5 sigma)."""
    n = 4
    S = 40000
    rng = np.random.default_rng(2700)
    ev = make_events(n, 1, seed=2700, cuts=True)
    ref = me2.me2_cobg(ev["mom"], None)[0]
    mom = np.repeat(ev["mom"], S, axis=2)
    phi = rng.uniform(0.0, 2 * np.pi, (n, S))
    eta = np.stack([cdmc.sphere_vector(rng.uniform(size=(n, S)), rng.uniform(size=(n, S))).transpose(1, 0, 2)
                    for _ in range(2)])
    w = cdmc.COLOUR_WEIGHT ** n * cdmc.me2_continuous(mom, phi, eta)
    mean, err = w.mean(), w.std() / np.sqrt(S)
    assert abs(mean - ref) < 5 * err
