"""Pins of the oracle's colour-dressed recursion and gradient (CPU only)."""
import itertools

import numpy as np
import pytest

from bg_inputs import make_events
from oracle import cdbg, grad, me2
from tests.helpers import valid_colours, mhv_helicities


def _scale_rel(a, b):
    """|a-b| relative to the largest |b| among events (zeros are rounding-level)."""
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# --------------------------------------------------------------------------
# colour-dressed recursion (eq. cdcurrents, eq. color_dressed_currents)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_dressed_equals_bruteforce_colour_flow(n):
    """Recursion over partitions = literal sum over orderings with delta chains
    (eq. color_decomposition_colorflow)."""
    E = 8
    ev = make_events(n, E, seed=1000 + n, cuts=True)
    col = valid_colours(n, E, np.random.default_rng(n))
    bf = cdbg.flow_amplitude_bruteforce(ev["mom"], ev["hel"], col)
    d = cdbg.flow_amplitude(ev["mom"], ev["hel"], col)
    assert _scale_rel(d, bf) < 1e-12
    big = np.abs(bf) > 1e-6 * np.max(np.abs(bf))
    np.testing.assert_allclose(d[big], bf[big], rtol=1e-9)


@pytest.mark.parametrize("n", [5, 6])
def test_dressed_tensor_equals_explicit_v4(n):
    E = 6
    ev = make_events(n, E, seed=1100 + n, cuts=True)
    col = valid_colours(n, E, np.random.default_rng(10 + n))
    a = cdbg.flow_amplitude(ev["mom"], ev["hel"], col, tensor=True)
    b = cdbg.flow_amplitude(ev["mom"], ev["hel"], col, tensor=False)
    assert _scale_rel(a, b) < 1e-12


def test_dressed_n8_few_events():
    n = 8
    E = 3
    ev = make_events(n, E, seed=1208, cuts=True)
    col = valid_colours(n, E, np.random.default_rng(8))
    bf = cdbg.flow_amplitude_bruteforce(ev["mom"], ev["hel"], col)
    d = cdbg.flow_amplitude(ev["mom"], ev["hel"], col)
    assert _scale_rel(d, bf) < 1e-12


@pytest.mark.parametrize("n", [5, 6])
def test_dressed_currents_traceless(n):
    """The kinematic part of a split (three-gluon vertex and tensor terms)
    changes sign when its two operands are exchanged, so the two orders of a
    split enter eq. color_dressed_currents as the colour commutator
    [J(S1), J(S2)], and every dressed current of two or more gluons has zero
    colour trace.  A vertex term with a wrong sign or momentum (which breaks
    that antisymmetry) leaves an O(1) trace; a reversed colour product flips
    the sign of every current alike and is not seen here.  Currents that are themselves cancellation noise (subsets
    of diagonal gluons of one colour) are left out by their size, and so are
    flows of diagonal gluons only, where every such current is noise."""
    E = 48
    rng = np.random.default_rng(1400 + n)
    ev = make_events(n, E, seed=1400 + n, cuts=True)
    col = valid_colours(n, E, rng)
    J = cdbg.dressed_currents(ev["mom"], ev["hel"], col)
    checked = 0
    for size in range(2, n):
        masks = [S for S in J if bin(S).count("1") == size]
        mag = {S: np.max(np.abs(J[S]), axis=(0, 1, 2)) for S in masks}  # [E]
        top = np.max([mag[S] for S in masks], axis=0)
        for S in masks:
            tr = np.max(np.abs(J[S][0, 0] + J[S][1, 1] + J[S][2, 2]), axis=0)
            use = (mag[S] > 1e-6 * top) & np.any(col[0] != col[1], axis=0)
            assert np.all(tr[use] <= 1e-10 * mag[S][use]), (n, size, S)
            checked += int(use.sum())
    assert checked > E


def test_invalid_colour_flows_vanish():
    """No closed colour chain -> every delta chain is zero -> amplitude exactly 0."""
    n = 6
    E = 64
    ev = make_events(n, E, seed=1300, cuts=True, sample_col=True)
    col = ev["col"]
    valid = cdbg.is_valid_flow(col)
    assert (~valid).sum() > 10
    d = cdbg.flow_amplitude(ev["mom"], ev["hel"], col)
    assert np.all(d[~valid] == 0.0)


@pytest.mark.parametrize("n", [4, 5])
def test_colour_flow_sum_equals_colour_summed(n):
    """sum over all 9^n (i_k, j_k) of |A_flow|^2 = sum_a |A_a|^2 = A^dagger C A."""
    ev = make_events(n, 2, seed=1400 + n, cuts=True)
    hel = mhv_helicities(n, 2, np.random.default_rng(n))
    ref = me2.me2_cobg(ev["mom"], hel)
    cols = np.array(list(itertools.product(range(3), repeat=2 * n)), dtype=np.int8).T
    col = np.stack([cols[0::2], cols[1::2]])
    E = col.shape[2]
    for e in range(2):
        momE = np.repeat(ev["mom"][:, :, e:e + 1], E, axis=2)
        helE = np.repeat(hel[:, e:e + 1], E, axis=1)
        if n == 4:
            a = cdbg.flow_amplitude(momE, helE, col)
        else:
            keep = cdbg.is_valid_flow(col)
            a = cdbg.flow_amplitude(momE[:, :, keep], helE[:, keep], col[:, :, keep])
        np.testing.assert_allclose(np.sum(np.abs(a) ** 2), ref[e], rtol=1e-11)


# --------------------------------------------------------------------------
# gradient of |M|^2 with respect to the momenta
# --------------------------------------------------------------------------
def _nonvanishing_helicities(n, E, seed):
    """MHV, and for n >= 6 alternately next-to-MHV, helicity configurations
    (all-plus and one-minus amplitudes vanish, leaving only rounding noise)."""
    rng = np.random.default_rng(seed)
    h = mhv_helicities(n, E, rng)
    if n >= 6:
        for e in range(1, E, 2):
            k = rng.choice(np.nonzero(h[:, e] > 0)[0])
            h[k, e] = -1
    return h


def _me2_plain(mom, hel):
    return me2.me2_cobg(mom, hel)


@pytest.mark.parametrize("n", [4, 5, 6])
def test_gradient_matches_central_differences(n):
    E = 6 if n < 6 else 4
    ev = make_events(n, E, seed=1500 + n, cuts=True)
    mom = ev["mom"]
    hel = _nonvanishing_helicities(n, E, 1500 + n)
    f, g = grad.me2_and_grad(mom, hel)
    np.testing.assert_allclose(f, _me2_plain(mom, hel), rtol=1e-13)
    for i in range(n):
        for mu in range(4):
            h = 1e-6 * np.abs(mom[i, 0])
            mp = mom.copy()
            mm = mom.copy()
            mp[i, mu] += h
            mm[i, mu] -= h
            fd = (_me2_plain(mp, hel) - _me2_plain(mm, hel)) / (2 * h)
            scale = np.abs(f) / np.abs(mom[i, 0])
            assert np.max(np.abs(fd - g[i, mu]) / (scale + np.abs(g[i, mu]))) < 1e-5, (i, mu)


@pytest.mark.parametrize("n", [5, 6])
def test_gradient_lorentz_and_scaling_identities(n):
    """On-shell, momentum-conserving directions are independent of the
    polarization construction: Euler homogeneity of degree 8 - 2n and the
    vanishing of the rotation and boost generators."""
    E = 6
    ev = make_events(n, E, seed=1600 + n, cuts=True)
    mom = ev["mom"]
    hel = _nonvanishing_helicities(n, E, 1600 + n)
    f, g = grad.me2_and_grad(mom, hel)
    euler = np.einsum("ime,ime->e", mom, g)
    np.testing.assert_allclose(euler, (8 - 2 * n) * f, rtol=1e-8)
    p3 = mom[:, 1:, :]
    g3 = g[:, 1:, :]
    scale = np.abs(f)
    for a, b in ((1, 2), (2, 0), (0, 1)):
        rot = np.sum(p3[:, a] * g3[:, b] - p3[:, b] * g3[:, a], axis=0)
        assert np.max(np.abs(rot) / scale) < 1e-8
    for a in range(3):
        boost = np.sum(mom[:, 0] * g3[:, a] + p3[:, a] * g[:, 0], axis=0)
        assert np.max(np.abs(boost) / scale) < 1e-8
