"""Condition numbers of the colour-summed |M|^2 (TEST INFRASTRUCTURE).

``me2_cobg_magnitude`` runs the colour-ordered recursion of Section 2.3 (eqs.
cobg, cobg_full_amplitude) and the colour sum of Section 2.2 (eq.
color_summed_analytic) on magnitude numbers (``magnitude.Mag``): momenta,
external currents and 1/P^2 enter as rounded inputs, every vertex term adds
its magnitude.  It returns |M|^2 and its magnitude m, so that a
floating-point evaluation with unit roundoff u is expected within a small
multiple of u m of the exact value.
"""
import numpy as np

from .cobg import ddm_orderings, external_currents, momenta_list, ordered_amplitude
from .color import color_matrix_cached
from .magnitude import Mag, lift


def amplitudes_magnitude(mom, hel):
    """(A [K, E] complex, m_A [K, E]) for the adjoint-basis orderings."""
    n = mom.shape[0]
    ps_plain = momenta_list(mom)
    eps = [lift(e) for e in external_currents(ps_plain, hel)]
    ps = [lift(p) for p in ps_plain]
    vals, mags = [], []
    for o in ddm_orderings(n):
        a = ordered_amplitude(ps, eps, o)
        vals.append(a.v)
        mags.append(a.m)
    return np.array(vals), np.array(mags)


def me2_cobg_magnitude(mom, hel, C=None):
    """(|M|^2 [E], m [E]) for one helicity configuration per event."""
    n = mom.shape[0]
    if C is None:
        C = color_matrix_cached(n)
    Cf = np.asarray(C, dtype=np.float64)
    A, mA = amplitudes_magnitude(mom, hel)
    me2 = np.real(np.einsum("se,st,te->e", A, Cf, np.conj(A)))
    mag = np.einsum("se,st,te->e", mA, np.abs(Cf), mA)
    return me2, mag


def _closing_orderings(col_e):
    """Orderings (0, s) whose colour chain closes for one event's colour
    labels col_e [2][n] (a depth-first walk along the chain: the gluon after
    position a must have j equal to i of the gluon at a)."""
    n = col_e.shape[1]
    i, j = col_e[0], col_e[1]
    out = []

    def walk(order, left):
        if not left:
            if i[order[-1]] == j[order[0]]:
                out.append(tuple(order))
            return
        for k in sorted(left):
            if j[k] == i[order[-1]]:
                walk(order + [k], left - {k})

    walk([0], set(range(1, n)))
    return out


def flow_amplitude_magnitude(mom, hel, col):
    """(A [E] complex, m_A [E]) for the colour-flow amplitude of eq.
    color_decomposition_colorflow, written as the sum of the colour-ordered
    amplitudes whose delta chain closes (each with weight 1), every one
    evaluated on magnitude numbers.  One event at a time (small samples)."""
    n, _, E = mom.shape
    vals = np.zeros(E, dtype=complex)
    mags = np.zeros(E)
    for e in range(E):
        m1 = mom[:, :, e:e + 1]
        h1 = hel[:, e:e + 1]
        ps_plain = momenta_list(m1)
        eps = [lift(x) for x in external_currents(ps_plain, h1)]
        ps = [lift(p) for p in ps_plain]
        for o in _closing_orderings(col[:, :, e]):
            a = ordered_amplitude(ps, eps, o)
            vals[e] += complex(np.ravel(a.v)[0])
            mags[e] += float(np.ravel(a.m)[0])
    return vals, mags
