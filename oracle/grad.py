"""Gradient d|M|^2/dp_i^mu of the colour-summed squared matrix element.

The function differentiated is the oracle's |M|^2 for one helicity
configuration per event, evaluated with the generic Minkowski P^2 and the
polarization construction of ``polarization`` (both applied verbatim off the
mass shell).  Each of the 4n partial derivatives is one forward-mode pass of
the unchanged recursion on dual numbers: with A_sigma and dA_sigma,
    d|M|^2 = 2 Re sum_{sigma sigma'} C_{sigma sigma'} dA_sigma conj(A_sigma')
(C real symmetric, eq. color_summed_analytic).
"""
import numpy as np

from .cobg import G_S, ddm_orderings, external_currents, ordered_amplitude
from .color import color_matrix_cached
from .dual import Dual


def me2_and_grad(mom, hel, g=None, C=None):
    """(me2 [E], grad [n][4][E]) for per-event helicities hel [n][E]."""
    n = mom.shape[0]
    E = mom.shape[2]
    if C is None:
        C = color_matrix_cached(n)
    Cf = np.asarray(C, dtype=np.float64)
    orders = ddm_orderings(n)
    grad = np.zeros((n, 4, E))
    me2 = None
    for i in range(n):
        for mu in range(4):
            ps = []
            for a in range(n):
                vec = []
                for nu in range(4):
                    d = np.ones(E) if (a == i and nu == mu) else np.zeros(E)
                    vec.append(Dual(mom[a, nu].copy(), d))
                ps.append(vec)
            eps = external_currents(ps, hel)
            amps = [ordered_amplitude(ps, eps, o, g=g) for o in orders]
            A = np.array([a.v for a in amps])
            dA = np.array([a.d for a in amps])
            if me2 is None:
                me2 = np.real(np.einsum("se,st,te->e", A, Cf, np.conj(A)))
            grad[i, mu] = 2.0 * np.real(np.einsum("se,st,te->e", dA, Cf, np.conj(A)))
    return me2, grad
