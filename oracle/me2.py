"""Colour- and helicity-summed squared matrix elements (Section 2.2).

eq. color_summed_analytic:
    |A|^2 = sum_{sigma, sigma'} C_{sigma sigma'} sum_lambda A_sigma A_sigma'^*
with C from ``color``.  ``me2_cobg`` returns the colour-summed value for one
helicity configuration per event (hel given) or summed over all 2^n
configurations (hel None, eq. full_amplitude_decomposition_discrete_summation).
No averaging over initial states and no symmetry factor is applied.

``me2_leading_colour`` is the leading-colour formula of Section 3.1,
N^(n-2) (N^2 - 1) sum_{S_(n-1)} |A(1, sigma)|^2, used as a check: it is exact
for n = 4, 5.
"""
import itertools

import numpy as np

from .cobg import G_S, partial_amplitudes, momenta_list, external_currents, ordered_amplitude
from .color import color_matrix_cached, NC


def helicity_configs(n):
    """All 2^n helicity tuples, +1 before -1 per gluon (gluon 1 slowest)."""
    return list(itertools.product((1, -1), repeat=n))


def contract(amps, C):
    """sum_{s,s'} C_{ss'} Re(A_s conj(A_s')) for amps [K, E]."""
    Cf = np.asarray(C, dtype=np.float64)
    return np.real(np.einsum("se,st,te->e", amps, Cf, np.conj(amps)))


def me2_cobg(mom, hel=None, g=None, C=None):
    """Colour-summed |M|^2 per event: float64 [E]."""
    n = mom.shape[0]
    if C is None:
        C = color_matrix_cached(n)
    if hel is not None:
        return contract(partial_amplitudes(mom, hel, g=g), C)
    out = 0.0
    for h in helicity_configs(n):
        hh = [np.full(mom.shape[2:], hi, dtype=np.float64) for hi in h]
        out = out + contract(partial_amplitudes(mom, hh, g=g), C)
    return out


def me2_leading_colour(mom, hel, g=None, nc=NC):
    """N^(n-2)(N^2-1) sum over orderings (1, rho) of |A|^2 for one helicity."""
    n = mom.shape[0]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    tot = 0.0
    for rho in itertools.permutations(range(1, n)):
        a = ordered_amplitude(ps, eps, (0,) + rho, g=g)
        tot = tot + np.abs(a) ** 2
    return nc ** (n - 2) * (nc * nc - 1) * tot
