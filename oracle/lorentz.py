"""Minkowski-space helpers.  Metric (+,-,-,-), Levi-Civita eps^{0123} = +1.

Four-vectors are Python lists of four scalars; a scalar is a numpy array over
events (real or complex) or a ``Dual``.  The paper does not state its metric
signature; mostly-minus is the reading consistent with the projector
-g + (pk + kp)/(p.k) of Section 2.1 being positive on physical polarizations.
"""
import itertools


def mdot(a, b):
    """a.b = a0 b0 - a1 b1 - a2 b2 - a3 b3 (no complex conjugation)."""
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def vadd(a, b):
    return [a[i] + b[i] for i in range(4)]


def vsub(a, b):
    return [a[i] - b[i] for i in range(4)]


def vscale(s, a):
    return [s * a[i] for i in range(4)]


def lower(a):
    return [a[0], -a[1], -a[2], -a[3]]


def _perm_sign(p):
    sign = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                sign = -sign
    return sign


_LEVI = [(p, _perm_sign(p)) for p in itertools.permutations(range(4))]


def levi_civita_contract(a, b, c):
    """v^mu = eps^{mu nu rho sigma} a_nu b_rho c_sigma (indices lowered with g)."""
    al, bl, cl = lower(a), lower(b), lower(c)
    out = [0.0, 0.0, 0.0, 0.0]
    for (mu, nu, rho, sg), s in _LEVI:
        term = al[nu] * bl[rho] * cl[sg]
        out[mu] = out[mu] + term if s > 0 else out[mu] - term
    return out
