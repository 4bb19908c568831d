"""External gluon polarization vectors (Section 2.1).

The paper defines the light-cone projector
    P_{mu nu}(p, k) = -g_{mu nu} + (p_mu k_nu + p_nu k_mu) / (p.k)
(eq. tensor_axial) and its dyadic split into helicity vectors,
P = sum_lambda eps^lambda eps^lambda-dagger (eq. helicity_axial), and states
that external currents are these polarization vectors (Section 2.3).  It does
not fix a construction; the reading used here (shared as a definition with
the HIP library, not as code):

  * k = sign(p^0) p is the physical (positive-energy) momentum of a gluon whose
    all-outgoing momentum is p.
  * Gauge vector q = (1, 2/7, 3/7, 6/7) (light-like) and a fixed space-like
    r = (0, 3/7, -6/7, 2/7) with q.r = 0.
  * e1 = P(k, q) r = -r + q (k.r)/(k.q)   (e1.k = e1.q = 0, e1.e1 = -1)
    e2^mu = eps^{mu nu rho sigma} k_nu q_rho e1_sigma / (k.q)
  * eps^+ = (e1 + i e2)/sqrt(2), eps^- = (e1 - i e2)/sqrt(2) = (eps^+)*;
    for k along +z, e1 = x, e2 = y and eps^+ carries J_z = +1.
  * A gluon with (all-outgoing) helicity label h uses the external current
    (eps^h(k))* = (e1 - i h e2)/sqrt(2).
The formulas are applied verbatim off the mass shell, which defines the
function that the gradient differentiates.
"""
import math

import numpy as np

from .dual import value
from .lorentz import mdot, levi_civita_contract

Q_REF = (1.0, 2.0 / 7.0, 3.0 / 7.0, 6.0 / 7.0)
R_REF = (0.0, 3.0 / 7.0, -6.0 / 7.0, 2.0 / 7.0)
INV_SQRT2 = 1.0 / math.sqrt(2.0)


def basis(p):
    """(e1, e2) for the all-outgoing momentum p (list of 4 scalars)."""
    s = np.where(value(p[0]) > 0.0, 1.0, -1.0)
    k = [s * p[i] for i in range(4)]
    q = list(Q_REF)
    r = list(R_REF)
    kq = mdot(k, q)
    kr = mdot(k, r)
    c = kr / kq
    e1 = [-r[i] + q[i] * c for i in range(4)]
    w = levi_civita_contract(k, q, e1)
    e2 = [w[i] / kq for i in range(4)]
    return e1, e2


def external_current(p, h):
    """(eps^h(k))* = (e1 - i h e2)/sqrt(2); h is an array of +-1."""
    e1, e2 = basis(p)
    ih = 1j * np.asarray(h, dtype=np.float64)
    return [(e1[i] - ih * e2[i]) * INV_SQRT2 for i in range(4)]


def projector(p, kref):
    """P_{mu nu}(p, kref) with both indices up (4x4 nested list)."""
    g = [1.0, -1.0, -1.0, -1.0]
    pk = mdot(p, kref)
    return [[(-g[m] if m == n else 0.0) + (p[m] * kref[n] + p[n] * kref[m]) / pk
             for n in range(4)] for m in range(4)]
