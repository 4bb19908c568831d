"""External gluon polarization vectors (Section 2.1).

The paper defines the light-cone projector
    P_{mu nu}(p, k) = -g_{mu nu} + (p_mu k_nu + p_nu k_mu) / (p.k)
with an arbitrary light-like gauge vector k (eq. tensor_axial; one per gluon in
eq. full_amplitude_decomposition), its dyadic split into helicity vectors,
P = sum_lambda eps^lambda eps^lambda-dagger (eq. helicity_axial), and takes
these vectors as the external currents (Section 2.3).  It fixes no explicit
construction.  The reading used here (shared with the HIP library as a
definition, not as code) is the light-cone gauge with the gauge vector
q = (|k|, -k_vec) opposite to each gluon, i.e. purely spatial polarizations:

  * k = sign(p^0) p is the physical (positive-energy) momentum of a gluon whose
    all-outgoing momentum is p; kappa = |k_vec|.
  * a fixed unit three-vector r = (3, -6, 2)/7 orients the transverse plane:
        e1 = (r kappa^2 - (r.k) k) / |r kappa^2 - (r.k) k|,   e1^0 = 0,
        e2 = (k_vec x e1) / kappa,                             e2^0 = 0.
    (e1, e2, k_vec) is right-handed, e1.e1 = e2.e2 = -1, both transverse to k
    and to q.
  * eps^+ = (e1 + i e2)/sqrt2, eps^- = (eps^+)*; for k along +z and r along x
    this is (x + i y)/sqrt2, J_z = +1.
  * A gluon with (all-outgoing) helicity label h uses the external current
    (eps^h(k))* = (e1 - i h e2)/sqrt2.
All components are bounded by 1, so no large pure-gauge parts enter the
recursion (a fixed light-like q makes eps grow like 1/angle(k, q) and the
amplitude ill-conditioned).  The formulas are applied verbatim off the mass
shell, which defines the function that the gradient differentiates.

``basis_lightcone`` is the construction with a fixed light-like gauge vector;
it is used by the tests to check that |A| does not depend on the gauge.
"""
import math

import numpy as np

from .dual import value
from .lorentz import mdot, levi_civita_contract
from .numeric import sqrt2

R_REF = (3.0 / 7.0, -6.0 / 7.0, 2.0 / 7.0)
INV_SQRT2 = 1.0 / math.sqrt(2.0)


def _sign_k(p):
    s = np.where(value(p[0]) > 0.0, 1.0, -1.0)
    return [s * p[i] for i in range(4)]


def basis(p):
    """(e1, e2) for the all-outgoing momentum p (list of 4 scalars)."""
    k = _sign_k(p)
    kv = k[1:]
    r = list(R_REF)
    kk = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]
    rk = r[0] * kv[0] + r[1] * kv[1] + r[2] * kv[2]
    v = [r[i] * kk - rk * kv[i] for i in range(3)]
    nv = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) ** 0.5
    e1 = [v[i] / nv for i in range(3)]
    kap = kk ** 0.5
    e2 = [(kv[1] * e1[2] - kv[2] * e1[1]) / kap,
          (kv[2] * e1[0] - kv[0] * e1[2]) / kap,
          (kv[0] * e1[1] - kv[1] * e1[0]) / kap]
    zero = 0.0 * kap
    return [zero] + e1, [zero] + e2


def gauge_vector(p):
    """The light-like gauge vector q = (|k|, -k_vec) of ``basis``."""
    k = _sign_k(p)
    kap = (k[1] * k[1] + k[2] * k[2] + k[3] * k[3]) ** 0.5
    return [kap, -k[1], -k[2], -k[3]]


def basis_lightcone(p, q, r):
    """(e1, e2) in light-cone gauge with a fixed light-like q and space-like r, q.r = 0:
    e1 = -r + q (k.r)/(k.q), e2^mu = eps^{mu nu rho sigma} k_nu q_rho e1_sigma / (k.q)."""
    k = _sign_k(p)
    kq = mdot(k, q)
    c = mdot(k, r) / kq
    e1 = [-r[i] + q[i] * c for i in range(4)]
    w = levi_civita_contract(k, q, e1)
    return e1, [w[i] / kq for i in range(4)]


def external_current(p, h, basis_fn=None):
    """(eps^h(k))* = (e1 - i h e2)/sqrt(2); h is an array of +-1."""
    e1, e2 = (basis_fn or basis)(p)
    ih = 1j * np.asarray(h, dtype=np.float64)
    inv = 1 / sqrt2(p[0])
    return [(e1[i] - ih * e2[i]) * inv for i in range(4)]


def projector(p, kref):
    """P_{mu nu}(p, kref) with both indices up (4x4 nested list)."""
    g = [1.0, -1.0, -1.0, -1.0]
    pk = mdot(p, kref)
    return [[(-g[m] if m == n else 0.0) + (p[m] * kref[n] + p[n] * kref[m]) / pk
             for n in range(4)] for m in range(4)]
