"""Colour-ordered Berends-Giele recursion (Section 2.3).

Off-shell current of an ordered range of gluons (eq. cobg):
    J(1..n) = (-i / p_{1,n}^2) { sum_k V3(p_{1,k}, p_{k+1,n}) J(1..k) J(k+1..n)
                                 + sum_{j<k} V4 J(1..j) J(j+1..k) J(k+1..n) }
with the colour-ordered vertices
    V3^{nu kappa lambda}(p, q) = i g/sqrt2 (g^{kl}(p-q)^nu + g^{l nu}(2q+p)^k
                                             - g^{nu k}(2p+q)^l),
    V4^{nu rho kappa lambda}   = i g^2/2 (2 g^{nu k} g^{rho l} - g^{nu rho} g^{kl}
                                          - g^{nu l} g^{rho k}),
external currents equal to the polarization vectors, and the amplitude
(eq. cobg_full_amplitude) obtained by putting J(1..n-1) on shell and
contracting with the polarization of gluon n.  The printed factor
"p^2_{1,n}" vanishes by momentum conservation; the reading taken here is the
inverse propagator of J(1..n-1), so the amplitude is eps_n . (p^2 J(1..n-1)),
i.e. the bracket of J(1..n-1) times -i without the 1/p^2.

The tensor form (eq. prop_pseudo, cobg_tensor, cobg_tensor_current,
cobg_tensor_vertex) replaces V4 by an antisymmetric auxiliary current; it is
implemented separately and must agree with the explicit-V4 recursion.

Gluons are referred to by 0-based position in the momentum array; an ordering
is a tuple of such indices.  The DDM basis orderings are (0, sigma, n-1) with
sigma running over permutations of 1..n-2 in lexicographic order.
"""
import itertools
import math

import numpy as np

from .lorentz import mdot
from .numeric import coupling, sqrt2
from .polarization import external_current

ALPHA_S = 0.118
G_S = math.sqrt(4.0 * math.pi * ALPHA_S)   # FP64 value; see ``numeric.coupling``


def _v3(p, q, ja, jb, g):
    """V3^{nu kappa lambda}(p, q) ja_kappa jb_lambda (paper's vertex, with i g/sqrt2)."""
    c = 1j * (g / sqrt2(g))
    ab = mdot(ja, jb)
    qa = mdot([2.0 * q[i] + p[i] for i in range(4)], ja)
    pb = mdot([2.0 * p[i] + q[i] for i in range(4)], jb)
    return [c * (ab * (p[i] - q[i]) + qa * jb[i] - pb * ja[i]) for i in range(4)]


def _v4(j1, j2, j3, g):
    """V4^{nu rho kappa lambda} j1_rho j2_kappa j3_lambda (with i g^2/2)."""
    c = 1j * (g * g / 2)
    d13 = mdot(j1, j3)
    d12 = mdot(j1, j2)
    d23 = mdot(j2, j3)
    return [c * (2.0 * d13 * j2[i] - d23 * j1[i] - d12 * j3[i]) for i in range(4)]


def range_momenta(ps, order):
    """P[(a, b)] = sum of momenta of order[a..b] (inclusive)."""
    m = len(order)
    P = {}
    for a in range(m):
        acc = list(ps[order[a]])
        P[(a, a)] = acc
        for b in range(a + 1, m):
            acc = [acc[i] + ps[order[b]][i] for i in range(4)]
            P[(a, b)] = acc
    return P


def currents(ps, eps, order, g=None, amputate_top=False):
    """All range currents J[(a, b)] of the ordered gluons ``order`` (eq. cobg).

    ps[i]: momentum (list of 4 arrays) of gluon i; eps[i]: its external current.
    With amputate_top the full range carries p^2 J instead of J.
    """
    m = len(order)
    if g is None:
        g = coupling(ps[0][0])
    P = range_momenta(ps, order)
    J = {}
    for a in range(m):
        J[(a, a)] = eps[order[a]]
    for length in range(2, m + 1):
        for a in range(0, m - length + 1):
            b = a + length - 1
            acc = [0.0, 0.0, 0.0, 0.0]
            for k in range(a, b):
                t = _v3(P[(a, k)], P[(k + 1, b)], J[(a, k)], J[(k + 1, b)], g)
                acc = [acc[i] + t[i] for i in range(4)]
            for j in range(a, b):
                for k in range(j + 1, b):
                    t = _v4(J[(a, j)], J[(j + 1, k)], J[(k + 1, b)], g)
                    acc = [acc[i] + t[i] for i in range(4)]
            if amputate_top and length == m:
                J[(a, b)] = [-1j * acc[i] for i in range(4)]
            else:
                p2 = mdot(P[(a, b)], P[(a, b)])
                J[(a, b)] = [(-1j / p2) * acc[i] for i in range(4)]
    return J


def _vt_jj(ja, jb, g):
    """V_T^{gamma delta kappa lambda} ja_kappa jb_lambda, both tensor indices up."""
    c = 0.5j * (g / sqrt2(g))
    return [[c * (ja[x] * jb[y] - ja[y] * jb[x]) for y in range(4)] for x in range(4)]


def _metric(i):
    return 1.0 if i == 0 else -1.0


def _vt_jt(j, t, g):
    """V_T^{nu kappa alpha beta} j_kappa T_{alpha beta} (gluon left of tensor)."""
    c = 0.5j * (g / sqrt2(g))
    out = []
    for nu in range(4):
        s1 = 0.0
        s2 = 0.0
        for b in range(4):
            s1 = s1 + t[nu][b] * (_metric(b) * j[b])   # T^{nu beta} j_beta
            s2 = s2 + (_metric(b) * j[b]) * t[b][nu]   # j_alpha T^{alpha nu}
        out.append(c * (s1 - s2))
    return out


def _vt_tj(t, j, g):
    """V_T^{lambda nu alpha beta} T_{alpha beta} j_lambda (tensor left of gluon)."""
    c = 0.5j * (g / sqrt2(g))
    out = []
    for nu in range(4):
        s1 = 0.0
        s2 = 0.0
        for a in range(4):
            s1 = s1 + (_metric(a) * j[a]) * t[a][nu]   # j_alpha T^{alpha nu}
            s2 = s2 + t[nu][a] * (_metric(a) * j[a])   # T^{nu beta} j_beta
        out.append(c * (s1 - s2))
    return out


def _prop_tensor(x):
    """-i D^{alpha beta}_{gamma delta} X^{gamma delta} (eq. prop_pseudo)."""
    return [[-1j * (x[a][b] - x[b][a]) for b in range(4)] for a in range(4)]


def currents_tensor(ps, eps, order, g=None, amputate_top=False):
    """Range currents from the tensor form (eqs. cobg_tensor, cobg_tensor_current)."""
    m = len(order)
    if g is None:
        g = coupling(ps[0][0])
    P = range_momenta(ps, order)
    J = {}
    T = {}
    zero_t = [[0.0] * 4 for _ in range(4)]
    for a in range(m):
        J[(a, a)] = eps[order[a]]
        T[(a, a)] = zero_t
    for length in range(2, m + 1):
        for a in range(0, m - length + 1):
            b = a + length - 1
            acc = [0.0, 0.0, 0.0, 0.0]
            tacc = [[0.0] * 4 for _ in range(4)]
            for k in range(a, b):
                jl, jr = J[(a, k)], J[(k + 1, b)]
                t3 = _v3(P[(a, k)], P[(k + 1, b)], jl, jr, g)
                t1 = _vt_jt(jl, T[(k + 1, b)], g)
                t2 = _vt_tj(T[(a, k)], jr, g)
                acc = [acc[i] + t3[i] + t1[i] + t2[i] for i in range(4)]
                x = _vt_jj(jl, jr, g)
                tacc = [[tacc[u][v] + x[u][v] for v in range(4)] for u in range(4)]
            T[(a, b)] = _prop_tensor(tacc)
            if amputate_top and length == m:
                J[(a, b)] = [-1j * acc[i] for i in range(4)]
            else:
                p2 = mdot(P[(a, b)], P[(a, b)])
                J[(a, b)] = [(-1j / p2) * acc[i] for i in range(4)]
    return J


def momenta_list(mom):
    """mom [n][4][E] -> list of n four-vectors (lists of arrays)."""
    return [[mom[i, mu] for mu in range(4)] for i in range(mom.shape[0])]


def external_currents(ps, hel):
    """hel [n][E] (or [n] of scalars) -> list of external currents."""
    return [external_current(ps[i], hel[i]) for i in range(len(ps))]


def ordered_amplitude(ps, eps, order, g=None, tensor=False):
    """A(order) = eps_last . (p^2 J(order[:-1])) (eq. cobg_full_amplitude)."""
    f = currents_tensor if tensor else currents
    J = f(ps, eps, order[:-1], g=g, amputate_top=True)
    top = J[(0, len(order) - 2)]
    return mdot(eps[order[-1]], top)


def ddm_orderings(n):
    """(0, sigma, n-1) for sigma in permutations of 1..n-2, lexicographic."""
    return [(0,) + s + (n - 1,) for s in itertools.permutations(range(1, n - 1))]


def partial_amplitudes(mom, hel, g=None, tensor=False):
    """A_sigma for the (n-2)! DDM orderings: complex array [K, E].

    mom: [n][4][E] float64 (or long double / mpmath objects: the evaluation
    runs in that precision); hel: [n][E] of +-1 (or [n] scalars).
    """
    n = mom.shape[0]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    amps = [ordered_amplitude(ps, eps, o, g=g, tensor=tensor) for o in ddm_orderings(n)]
    return np.array([np.broadcast_to(a, mom.shape[2:]) for a in amps])


def amplitude_of(mom, hel, order, g=None):
    """A(order) for an arbitrary ordering of all n gluons: complex array [E]."""
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    return ordered_amplitude(ps, eps, tuple(order), g=g)
