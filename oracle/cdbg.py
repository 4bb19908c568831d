"""Colour-dressed Berends-Giele recursion in the colour-flow basis (Section 2.3).

Colour-flow amplitude for one assignment (i_k, j_k) per gluon
(eq. color_decomposition_colorflow):
    A_{i1 j1 .. in jn} = sum_{sigma in S_(n-1)} d(i1, j_s2) d(i_s2, j_s3) ...
                         d(i_sn, j1) A(1, s2, ..., sn).
With the 3x3 unit matrices E_k = e_{j_k i_k} (row j_k, column i_k) the chain
of deltas is Tr(E_1 E_s2 ... E_sn); ``flow_amplitude_bruteforce`` evaluates
this sum literally from colour-ordered amplitudes.

Colour-dressed currents (eq. cdcurrents) are 3x3 matrices of currents,
    J(S) = sum over orderings s of S of  E_s1 E_s2 ... E_sk  J(s1..sk),
(likewise the tensor currents).  Inserting the colour-ordered recursion of
eq. cobg (or its tensor form eq. cobg_tensor) into this definition gives the
recursion over partitions of eq. color_dressed_currents:
    J(S) = -i/P_S^2 { sum_{ordered (S1,S2)} V3(P1, P2) [J(S1) J(S2)]
                      + V_T [J(S1) T(S2)] + V_T [T(S1) J(S2)] }
    T(S) = -i D sum_{ordered (S1,S2)} V_T [J(S1) J(S2)]
where [X Y] is the 3x3 colour-matrix product and the kinematic part is the
colour-ordered vertex with X to the left of Y.  Reading: the paper's dressed
vertices pair the colour product with the opposite kinematic order; that is
the same recursion for the transposed colour chain and changes A only by a
sign common to all terms, so |A|^2 is unaffected.  The variant with the
explicit four-gluon vertex sums V4 over ordered 3-partitions instead of the
tensor terms.  The amplitude is
    A = eps_n . (P^2 J(1..n-1))_{i_n j_n}    (since Tr(M E_n) = M_{i_n j_n}).
Arrays: a dressed current is complex [3, 3, 4, E]; a tensor [3, 3, 4, 4, E].
"""
import itertools
import math

import numpy as np

from .cobg import G_S, momenta_list, external_currents, ordered_amplitude
from .lorentz import mdot
from .numeric import complex_type, coupling, sqrt2

_G = np.array([1.0, -1.0, -1.0, -1.0])


def _mdot_vec(p, J):
    """p.J[..., mu, E] for a real four-vector p (list of arrays)."""
    return sum(_G[m] * p[m] * J[..., m, :] for m in range(4))


def _v3_dressed(P1, P2, J1, J2, g):
    """sum_k V3(P1,P2; J1[i,k], J2[k,j]) including i g/sqrt2: [3,3,4,E]."""
    c = 1j * (g / sqrt2(g))
    ab = np.einsum("ikme,kjme,m->ije", J1, J2, _G)
    q = [2.0 * P2[m] + P1[m] for m in range(4)]
    p = [2.0 * P1[m] + P2[m] for m in range(4)]
    qa = _mdot_vec(q, J1)  # [3,3,E]
    pb = _mdot_vec(p, J2)
    diff = np.array([P1[m] - P2[m] for m in range(4)])  # [4,E]
    out = ab[:, :, None, :] * diff[None, None]
    out = out + np.einsum("ike,kjme->ijme", qa, J2) - np.einsum("ikme,kje->ijme", J1, pb)
    return c * out


def _v4_dressed(J1, J2, J3, g):
    """sum V4(J1[i,k], J2[k,l], J3[l,j]) including i g^2/2."""
    c = 1j * (g * g / 2)
    d12 = np.einsum("ikme,klme,m->ile", J1, J2, _G)
    d23 = np.einsum("klme,ljme,m->kje", J2, J3, _G)
    # 2 (J1.J3) J2 - (J2.J3) J1 - (J1.J2) J3
    t1 = 2.0 * np.einsum("ikme,ljme,m,klne->ijne", J1, J3, _G, J2)
    t2 = np.einsum("ikne,kje->ijne", J1, d23)
    t3 = np.einsum("ile,ljne->ijne", d12, J3)
    return c * (t1 - t2 - t3)


def _vt_jj(J1, J2, g):
    """V_T[J1 J2] with both tensor indices up: [3,3,4,4,E]."""
    c = 0.5j * (g / sqrt2(g))
    x = np.einsum("ikae,kjbe->ijabe", J1, J2)
    return c * (x - np.swapaxes(x, 2, 3))


def _vt_jt(J, T, g):
    """V_T^{nu kappa alpha beta} J_kappa T_alpha_beta with colour [J T]."""
    c = 0.5j * (g / sqrt2(g))
    s1 = np.einsum("ikbe,kjnbe,b->ijne", J, T, _G)  # T^{nu b} J_b
    s2 = np.einsum("ikae,kjane,a->ijne", J, T, _G)  # J_a T^{a nu}
    return c * (s1 - s2)


def _vt_tj(T, J, g):
    """V_T^{lambda nu alpha beta} T_alpha_beta J_lambda with colour [T J]."""
    c = 0.5j * (g / sqrt2(g))
    s1 = np.einsum("ikane,kjae,a->ijne", T, J, _G)  # J_a T^{a nu}
    s2 = np.einsum("iknbe,kjbe,b->ijne", T, J, _G)  # T^{nu b} J_b
    return c * (s1 - s2)


def _submasks(mask):
    """Non-empty proper submasks of mask."""
    s = (mask - 1) & mask
    while s:
        yield s
        s = (s - 1) & mask


def _flow_matrix(i_k, j_k, E):
    """E_k = e_{j_k i_k} per event: [3,3,E] float."""
    M = np.zeros((3, 3, E))
    ev = np.arange(E)
    M[j_k, i_k, ev] = 1.0
    return M


def dressed_recursion(ps, eps, colmats, g=None, tensor=True):
    """Dressed currents of all subsets of gluons 1..n-1 (0-based 0..n-2) for
    external currents eps[k] [4,E] and external colour matrices colmats[k]
    [3,3,E] (a colour-flow assignment, or any other colour wavefunction).

    Returns dict mask -> J [3,3,4,E]; the full mask holds P^2 J (amputated).
    """
    m = len(ps) - 1
    E = np.shape(ps[0][0])[-1]
    if g is None:
        g = coupling(ps[0][0])
    ct = complex_type(ps[0][0])
    J, T, P = {}, {}, {}
    for k in range(m):
        mk = 1 << k
        e = np.array(eps[k])  # [4,E]
        J[mk] = colmats[k][:, :, None, :] * e[None, None]
        T[mk] = np.zeros((3, 3, 4, 4, E), dtype=ct)
        P[mk] = ps[k]
    full = (1 << m) - 1
    for size in range(2, m + 1):
        for bits in itertools.combinations(range(m), size):
            S = sum(1 << b for b in bits)
            P[S] = [sum(ps[b][mu] for b in bits) for mu in range(4)]
            acc = np.zeros((3, 3, 4, E), dtype=ct)
            tacc = np.zeros((3, 3, 4, 4, E), dtype=ct)
            for A in _submasks(S):
                B = S ^ A
                acc = acc + _v3_dressed(P[A], P[B], J[A], J[B], g)
                if tensor:
                    acc = acc + _vt_jt(J[A], T[B], g) + _vt_tj(T[A], J[B], g)
                    tacc = tacc + _vt_jj(J[A], J[B], g)
            if not tensor:
                for A in _submasks(S):
                    rest = S ^ A
                    for B in _submasks(rest):
                        Cm = rest ^ B
                        acc = acc + _v4_dressed(J[A], J[B], J[Cm], g)
            if tensor:
                T[S] = -1j * (tacc - np.swapaxes(tacc, 2, 3))
            if S == full:
                J[S] = -1j * acc
            else:
                p2 = mdot(P[S], P[S])
                J[S] = (-1j / p2) * acc
    return J


def dressed_currents(mom, hel, col, g=None, tensor=True):
    """Dressed currents for helicity labels hel [n][E] and the colour-flow
    assignment col [2][n][E] (see dressed_recursion)."""
    n = mom.shape[0]
    E = mom.shape[2]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    colmats = [_flow_matrix(col[0, k], col[1, k], E) for k in range(n - 1)]
    return dressed_recursion(ps, eps, colmats, g=g, tensor=tensor)


def flow_amplitude(mom, hel, col, g=None, tensor=True):
    """Colour-flow amplitude from the dressed recursion: complex [E]."""
    n = mom.shape[0]
    E = mom.shape[2]
    Jd = dressed_currents(mom, hel, col, g=g, tensor=tensor)
    top = Jd[(1 << (n - 1)) - 1]  # [3,3,4,E]
    ev = np.arange(E)
    sel = top[col[0, n - 1], col[1, n - 1], :, ev].T  # [4,E]
    ps = momenta_list(mom)
    en = external_currents(ps, hel)[n - 1]
    return mdot(en, [sel[mu] for mu in range(4)])


def chain_weight(col, order):
    """Tr(E_o1 E_o2 ... E_on) per event (0 or 1): the delta chain of the ordering."""
    i, j = col[0], col[1]
    w = np.ones(col.shape[2])
    L = len(order)
    for a in range(L):
        w = w * (i[order[a]] == j[order[(a + 1) % L]])
    return w


def flow_amplitude_bruteforce(mom, hel, col, g=None):
    """sum over orderings (1, s) with s in S_(n-1) of chain weight x A(1, s)."""
    n = mom.shape[0]
    ps = momenta_list(mom)
    eps = external_currents(ps, hel)
    out = np.zeros(mom.shape[2], dtype=complex_type(mom))
    for s in itertools.permutations(range(1, n)):
        order = (0,) + s
        w = chain_weight(col, order)
        if not w.any():
            continue
        out = out + w * ordered_amplitude(ps, eps, order, g=g)
    return out


def is_valid_flow(col):
    """True where some ordering has a closed colour chain (the amplitude can be non-zero)."""
    n = col.shape[1]
    ok = np.zeros(col.shape[2], dtype=bool)
    for s in itertools.permutations(range(1, n)):
        ok |= chain_weight(col, (0,) + s) > 0
    return ok
