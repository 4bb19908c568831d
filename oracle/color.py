"""Colour coefficients of the adjoint (DDM) decomposition (Section 2.2).

The amplitude is decomposed as (eq. color_decomposition_adjoint)
    A_{a1..an} = sum_{sigma in S_{n-2}} (F^{a_sigma2} ... F^{a_sigma(n-1)})_{a1 an}
                 A(1, sigma, n),   F^a_bc = i f^abc,
and the colour sum gives the matrix (eq. color_coefficient_adjoint)
    C_{sigma sigma'} = sum_a (F..F)_{a1 an} (F..F)*_{a1 an}.
Generators are normalised as Tr(T^a T^b) = delta^ab (the Dixon convention the
paper adopts in Section 2.3), so i f^abc reads i f~^abc with
f~^abc = -i Tr([T^a, T^b] T^c), i.e. F^a_bc = Tr([T^a, T^b] T^c).  This is the
only normalisation under which the projection identity of Section 2.3
(F^a_bc T^a_ij T^b_kl T^c_mn = d_il d_kn d_mj - d_in d_kj d_ml) holds.

Two independent evaluations are given:
  * ``color_matrix_gellmann``: the definition above with explicit 8x8
    matrices built from the Gell-Mann matrices (brute force, n <= 6);
  * ``color_matrix``: exact integers.  Contracting the F-chain with
    completeness relations gives, up to a sign common to all sigma,
    c_sigma(a) = Tr(T^a1 [T^s2, [T^s3, ..., [T^s(n-1), T^an]...]]).
    The nested commutator expands into 2^(n-2) signed trace words; each pair
    of words contributes N^(number of index loops) under the U(N) Fierz
    identity sum_a T^a_ij T^a_kl = d_il d_jk.  The U(1) generator drops out
    because every gluon sits inside a commutator or against a traceless one.
"""
import functools
import itertools

import numpy as np

NC = 3


def _nested_commutator_words(middle, last):
    """Signed words of [m1, [m2, ..., [mk, last]...]] as (sign, tuple)."""
    words = [(1, (last,))]
    for x in reversed(middle):
        nxt = []
        for s, w in words:
            nxt.append((s, (x,) + w))
            nxt.append((-s, w + (x,)))
        words = nxt
    return words


def coefficient_words(n, sigma):
    """Trace words of c_sigma: list of (sign, word), each word starts with gluon 0."""
    return [(s, (0,) + w) for s, w in _nested_commutator_words(list(sigma), n - 1)]


def _loops(w, v):
    """Index loops of sum_a Tr(T^{w}) Tr(T^{v}) with the U(N) Fierz identity."""
    n = len(w)
    parent = list(range(2 * n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    def union(x, y):
        rx, ry = find(x), find(y)
        if rx != ry:
            parent[rx] = ry

    pos_v = {g: q for q, g in enumerate(v)}
    for p, g in enumerate(w):
        q = pos_v[g]
        # T^g_{i_p i_(p+1)} T^g_{j_q j_(q+1)} -> d(i_p, j_(q+1)) d(i_(p+1), j_q)
        union(p, n + (q + 1) % n)
        union((p + 1) % n, n + q)
    return len({find(x) for x in range(2 * n)})


def color_entry(n, sigma, sigma_p, nc=NC):
    """Exact integer C_{sigma sigma'}."""
    total = 0
    for s1, w1 in coefficient_words(n, sigma):
        for s2, w2 in coefficient_words(n, sigma_p):
            # conjugate trace: Tr(X)* = Tr(X^dagger) = trace of the reversed word
            total += s1 * s2 * nc ** _loops(w1, tuple(reversed(w2)))
    return total


def middle_permutations(n):
    return list(itertools.permutations(range(1, n - 1)))


def color_matrix(n, nc=NC, relabel=None):
    """Exact C(n) as an int64 array [K, K], K = (n-2)!, lexicographic sigma.

    With relabel (default for n >= 7) only the first row is evaluated and the
    rest follows from renaming the summed colour labels of gluons 2..n-1:
    C_{sigma sigma'} = C_{id, pi(sigma')} with pi the label map taking sigma
    to the identity.  The direct and relabelled forms are compared in the
    tests for n <= 6.
    """
    perms = middle_permutations(n)
    K = len(perms)
    if relabel is None:
        relabel = n >= 7
    C = np.zeros((K, K), dtype=np.int64)
    if not relabel:
        for i in range(K):
            for j in range(i, K):
                C[i, j] = C[j, i] = color_entry(n, perms[i], perms[j], nc)
        return C
    ident = perms[0]
    return color_matrix_from_row0(n, [color_entry(n, ident, p, nc) for p in perms])


def color_matrix_from_row0(n, row0):
    """C(n) [K, K] from its first row (sigma = identity), by renaming the
    summed colour labels: C_{sigma sigma'} = C_{id, pi(sigma')} with pi the
    label map taking sigma to the identity."""
    perms = middle_permutations(n)
    ident = perms[0]
    row = {p: int(v) for p, v in zip(perms, row0)}
    C = np.zeros((len(perms), len(perms)), dtype=np.int64)
    for i, s in enumerate(perms):
        pi = {lab: ident[pos] for pos, lab in enumerate(s)}
        for j, t in enumerate(perms):
            C[i, j] = row[tuple(pi[x] for x in t)]
    return C


@functools.lru_cache(maxsize=None)
def _color_matrix_cached(n, nc):
    C = color_matrix(n, nc)
    C.setflags(write=False)
    return C


def color_matrix_cached(n, nc=NC):
    """Read-only C(n), computed once per process."""
    return _color_matrix_cached(n, nc)


def gellmann_generators():
    """T^a = lambda^a / sqrt(2), so that Tr(T^a T^b) = delta^ab."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / np.sqrt(2.0)


def adjoint_F():
    """F[a, b, c] = Tr([T^a, T^b] T^c) = i f~^abc."""
    T = gellmann_generators()
    comm = np.einsum("aij,bjk->abik", T, T) - np.einsum("bij,ajk->abik", T, T)
    return np.einsum("abij,cji->abc", comm, T)


def color_row_gellmann(n, row=0):
    """Row `row` of C(n) from the definition with explicit F matrices (float).

    Only two colour chains are held at a time (8^n entries each), so this
    reaches n = 7 where the full brute-force matrix would not fit."""
    F = adjoint_F()
    perms = middle_permutations(n)
    k = n - 2

    def chain(sigma):
        M = None
        for gl in sigma:
            Fb = np.moveaxis(F.reshape((8,) + (1,) * (k - 1) + (8, 8)), 0, gl - 1)
            M = Fb if M is None else np.einsum("...ij,...jk->...ik", M, Fb)
        return M

    ref = chain(perms[row])
    out = np.zeros(len(perms))
    for j, sigma in enumerate(perms):
        out[j] = np.real(np.sum(ref * np.conj(chain(sigma))))
    return out


def color_entry_gellmann(n, i, j):
    """C(n)[i, j] from the definition with explicit F matrices (float), two
    colour chains of 8^n entries: an entry check where a whole row would be
    too slow (n = 8: 16.8 M complex entries per chain)."""
    F = adjoint_F()
    perms = middle_permutations(n)
    k = n - 2

    def chain(sigma):
        M = None
        for gl in sigma:
            Fb = np.moveaxis(F.reshape((8,) + (1,) * (k - 1) + (8, 8)), 0, gl - 1)
            M = Fb if M is None else np.einsum("...ij,...jk->...ik", M, Fb)
        return M

    return float(np.real(np.sum(chain(perms[i]) * np.conj(chain(perms[j])))))


def color_matrix_gellmann(n):
    """C(n) from its definition with explicit F matrices (float, n <= 6)."""
    F = adjoint_F()
    perms = middle_permutations(n)
    k = n - 2
    chains = []
    for sigma in perms:
        # M[a_2, ..., a_{n-1}, a1, an] = (F^{a_s2} ... F^{a_s(n-1)})_{a1 an}
        # sigma lists which gluon's colour index sits in each chain slot.
        M = None
        for gl in sigma:
            Fg = F  # indexed [colour of gluon gl, row, column]
            if M is None:
                M = Fg.reshape((8,) + (1,) * (k - 1) + (8, 8))
                M = np.moveaxis(M, 0, gl - 1)
            else:
                # contract column of M with row of F^{a_gl}
                Fb = np.moveaxis(Fg.reshape((8,) + (1,) * (k - 1) + (8, 8)), 0, gl - 1)
                M = np.einsum("...ij,...jk->...ik", M, Fb)
        chains.append(M.reshape(-1, 8, 8) if M.ndim > 2 else M)
    K = len(perms)
    C = np.zeros((K, K))
    for i in range(K):
        for j in range(K):
            C[i, j] = np.real(np.sum(chains[i] * np.conj(chains[j])))
    return C
