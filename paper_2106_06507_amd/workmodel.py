"""Algorithmic work and traffic per event, used for roofline fractions.

Flop constants are the real floating-point operations of the vertex formulas
as written (a fused multiply-add counts 2, a complex product 6 = 4 mul + 2 add):
  V3(P,Q;A,B) = (A.B)(P-Q) + ((2Q+P).A)B - ((2P+Q).B)A        166
  V4(J1,J2,J3) = 2(J1.J3)J2 - (J2.J3)J1 - (J1.J2)J3            188
  propagator (complex current times real 1/P^2)                   8
  range momentum (four additions)                                 4
  final contraction with the last polarization (+ coupling)      32
Colour contraction x^T C x + y^T C y with K orderings:     4K^2 + 4K
  (the fused kernel uses the symmetry of C: 2K(K+1) + 4K)
The colour-ordered recursion walks the orderings depth first and shares
prefixes: column d (ranges ending at position d) is evaluated once per
distinct prefix of length d+1, i.e. (n-2)!/(n-2-d)! times.
"""
import math

import numpy as np

FLOP_V3 = 166
FLOP_V4 = 188
FLOP_PROP = 8
FLOP_PMOM = 4
FLOP_TOP = 32


def cobg_vertex_counts(n):
    """(V3, V4, propagators, range momenta, tops) evaluated per event and helicity."""
    M = n - 1
    v3 = v4 = prop = pm = top = 0
    for d in range(1, M):
        times = math.factorial(n - 2) // math.factorial(n - 2 - d)
        for a in range(d - 1, -1, -1):
            L = d - a + 1
            v3 += times * (L - 1)
            v4 += times * ((L - 1) * (L - 2) // 2)
            pm += times
            if a == 0 and d == M - 1:
                top += times
            else:
                prop += times
    return v3, v4, prop, pm, top


def cobg_flops_per_event(n):
    v3, v4, prop, pm, top = cobg_vertex_counts(n)
    return v3 * FLOP_V3 + v4 * FLOP_V4 + prop * FLOP_PROP + pm * FLOP_PMOM + top * FLOP_TOP


def contraction_flops_per_event(n):
    K = math.factorial(n - 2)
    return 4 * K * K + 4 * K


def colour_sum_flops_per_event(n):
    """FP64 flops of the fused colour sum x^T C x + y^T C y using the symmetry
    of C: K(K+1)/2 multiply-adds for the triangle and K for the outer
    products, per plane."""
    K = math.factorial(n - 2)
    return 2 * 2 * (K * (K + 1) // 2 + K)


def continuous_flops_per_event(n):
    """Real flops of the continuous-colour dressed recursion per event, from
    the formulas as written, summed over every subset S of gluons 1..n-1
    with |S| >= 2 and every ordered split (A, B) of S:
      per split: (2P_B + P_A), (2P_A + P_B), P_A - P_B            20
      per split and colour entry (nine entries):
        V3 with the 3x3 colour product (3 + 6 Minkowski dots,
          the two k-sums and the (P_A - P_B) term)              121
        J(A) T(B) term when |B| >= 2                              72
        T(A) J(B) term when |A| >= 2                              72
        tensor current of S (six components) unless S is full     72
      per subset and entry: times 1/P^2 (4); at the full set the
      contraction with e_n and the two colour vectors (10)."""
    m = n - 1
    full = (1 << m) - 1
    total = 0
    for S in range(1, full + 1):
        if bin(S).count("1") < 2:
            continue
        A = (S - 1) & S
        while A:
            B = S ^ A
            per = 121 + (72 if bin(B).count("1") >= 2 else 0) + (72 if bin(A).count("1") >= 2 else 0)
            per += 72 if S != full else 0
            total += 20 + 9 * per
            A = (A - 1) & S
        total += 9 * (10 if S == full else 4)
    return total


def cobg_bytes_per_event(n, amp_out=True):
    """HBM bytes of the recursion kernel: momenta and helicities in, amplitudes out."""
    K = math.factorial(n - 2)
    return n * 4 * 8 + n * 1 + (2 * K * 8 if amp_out else 0)


def contraction_bytes_per_event(n):
    K = math.factorial(n - 2)
    return 2 * K * 8 + 8


# Published MI355X peaks (dense, no sparsity)
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_FP32_VALU_TFLOPS = 157.3
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: FP32 without packed
# (two-wide) instructions, the same rate as FP64
PEAK_FP32_VALU_NOPK_TFLOPS = 78.6
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


# Colour-dressed recursion (Section 2.3, eq. color_dressed_currents in the
# tensor form).  A dressed current of subset S is a 3x3 colour matrix with at
# most three non-zero entries (the colour-flow chains of eq.
# color_decomposition_colorflow through S's edges); a split (S1, S2)
# contributes to entry (r, c) of S iff J(S1)_{r k} J(S2)_{k c} != 0 for some
# k.  Per contributing (target entry, split) the formulas as written cost:
#   V3(P1, P2; J1, J2)                                         166
#   tensor couplings T2.J1 and T1.J2 (12 complex x real
#     products with a sign each, twice)                        2 x 120
#   the tensor current J1^a J2^b - J1^b J2^a (six components,
#     four complex products each), not at the full set          96
# and per target entry: times 1/P^2 (8); at the full set the contraction
# with the last polarization (32).
FLOP_CD_SPLIT = 166 + 240
FLOP_CD_TENSOR = 96


def _dressed_entries(i, j, S, M):
    """Non-zero colour entries of the dressed current of subset S for the
    colour labels i, j [M, E] of gluons 0..M-1: a list over (r, c) of
    boolean arrays [E].  Entry (r, c) is non-zero iff S's edges j_k -> i_k
    form one trail from r to c (all edges used once): connected, and out-in
    degrees +1 at r, -1 at c, 0 elsewhere (or all 0 with r = c touched)."""
    E = i.shape[1]
    deg = np.zeros((3, E), dtype=np.int64)
    touched = np.zeros((3, E), dtype=bool)
    parent = np.tile(np.arange(3)[:, None], (1, E))

    def find(a):
        # a [E] colour index per event
        for _ in range(3):
            a = parent[a, np.arange(E)]
        return a

    for k in range(M):
        if not (S >> k) & 1:
            continue
        for v in range(3):
            deg[v] += (j[k] == v).astype(np.int64) - (i[k] == v).astype(np.int64)
            touched[v] |= (j[k] == v) | (i[k] == v)
        ra, rb = find(j[k]), find(i[k])
        parent[ra, np.arange(E)] = rb
    roots = [find(np.full(E, v)) for v in range(3)]
    conn = np.ones(E, dtype=bool)
    for a in range(3):
        for b in range(3):
            conn &= ~(touched[a] & touched[b]) | (roots[a] == roots[b])
    balanced = np.all(deg == 0, axis=0)
    out = {}
    for r in range(3):
        for c in range(3):
            if r == c:
                ok = balanced & touched[r]
            else:
                ok = (deg[r] == 1) & (deg[c] == -1) & (np.sum(np.abs(deg), axis=0) == 2)
            out[(r, c)] = ok & conn
    return out


def cdbg_flops_per_event(col):
    """Algorithmic flops of the colour-dressed recursion for each event of
    col [2][n][E] (colour labels i_k = col[0][k], j_k = col[1][k]): the sum
    over subsets S of gluons 0..n-2 (|S| >= 2), over their non-zero colour
    entries and over the unordered splits {S1, S2} of S whose colour
    commutator reaches that entry, of the per-split costs above.  The
    kinematic part of a split changes sign when its operands are exchanged,
    so its two orders take one evaluation, and a split of two balanced
    subsets (diagonal currents, which commute) costs nothing.  Events whose
    flow does not close (no closed chain of all n edges) cost 0: they are
    classified and skip the recursion."""
    n, E = col.shape[1], col.shape[2]
    M = n - 1
    i, j = col[0].astype(np.int64), col[1].astype(np.int64)
    full = (1 << M) - 1
    ent = {S: _dressed_entries(i, j, S, M) for S in range(1, full + 1)}
    flops = np.zeros(E)
    # the amplitude needs entry (i_n, j_n) of the full set
    last_r, last_c = col[0][n - 1], col[1][n - 1]
    for S in range(1, full + 1):
        if bin(S).count("1") < 2:
            continue
        targets = ent[S]
        for (r, c), okS in targets.items():
            if S == full:
                okS = okS & (last_r == r) & (last_c == c)
            if not okS.any():
                continue
            nsplit = np.zeros(E)
            top = 1 << (S.bit_length() - 1)
            A = (S - 1) & S
            while A:
                if not A & top:  # each unordered split once
                    B = S ^ A
                    e1, e2 = ent[A], ent[B]
                    hit = np.zeros(E, dtype=bool)
                    for k in range(3):
                        hit |= (e1[(r, k)] & e2[(k, c)]) | (e2[(r, k)] & e1[(k, c)])
                    bal1 = e1[(0, 0)] | e1[(1, 1)] | e1[(2, 2)]
                    bal2 = e2[(0, 0)] | e2[(1, 1)] | e2[(2, 2)]
                    nsplit += hit & ~(bal1 & bal2)
                A = (A - 1) & S
            per = FLOP_CD_SPLIT + (0 if S == full else FLOP_CD_TENSOR)
            flops += okS * (nsplit * per + (32 if S == full else 8))
    closed = _dressed_entries(col[0].astype(np.int64), col[1].astype(np.int64), (1 << n) - 1, n)
    valid = closed[(0, 0)] | closed[(1, 1)] | closed[(2, 2)]
    return flops * valid


def adjoint_flops_per_event(n):
    """Algorithmic flops of the gradient d|M|^2/dp (reverse mode, currents
    recomputed per ordering): the forward amplitudes (prefix-shared walk),
    Y = C A in FP64 (4 K^2), and per ordering one recomputation of its range
    currents plus a reverse sweep counted at twice the forward flops (the
    adjoint of a product needs one product per operand), i.e. 3x the
    unshared forward recursion of one ordering."""
    K = math.factorial(n - 2)
    M = n - 1
    v3 = sum((M - L + 1) * (L - 1) for L in range(2, M + 1))
    v4 = sum((M - L + 1) * (L - 1) * (L - 2) // 2 for L in range(2, M + 1))
    ranges = sum(M - L + 1 for L in range(2, M + 1))
    per_order = v3 * FLOP_V3 + v4 * FLOP_V4 + ranges * (FLOP_PROP + FLOP_PMOM) + FLOP_TOP
    return cobg_flops_per_event(n) + 4 * K * K + K * 3 * per_order
