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
