"""Small shared helpers for the tests (no matrix-element arithmetic)."""
import numpy as np


def mhv_helicities(n, E, rng):
    """Random helicities with exactly two minus signs per event: [n][E]."""
    h = np.ones((n, E), dtype=np.int8)
    for e in range(E):
        a, b = rng.choice(n, 2, replace=False)
        h[a, e] = -1
        h[b, e] = -1
    return h


def valid_colours(n, E, rng):
    """Colour-flow labels that close one chain through a random ordering: [2][n][E]."""
    col = np.zeros((2, n, E), dtype=np.int8)
    for e in range(E):
        perm = rng.permutation(n)
        ii = rng.integers(0, 3, n)
        for k in range(n):
            col[0, perm[k], e] = ii[k]
            col[1, perm[(k + 1) % n], e] = ii[k]
    return col


def mink(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def sij(mom, i, j):
    """2 p_i.p_j from the momentum array [n][4][E]."""
    return 2.0 * mink(mom[i], mom[j])


def nonvanishing(hel):
    """Events whose helicity configuration has a non-zero tree amplitude.

    All-equal and one-different configurations vanish identically at tree
    level (the oracle pins this), so both implementations return rounding
    noise there and a relative error is meaningless."""
    m = np.sum(np.asarray(hel) < 0, axis=0)
    n = np.asarray(hel).shape[0]
    return (m >= 2) & (m <= n - 2)


def amplitude_scale(n, sqrt_s=1000.0):
    """Natural size g'^(n-2) sqrt(s)^(4-n) of an n-gluon tree amplitude."""
    g = (4 * np.pi * 0.118) ** 0.5 / 2 ** 0.5
    return g ** (n - 2) * sqrt_s ** (4 - n)


def helicity_scale(mom):
    """Helicity-averaged colour-summed |M|^2 per event from the oracle: the
    natural scale of the sampled estimator 2^n |M|^2_h (its mean is the
    helicity sum).  Used to state errors of sampled configurations whose own
    |M|^2 is suppressed by many orders of magnitude."""
    from oracle import me2 as ome2
    return ome2.me2_cobg(mom, None) / 2 ** mom.shape[0]


U64 = 2.0 ** -53


def fp64_allowance(n, ref, mag):
    """Per-event bar of an FP64 evaluation against the extended reference:
    max(1e-12 |ref|, 12 (n - 2) u m), m the magnitude of the evaluation (every
    product and sum taken in modulus, oracle.conditioning).  12 (n - 2) is
    the number of roundings along the deepest path of the recursion (at most
    n - 2 levels, each a four-term dot product, a scaling and an accumulation
    over at most six splits); the FP64 oracle itself is held to the same
    bound against the long-double evaluation on the CPU."""
    return np.maximum(1e-12 * np.abs(ref), 12 * (np.asarray(n) - 2) * U64 * mag)


def reference_cobg(mom, hel, with_oracle_fp64=False, C=None):
    """Colour-summed |M|^2 from the oracle in long double (float64 result)
    and its FP64 magnitude m (see fp64_allowance); optionally also the FP64
    oracle's own result (an independent FP64 evaluation, see
    fp64_comparable).  C: the colour matrix, if the caller has it (n = 8:
    colour_matrix_n8)."""
    from oracle import me2 as ome2
    from oracle.conditioning import me2_cobg_magnitude
    from oracle.numeric import extended
    ref = ome2.me2_cobg(extended(mom), hel, C=C).astype(np.float64)
    _, mag = me2_cobg_magnitude(mom, hel, C=C)
    if with_oracle_fp64:
        return ref, mag, ome2.me2_cobg(mom, hel, C=C)
    return ref, mag


def colour_matrix_n8():
    """C(8) from its stored first row (tests/golden, written by make_golden.py
    from the oracle, pinned in test_oracle_precision) by the oracle's
    relabelling; recomputing the row takes about 30 s."""
    import os
    from oracle.color import color_matrix_from_row0
    row0 = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "colour_matrix_n8_row0.txt"),
                      dtype=np.int64)
    return color_matrix_from_row0(8, row0)


def fp64_comparable(err_gpu, err_oracle, factor=10.0, floor=1e-15):
    """The GPU's FP64 errors on a sample are those of an FP64 evaluation:
    their p99 and max within `factor` of the FP64 oracle's own errors on the
    same events (both against the long-double reference; floor guards the
    case where both are at rounding level).  The magnitude bound of
    fp64_allowance is rigorous but loose (m / |ref| reaches 1e8 at n = 6 in
    this gauge); this criterion is tight."""
    g99, o99 = np.percentile(err_gpu, 99), np.percentile(err_oracle, 99)
    return (g99 <= factor * max(o99, floor)) and (err_gpu.max() <= factor * max(err_oracle.max(), floor))
