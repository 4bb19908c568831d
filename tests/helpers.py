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
