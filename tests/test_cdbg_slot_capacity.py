"""Capacity of the packed colour slots of the colour-dressed kernel.

The dressed current of a subset S of gluons 1..n-1 (Section 2.3, eqs.
cdcurrents and color_dressed_currents, for one colour-flow assignment of
eq. color_decomposition_colorflow) is a 3x3 colour matrix whose non-zero
entries are fixed by the colour edges j_k -> i_k of S: one entry (the trail
r -> c) when the edges are unbalanced but form a trail, one diagonal entry per
touched colour when they are balanced, none when they are disconnected or
admit no trail.  The kernel stores only those entries, packed in subset
order, and sizes its LDS for (2^(n-1) - 1) + 2^(n-1) / 4 of them.

Every colour assignment of n = 4..7 gluons is enumerated; for the flows whose
edges close into one circuit (balanced and connected: the others have a zero
amplitude and never reach the recursion) the total over all non-empty subsets
of gluons 1..n-1 must never exceed that capacity, and reaches it.
"""
import numpy as np
import pytest


def _all_flows(n):
    f = np.arange(9 ** n, dtype=np.int64)
    i = np.empty((n, f.size), np.int8)
    j = np.empty((n, f.size), np.int8)
    for k in range(n):
        d = f % 9
        f //= 9
        i[k] = d // 3
        j[k] = d % 3
    return i, j


def _entries(i, j, gluons):
    """Non-zero colour entries of the current of the subset `gluons`, for
    every flow (columns of i, j)."""
    deg = np.zeros((3, i.shape[1]), np.int16)
    touched = np.zeros((3, i.shape[1]), bool)
    link = np.zeros((3, i.shape[1]), bool)  # an edge between colours (0,1), (0,2), (1,2)
    for k in gluons:
        for c in range(3):
            deg[c] += (j[k] == c).astype(np.int16) - (i[k] == c)
            touched[c] |= (i[k] == c) | (j[k] == c)
        for x, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
            link[x] |= ((i[k] == a) & (j[k] == b)) | ((i[k] == b) & (j[k] == a))
    nt = touched.sum(axis=0)
    pairs = [(0, 1), (0, 2), (1, 2)]
    both = [touched[a] & touched[b] for a, b in pairs]
    linked_pairs = sum((both[x] & link[x]).astype(int) for x in range(3))
    connected = (nt <= 1) | ((nt == 2) & (linked_pairs >= 1)) | ((nt == 3) & (linked_pairs >= 2))
    balanced = np.all(deg == 0, axis=0)
    trail = (np.sum(deg == 1, axis=0) == 1) & (np.sum(deg == -1, axis=0) == 1) & \
        (np.sum(deg == 0, axis=0) == 1)
    return np.where(connected & balanced, nt, np.where(connected & trail, 1, 0))


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_packed_slot_capacity(n):
    i, j = _all_flows(n)
    closes = _entries(i, j, range(n)) > 0
    closes &= np.all(np.stack([np.sum(j == c, 0) == np.sum(i == c, 0) for c in range(3)]), 0)
    i, j = i[:, closes], j[:, closes]
    ns = 1 << (n - 1)
    total = np.zeros(i.shape[1], np.int64)
    for mask in range(1, ns):
        total += _entries(i, j, [k for k in range(n - 1) if mask >> k & 1])
    cap = (ns - 1) + ns // 4
    assert total.max() == cap
    # a single gluon always holds exactly one entry
    assert np.all(_entries(i, j, [0]) == 1)
