"""The oracle's own floating-point error, measured against an extended
reference, and pins that close gaps of the FP64 oracle's checks.

Extended reference.  Every oracle function computes in the precision of its
inputs (``oracle.numeric``): long-double momenta (64-bit significand) give
the reference the GPU bars are measured against.  That mode is pinned here to
a 40-digit mpmath evaluation of the same functions, so an FP64 constant or a
silent conversion somewhere in the oracle would show.

FP64 error budget.  Per event, e64 = |oracle FP64 - reference| / |reference|.
The magnitude numbers of ``oracle.magnitude`` give m, the value of the same
computation with every term taken in modulus; classical error analysis bounds
the rounding error of any evaluation order by a small multiple of u m
(u = 2^-53).  The tests check that bound on the FP64 oracle and report e64,
which is what the GPU FP64 bars are built on.
"""
import itertools

import numpy as np
import pytest

from bg_inputs import make_events
from oracle import cdbg, cobg, color, me2
from oracle.conditioning import me2_cobg_magnitude
from oracle.numeric import arbitrary, extended
from tests.helpers import mhv_helicities, nonvanishing

U64 = 2.0 ** -53
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)


def _mp_contract(amps, C):
    """A^dagger C A per event for an object array of mpmath amplitudes [K, E]."""
    import mpmath
    K, E = amps.shape
    out = []
    for e in range(E):
        s = mpmath.mpf(0)
        for i in range(K):
            for j in range(K):
                if C[i][j]:
                    s += int(C[i][j]) * (amps[i, e] * mpmath.conj(amps[j, e])).real
        out.append(s)
    return out


@pytest.mark.parametrize("n", [4, 5, 6])
def test_extended_reference_matches_arbitrary_precision(n):
    """Long-double |M|^2 equals the 40-digit evaluation of the same
    definitions to long-double rounding: median relative error below 1e-18 and
    every event below 1e-16, where the FP64 oracle sits at 1e-15 (an FP64
    constant or conversion anywhere in the extended mode would put the median
    there too)."""
    import mpmath
    E = 4
    ev = make_events(n, E, seed=4100 + n, cuts=True)
    hel = mhv_helicities(n, E, np.random.default_rng(41 + n))
    C = color.color_matrix_cached(n)
    ld = me2.me2_cobg(extended(ev["mom"]), hel)
    assert ld.dtype == np.longdouble
    mp = _mp_contract(cobg.partial_amplitudes(arbitrary(ev["mom"], 40), hel), C)
    f64 = me2.me2_cobg(ev["mom"], hel)
    rel_ld, rel_64 = [], []
    for e in range(E):
        ref = np.longdouble(mpmath.nstr(mp[e], 30))
        rel_ld.append(float(abs(ld[e] - ref) / abs(ref)))
        rel_64.append(float(abs(f64[e] - ref) / abs(ref)))
        _say(f"n={n} e={e}: long double {rel_ld[-1]:.1e}, FP64 oracle {rel_64[-1]:.1e}")
    assert np.median(rel_ld) < 1e-18 and max(rel_ld) < 1e-16


def test_extended_dressed_and_gradient_modes_run_in_long_double():
    """The dressed recursion and the dual-number gradient keep long double
    throughout (their results carry the type) and agree with FP64 to FP64
    rounding on a well-conditioned event."""
    from oracle.grad import me2_and_grad
    n = 5
    ev = make_events(n, 2, seed=4150, cuts=True)
    hel = mhv_helicities(n, 2, np.random.default_rng(415))
    rng = np.random.default_rng(416)
    col = np.zeros((2, n, 2), dtype=np.int8)
    for e in range(2):  # one closed chain through a random ordering
        perm = rng.permutation(n)
        ii = rng.integers(0, 3, n)
        for k in range(n):
            col[0, perm[k], e] = ii[k]
            col[1, perm[(k + 1) % n], e] = ii[k]
    a_ld = cdbg.flow_amplitude(extended(ev["mom"]), hel, col)
    a_64 = cdbg.flow_amplitude(ev["mom"], hel, col)
    assert a_ld.dtype == np.clongdouble
    assert np.max(np.abs(a_ld - a_64) / np.abs(a_ld)) < 1e-12
    m_ld, g_ld = me2_and_grad(extended(ev["mom"]), hel)
    m_64, g_64 = me2_and_grad(ev["mom"], hel)
    assert g_ld.dtype == np.longdouble or m_ld.dtype == np.longdouble
    scale = np.max(np.abs(g_ld), axis=(0, 1))
    assert np.max(np.abs(g_ld - g_64) / scale) < 1e-11


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_fp64_oracle_error_within_running_bound(n):
    """e64 of the FP64 oracle on sampled gg -> (n-2)g events, against the
    long-double reference: within the running error bound N u m for every
    event, N = 12 (n - 2) roundings along the deepest path (at most n - 2
    recursion levels, each a four-term dot product, a scaling and an
    accumulation over at most six splits), and at the 1e-15 level for the
    median event (1e-14)."""
    E = {4: 600, 5: 400, 6: 150, 7: 24}[n]
    ev = make_events(n, E, seed=4200 + n, cuts=True, sample_hel=True)
    mom, hel = ev["mom"], ev["hel"]
    keep = nonvanishing(hel)
    ref = me2.me2_cobg(extended(mom), hel)
    f64 = me2.me2_cobg(mom, hel)
    _, mag = me2_cobg_magnitude(mom, hel)
    e64 = (np.abs(f64 - ref) / np.abs(ref)).astype(np.float64)[keep]
    kappa = (mag / np.abs(ref)).astype(np.float64)[keep]
    ratio = e64 / (U64 * kappa)
    _say(f"n={n}: e64 median {np.median(e64):.1e} p99 {np.percentile(e64, 99):.1e} "
         f"max {e64.max():.1e}; events above 1e-12: {np.mean(e64 > 1e-12):.2%}; "
         f"e64/(u m) max {ratio.max():.1e}")
    assert np.all(ratio < 12 * (n - 2))
    assert np.median(e64) < 1e-14


@pytest.mark.parametrize("n", [5, 6])
def test_fp64_dressed_oracle_error(n):
    """The dressed (colour-flow) amplitude in FP64 against its long-double
    evaluation: |A|^2 within 1e-13 at the median event of sampled valid flows."""
    E = 40
    ev = make_events(n, E, seed=4300 + n, cuts=True, sample_hel=True)
    rng = np.random.default_rng(43 + n)
    col = np.zeros((2, n, E), dtype=np.int8)
    for e in range(E):
        perm = rng.permutation(n)
        ii = rng.integers(0, 3, n)
        for k in range(n):
            col[0, perm[k], e] = ii[k]
            col[1, perm[(k + 1) % n], e] = ii[k]
    keep = nonvanishing(ev["hel"])
    ref = np.abs(cdbg.flow_amplitude(extended(ev["mom"]), ev["hel"], col)) ** 2
    f64 = np.abs(cdbg.flow_amplitude(ev["mom"], ev["hel"], col)) ** 2
    nz = keep & (ref > 0)
    e64 = (np.abs(f64 - ref) / ref).astype(np.float64)[nz]
    _say(f"dressed n={n}: e64 median {np.median(e64):.1e} max {e64.max():.1e}")
    assert np.median(e64) < 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("row", [0, 77])
def test_colour_matrix_n7_rows_equal_gellmann(row):
    """Rows of C(7) from the definition with explicit 8x8 F matrices
    (eq. color_coefficient_adjoint, 8^7-entry chains) equal the trace-word
    values.  Row 0 pins the method beyond n = 6, row 77 the relabelling
    C_{s s'} = C_{id, pi(s')} that fills the other rows."""
    Cg = color.color_row_gellmann(7, row)
    Ce = color.color_matrix(7)[row].astype(np.float64)
    assert np.max(np.abs(Cg - Ce)) < 1e-9 * np.max(np.abs(Ce))


def test_colour_flow_sum_n6_equals_colour_summed():
    """Sum over all 9^6 colour-flow assignments of |A_flow|^2 (eq.
    color_decomposition_colorflow, flow amplitudes as chain-weighted sums of
    the 120 colour-ordered amplitudes) equals A^dagger C(6) A; flows without
    a closed chain contribute exactly 0.  The dressed recursion is checked on
    a sample of the same flows."""
    n = 6
    ev = make_events(n, 1, seed=1406, cuts=True)
    hel = mhv_helicities(n, 1, np.random.default_rng(n))
    ref = me2.me2_cobg(ev["mom"], hel)[0]
    cols = np.array(list(itertools.product(range(3), repeat=2 * n)), dtype=np.int8).T
    col = np.stack([cols[0::2], cols[1::2]])
    orders = [(0,) + s for s in itertools.permutations(range(1, n))]
    amps = [cobg.amplitude_of(ev["mom"], hel, o)[0] for o in orders]
    a = np.zeros(col.shape[2], dtype=np.complex128)
    for o, A in zip(orders, amps):
        a += cdbg.chain_weight(col, o) * A
    total = np.sum(np.abs(a) ** 2)
    _say(f"9^6 flow sum / A^dagger C A - 1 = {total / ref - 1:.1e}")
    assert abs(total / ref - 1) < 1e-11
    valid = np.nonzero(np.abs(a) > 0)[0]
    pick = np.random.default_rng(7).choice(valid, 256, replace=False)
    d = cdbg.flow_amplitude(np.repeat(ev["mom"], 256, axis=2), np.repeat(hel, 256, axis=1),
                            col[:, :, pick])
    assert np.max(np.abs(d - a[pick])) < 1e-11 * np.max(np.abs(a))


@pytest.mark.parametrize("n", [4, 5, 6])
def test_golden_colour_matrices(n):
    """The stored colour matrices (tests/golden, written by make_golden.py
    from the oracle) still equal the oracle's, are symmetric and have the
    diagonal (2N)^(n-2)(N^2-1) of the adjoint Casimir in the
    Tr(T^a T^b) = delta^ab normalisation."""
    stored = np.loadtxt(f"{GOLDEN}/colour_matrix_n{n}.txt", dtype=np.int64, ndmin=2)
    C = color.color_matrix(n)
    assert np.array_equal(stored, C)
    assert np.array_equal(stored, stored.T)
    assert np.all(np.diag(stored) == 6 ** (n - 2) * 8)


def test_golden_colour_matrix_n7_row0():
    stored = np.loadtxt(f"{GOLDEN}/colour_matrix_n7_row0.txt", dtype=np.int64, ndmin=2)
    assert np.array_equal(stored[0], color.color_matrix(7)[0])
    assert stored[0, 0] == 6 ** 5 * 8


@pytest.mark.slow
def test_colour_matrix_n8_entries_equal_gellmann():
    """Entries of the stored first row of C(8) from the definition with
    explicit 8x8 F matrices (eq. color_coefficient_adjoint, chains of 8^8
    entries): the diagonal, a non-zero and a zero off-diagonal entry, the
    entry of the last ordering and six random ones.  This pins C(8) independently of the
    trace-word method that the oracle and the library share."""
    stored = np.loadtxt(f"{GOLDEN}/colour_matrix_n8_row0.txt", dtype=np.int64, ndmin=2)[0]
    zero = int(np.nonzero(stored == 0)[0][0])
    extra = np.random.default_rng(808).choice(np.arange(2, 719), 6, replace=False)
    for j in [0, 1, zero, 719] + [int(x) for x in extra]:
        g = color.color_entry_gellmann(8, 0, j)
        assert abs(g - stored[j]) < 1e-9 * stored[0], (j, g, stored[j])


def test_golden_colour_matrix_n8_row0():
    """The stored first row of C(8) (720 entries, about 30 s to recompute)
    on 40 sampled entries against the oracle's trace words; the diagonal
    value; and the matrix filled from it by relabelling is symmetric, as
    C(8) must be (a wrong relabelling map or a wrong stored entry breaks
    the symmetry)."""
    stored = np.loadtxt(f"{GOLDEN}/colour_matrix_n8_row0.txt", dtype=np.int64, ndmin=2)[0]
    perms = color.middle_permutations(8)
    assert stored.shape == (720,) and stored[0] == 6 ** 6 * 8
    for j in np.random.default_rng(88).choice(720, 40, replace=False):
        assert stored[j] == color.color_entry(8, perms[0], perms[j])
    C = color.color_matrix_from_row0(8, stored)
    assert np.array_equal(C, C.T)
    assert np.all(np.diag(C) == stored[0])
