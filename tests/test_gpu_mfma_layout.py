"""The matrix-core layout that the colour contraction relies on."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mfma_f64_accumulator_columns():
    """Every accumulator element of v_mfma_f64_16x16x4f64 decodes to a unique
    (row, column) of A x B under the assumed A/B lane layout, and its column is
    lane % 16 (the only accumulator property the contraction uses)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_06507_amd import api
    from paper_2106_06507_amd._lib import lib, check
    ctx = api.default_context()
    out = np.zeros(256)
    check(lib().bg_mfma_layout_probe(ctx.handle, out.ctypes.data_as(ctypes.c_void_p)), "probe")
    A = np.array([[(i + 1) + 100.0 * k for k in range(4)] for i in range(16)])
    B = np.array([[(j + 1) * 8.0 ** k for j in range(16)] for k in range(4)])
    D = A @ B
    lookup = {float(D[i, j]): (i, j) for i in range(16) for j in range(16)}
    seen = set()
    rows = np.zeros((64, 4), dtype=int)
    for l in range(64):
        for r in range(4):
            i, j = lookup[float(out[4 * l + r])]
            assert j == l % 16
            rows[l, r] = i
            seen.add((i, j))
    assert len(seen) == 256
    print("accumulator rows by (lane group, register):", rows[::16].tolist(), flush=True)
