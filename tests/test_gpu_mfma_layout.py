"""The matrix-core layout that the colour contraction relies on."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mfma_f64_accumulator_columns():
    """Every accumulator element of v_mfma_f64_16x16x4f64 decodes to a unique
    (row, column) of A x B under the assumed A/B lane layout: element r of lane
    l is D[l / 16 + 4 r][l % 16], the layout the contraction kernels read
    their accumulators in."""
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
    cols = np.zeros((64, 4), dtype=int)
    for l in range(64):
        for r in range(4):
            rows[l, r], cols[l, r] = lookup[float(out[4 * l + r])]
            seen.add((rows[l, r], cols[l, r]))
    print("accumulator rows by (lane group, register):", rows[::16].tolist(), flush=True)
    assert len(seen) == 256
    lanes = np.arange(64)[:, None]
    assert np.array_equal(cols, np.broadcast_to(lanes % 16, (64, 4)))
    assert np.array_equal(rows, lanes // 16 + 4 * np.arange(4)[None, :])
