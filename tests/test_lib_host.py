"""Host-side checks of libbg.so that need no GPU: symbols, colour matrices,
status strings and argument validation (calls that return before any launch)."""
import ctypes

import numpy as np
import pytest

from oracle import color
from paper_2106_06507_amd import _lib
from paper_2106_06507_amd._lib import lib, bg_request


def test_library_exports_every_header_symbol():
    L = lib()
    names = _lib.header_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_lib._SIGNATURES), "binding and header disagree"


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_colour_matrix_matches_oracle(n):
    K = _lib.lib().bg_num_orderings(n)
    out = np.zeros(K * K)
    st = lib().bg_color_matrix(n, out.ctypes.data_as(ctypes.c_void_p), K * K)
    assert st == _lib.BG_OK
    ref = color.color_matrix(n)
    assert np.array_equal(out.reshape(K, K), ref.astype(np.float64))


def test_colour_matrix_matches_golden_files():
    """The library's C(n) against the stored fixtures of tests/golden (n = 4..6
    whole, n = 7 first row)."""
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    for n in (4, 5, 6, 7):
        K = _lib.lib().bg_num_orderings(n)
        out = np.zeros(K * K)
        assert lib().bg_color_matrix(n, out.ctypes.data_as(ctypes.c_void_p), K * K) == 0
        name = f"colour_matrix_n{n}.txt" if n < 7 else "colour_matrix_n7_row0.txt"
        stored = np.loadtxt(os.path.join(gold, name), ndmin=2)
        assert np.array_equal(out.reshape(K, K)[: stored.shape[0]], stored)


def test_colour_matrix_n8_sampled_entries():
    n = 8
    K = 720
    out = np.zeros(K * K)
    assert lib().bg_color_matrix(n, out.ctypes.data_as(ctypes.c_void_p), K * K) == 0
    C = out.reshape(K, K)
    assert np.array_equal(C, C.T)
    import os
    row0 = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "colour_matrix_n8_row0.txt"),
                      dtype=np.int64)
    assert np.array_equal(C, color.color_matrix_from_row0(n, row0).astype(np.float64))
    perms = color.middle_permutations(n)
    rng = np.random.default_rng(8)
    for _ in range(6):
        i, j = rng.integers(0, K, 2)
        assert C[i, j] == color.color_entry(n, perms[i], perms[j])


def test_colour_matrix_rejects_bad_arguments():
    out = np.zeros(4)
    p = out.ctypes.data_as(ctypes.c_void_p)
    assert lib().bg_color_matrix(3, p, 4) == _lib.BG_EINVAL
    assert lib().bg_color_matrix(9, p, 4) == _lib.BG_EINVAL
    assert lib().bg_color_matrix(4, None, 4) == _lib.BG_EINVAL
    assert lib().bg_color_matrix(4, p, 3) == _lib.BG_ERANGE


def test_status_strings_and_orderings():
    for s in range(-6, 1):
        assert lib().bg_status_string(s)
    assert lib().bg_status_string(-99) == b"unknown status"
    assert [lib().bg_num_orderings(n) for n in range(3, 11)] == [0, 2, 6, 24, 120, 720, 5040, 0]


def test_entry_points_validate_before_launch():
    L = lib()
    req = bg_request()
    req.n = 6
    req.n_events = 10
    assert L.bg_currents(None, 6, 10, None, None, 0, None, None) == _lib.BG_EINVAL
    assert L.bg_color_contract(None, 6, 10, None, None, 0, None) == _lib.BG_EINVAL
    assert L.bg_me2(None, ctypes.byref(req), None) == _lib.BG_EINVAL
    assert L.bg_me2_grad(None, ctypes.byref(req), None, None, None) == _lib.BG_EINVAL
    assert L.bg_me2_batch(None, ctypes.byref(req), 1, None) == _lib.BG_EINVAL
    assert L.bg_me2_batch_tune(None, ctypes.byref(req), 1, None, None, None) == _lib.BG_EINVAL
    cfg = _lib.bg_batch_config(0, 64, 256, 0)
    assert L.bg_batch_config_get(None, 0, ctypes.byref(cfg)) == _lib.BG_EINVAL
    assert L.bg_batch_config_set(None, 0, ctypes.byref(cfg)) == _lib.BG_EINVAL
    gp = _lib.bg_gen_params(6, 1, 1000.0, 20.0, 0.4, 1, 0)
    assert L.bg_generate(None, ctypes.byref(gp), 10, 10, None, None, None, None, None, None) == _lib.BG_EINVAL
    assert L.bg_me2_continuous(None, 6, 0, 10, None, None, None, None, None) == _lib.BG_EINVAL
    assert L.bg_generate_continuous(None, 6, 1, 0, 10, None, None, None) == _lib.BG_EINVAL
    L.bg_context_destroy(None)  # no-op


def test_context_create_without_device_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib().bg_context_create(ctypes.byref(h), 0, 0) == _lib.BG_ENODEV
    assert lib().bg_context_create(None, 0, 0) == _lib.BG_EINVAL
    # unknown context flags are rejected before any device is touched
    assert lib().bg_context_create(ctypes.byref(h), 0, 1 << 10) == _lib.BG_EINVAL
