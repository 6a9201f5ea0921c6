"""CPU checks of the C ABI's synchronous argument and graph validation.
Malformed input is rejected before any device call, so these run without a
GPU (the library is called through ctypes directly)."""
import ctypes

import numpy as np
import pytest

from paper_2003_02450_amd import _lib

ARG, GRAPH, SIZE = 1, 2, 7


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _build(N, rp, ci, w, omega=0.5, gamma=1.0, flags=0):
    rp = np.ascontiguousarray(rp, np.int64)
    ci = np.ascontiguousarray(ci, np.int32)
    w = np.ascontiguousarray(w, np.float64)
    h = ctypes.c_void_p()
    st = _lib.load().qsw_superop_build(N, _ptr(rp), _ptr(ci), _ptr(w), omega, gamma, flags,
                                       None, ctypes.byref(h))
    assert not h.value  # nothing is returned on failure
    return st


def test_rejects_self_loop():
    assert _build(3, [0, 1, 1, 1], [0], [1.0]) == GRAPH


@pytest.mark.parametrize("w", [0.0, -1.0, float("nan"), float("inf")])
def test_rejects_non_positive_or_non_finite_weight(w):
    assert _build(3, [0, 1, 1, 1], [2], [w]) == GRAPH


def test_rejects_unsorted_and_duplicate_columns():
    assert _build(3, [0, 2, 2, 2], [2, 1], [1.0, 1.0]) == GRAPH
    assert _build(3, [0, 2, 2, 2], [1, 1], [1.0, 1.0]) == GRAPH


def test_rejects_out_of_range_and_bad_row_ptr():
    assert _build(3, [0, 1, 1, 1], [3], [1.0]) == GRAPH
    assert _build(3, [0, 1, 1, 1], [-1], [1.0]) == GRAPH
    assert _build(3, [1, 1, 1, 1], [], []) == GRAPH
    assert _build(3, [0, 2, 1, 2], [1, 2], [1.0, 1.0]) == GRAPH


@pytest.mark.parametrize("omega", [-0.1, 1.5, float("nan")])
def test_rejects_omega_outside_unit_interval(omega):
    assert _build(2, [0, 1, 1], [1], [1.0], omega=omega) == ARG


def test_rejects_bad_gamma_and_flags():
    assert _build(2, [0, 1, 1], [1], [1.0], gamma=0.0) == ARG
    assert _build(2, [0, 1, 1], [1], [1.0], flags=8) == ARG


def test_rejects_order_beyond_32_bit_columns():
    N = 46341  # N^2 > 2^31 - 1
    assert _build(N, np.zeros(N + 1), [], []) == SIZE


def _build_ops(N, H, ML, omega=0.5):
    import scipy.sparse as sp
    Hc = sp.csr_matrix(np.asarray(H, np.complex128))
    Mc = sp.csr_matrix(np.asarray(ML, np.float64))
    hp = np.ascontiguousarray(Hc.indptr, np.int64)
    hc = np.ascontiguousarray(Hc.indices, np.int32)
    hv = np.ascontiguousarray(Hc.data, np.complex128).view(np.float64)
    lp = np.ascontiguousarray(Mc.indptr, np.int64)
    lc = np.ascontiguousarray(Mc.indices, np.int32)
    lv = np.ascontiguousarray(Mc.data, np.float64)
    h = ctypes.c_void_p()
    st = _lib.load().qsw_superop_build_ops(N, _ptr(hp), _ptr(hc), _ptr(hv), _ptr(lp), _ptr(lc),
                                           _ptr(lv), omega, 0, None, ctypes.byref(h))
    assert not h.value
    return st


def test_build_ops_rejects_non_hermitian_h():
    ML = np.zeros((2, 2))
    assert _build_ops(2, [[0, 1], [2, 0]], ML) == GRAPH          # values
    assert _build_ops(2, [[0, 1], [0, 0]], ML) == GRAPH          # pattern
    assert _build_ops(2, [[0, 1j], [1j, 0]], ML) == GRAPH        # not conj-symmetric
    assert _build_ops(2, [[1j, 0], [0, 0]], ML) == GRAPH         # complex diagonal


def test_build_ops_rejects_bad_omega_and_flags():
    H = [[0, 1], [1, 0]]
    assert _build_ops(2, H, np.zeros((2, 2)), omega=2.0) == ARG


def test_propagate_rejects_null_handle_and_workspace_query():
    L = _lib.load()
    assert L.qsw_propagate(None, None, 0.0, 1.0, 1, None, None, 0, None) == ARG
    assert L.qsw_propagate_workspace_bytes(None, 0.0, 1.0, 1) == 0
    assert L.qsw_last_stats(None, None) == ARG
    assert L.qsw_apply(None, None, None, None) == ARG
    assert L.qsw_populations(None, None, 1, None, None) == ARG
    assert L.qsw_superop_set_precision(None, 0) == ARG
    assert L.qsw_superop_set_pacing(None, 4) == ARG
    L.qsw_superop_destroy(None)  # no-op
