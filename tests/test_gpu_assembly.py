"""GPU superoperator assembly and 1-norms against the oracle (through the C ABI)."""
import itertools

import numpy as np
import pytest

import oracle
import workloads
from oracle import native
from tests.gpu_util import build_gpu, oracle_superop, random_workload

pytestmark = pytest.mark.gpu


def canonical_rows(rp, col, val):
    """Sort the entries of every row by column (the device keeps rows in
    structural order; the oracle's rows are sorted)."""
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    order = np.lexsort((col, rows))
    return col[order], val[order]


def test_canonical_rows_helper():
    rp = np.array([0, 3, 5])
    col, val = canonical_rows(rp, np.array([5, 1, 3, 2, 0]), np.arange(5.0))
    assert col.tolist() == [1, 3, 5, 0, 2] and val.tolist() == [1, 2, 0, 4, 3]


def _compare_csr(op, A, val_tol=0.0):
    rp, col, val = op.csr()
    assert op.n == A.n and op.nnz == A.nnz
    assert np.array_equal(rp, A.row_ptr)
    col, val = canonical_rows(rp, col, val)
    assert np.array_equal(col, A.col)
    scale = max(1.0, float(np.abs(A.val).max()) if A.nnz else 1.0)
    assert float(np.abs(val - A.val).max() if A.nnz else 0.0) <= val_tol * scale


@pytest.mark.parametrize("h_mode,r_mode,dephasing",
                         list(itertools.product(["laplacian", "adjacency"],
                                                ["transition", "colnorm"], [False, True])))
def test_assembly_matches_oracle_all_modes(h_mode, r_mode, dephasing):
    for N, k, seed in ((2, 1, 1), (5, 2, 2), (13, 3, 3), (37, 4, 4)):
        for omega in (0.0, 0.37, 1.0):
            wl = random_workload(N, k, omega, seed, h_mode, r_mode, dephasing)
            op = build_gpu(wl)
            _compare_csr(op, oracle_superop(wl), 1e-15)
            op.close()


def test_assembly_cycle16_and_er256():
    for wl in (workloads.cycle16(), workloads.er256()):
        op = build_gpu(wl)
        _compare_csr(op, oracle_superop(wl), 1e-15)
        op.close()


def test_assembly_outdeg1024_full_size():
    """The benchmark superoperator (N = 1024, 4.28e7 entries), element by element."""
    wl = workloads.outdeg1024()
    op = build_gpu(wl)
    A = oracle_superop(wl)
    _compare_csr(op, A, 1e-15)
    info = op.info()
    assert abs(info["norm1"] - A.norm1()) <= 1e-13 * A.norm1()
    op.close()


def test_norm1_exact_matches_oracle():
    for seed in range(4):
        wl = random_workload(11 + seed, 3, 0.25 * seed, seed, dephasing=bool(seed & 1))
        op = build_gpu(wl)
        A = oracle_superop(wl)
        assert abs(op.info()["norm1"] - A.norm1()) <= 1e-14 * A.norm1()
        op.close()


def _apply_power(A, v, p):
    for _ in range(p):
        v = A.matvec(v)
    return v


def _probe(n, which):
    """The estimator's deterministic probe columns: all ones / n, and s_i / n
    with s_0 = -1 and s_i the sign of the top bit of SplitMix64(0x51A7E5 + i)."""
    if which == 0:
        return np.full(n, 1.0 / n, np.complex128)
    out = np.empty(n, np.complex128)
    mask = (1 << 64) - 1
    for i in range(n):
        x = (0x51A7E5 + i + 0x9E3779B97F4A7C15) & mask
        x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & mask
        x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & mask
        x = x ^ (x >> 31)
        out[i] = (-1.0 if (x >> 63) else 1.0) / n
    out[0] = -1.0 / n
    return out


@pytest.mark.parametrize("wl_fn", [workloads.cycle16,
                                   lambda: random_workload(9, 3, 0.6, 5, dephasing=True)])
def test_norm_estimates_are_attained_and_bounded(wl_fn):
    """Each d_p^p is ||L^p v||_1 for the unit 1-norm vector v the estimator
    reports, is at most the exact ||L^p||_1 (dense powers), and is within the
    estimator's usual factor of 3 of it (it is a lower bound, exact in most
    cases but not all: cycle16 at p = 4 gives 25.06 against 25.56)."""
    wl = wl_fn()
    op = build_gpu(wl)
    info = op.info()
    A = oracle_superop(wl)
    D = A.dense()
    P = D.copy()
    for p in range(2, 10):
        P = D @ P                      # P = D^p
        exact = np.abs(P).sum(axis=0).max()
        est = info["d"][p] ** p
        idx = info["d_index"][p]
        if idx >= 0:
            v = np.zeros(A.n, np.complex128)
            v[idx] = 1.0
        else:
            v = _probe(A.n, info["d_probe"][p])
        attained = np.abs(_apply_power(A, v, p)).sum()
        assert abs(est - attained) <= 1e-12 * max(attained, 1e-300), (p, est, attained)
        assert est <= exact * (1 + 1e-12)
        assert est >= exact / 3.0, (p, est, exact)
    op.close()


def test_norm_estimates_attained_on_er256():
    wl = workloads.er256()
    op = build_gpu(wl)
    info = op.info()
    A = oracle_superop(wl)
    nrm = A.norm1()
    for p in range(2, 10):
        est = info["d"][p] ** p
        idx = info["d_index"][p]
        if idx >= 0:
            v = np.zeros(A.n, np.complex128)
            v[idx] = 1.0
        else:
            v = _probe(A.n, info["d_probe"][p])
        attained = np.abs(_apply_power(A, v, p)).sum()
        assert abs(est - attained) <= 1e-12 * attained
        assert info["d"][p] <= nrm * (1 + 1e-12)
    op.close()


def test_apply_matches_oracle_matvec():
    import torch
    wl = workloads.er256()
    op = build_gpu(wl)
    A = oracle_superop(wl)
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    y = op.apply(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    ref = A.matvec(x)
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    op.close()


def test_empty_graph_and_single_vertex():
    import paper_2003_02450_amd as qsw
    # N = 1, no arcs: L = 0
    op = qsw.Superop.from_graph(1, np.array([0, 0]), np.array([], np.int32),
                                np.array([], np.float64), 0.5)
    rp, col, val = op.csr()
    assert op.nnz == 1 and rp.tolist() == [0, 1] and col.tolist() == [0]
    assert val[0] == 0
    assert op.info()["norm1"] == 0.0
    op.close()
    # N = 6, no arcs
    op = qsw.Superop.from_graph(6, np.zeros(7, np.int64), np.array([], np.int32),
                                np.array([], np.float64), 0.3)
    assert op.nnz == 36 and op.info()["norm1"] == 0.0
    op.close()


def test_build_ops_matches_graph_build_and_oracle():
    import paper_2003_02450_amd as qsw
    import scipy.sparse as sp
    G, Gu = workloads.two_sources_one_sink()
    for omega in (0.0, 0.9, 1.0):
        op = qsw.Superop.from_operators(sp.csr_matrix(Gu.dense()), sp.csr_matrix(G.dense()),
                                        omega)
        A = native.superop_csr(Gu.dense(), G.dense(), omega)
        _compare_csr(op, A, 1e-15)
        op2 = qsw.Superop.from_graph(3, G.row_ptr, G.col_idx, G.w, omega, h_mode="adjacency")
        assert np.array_equal(op.csr()[2], op2.csr()[2])
        op.close()
        op2.close()
