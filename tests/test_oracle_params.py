"""Pins for the oracle's parameter choice and its exact 1-norm.

The paper takes its Taylor degree m and scaling s from Al-Mohy and Higham's
analysis (Section 3.1), and computes the 1-norm series ||A^p||_1^(1/p) once at
construction (Section 4, footnote).  The oracle restates that choice in
``expmv.select_params``; these tests check it against what the rule itself
fixes, not against a second copy of the same loop:

* feasibility: the returned (m, s) meets the backward-error bound
  t max(d_p, d_{p+1}) / s <= theta_m for some p with p(p-1)-1 <= m;
* optimality: no admissible pair (m', p') has a smaller m' ceil(alpha_p'/theta_m'),
  and among the pairs of least cost m is the smallest degree;
* the switch of the cited condition (3.13) sits at
  2 ell p_max (p_max + 3) theta_{m_max} / (n0 m_max), checked on both sides,
  with theta_55 taken from the published table;
* a special case that reduces to the plain 1-norm rule (all d_p equal);
* end to end, the chosen (m, s) reach exp(tA)b to double precision.

``oracle_norm1`` (qsw_oracle.c) is checked against dense column sums.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import expmv, native
from oracle import theta as oth

TH = oth.theta_table()


def _admissible_pairs(m_max=oth.M_MAX, p_max=oth.P_MAX):
    for p in range(2, p_max + 1):
        for m in range(max(1, p * (p - 1) - 1), m_max + 1):
            yield m, p


def _alpha(d, p, t):
    return t * max(d[p], d[p + 1])


def _random_case(rng, large=True):
    nrm = float(10 ** rng.uniform(-1, 2))
    d = {p: nrm * float(rng.uniform(0.01, 1.0)) for p in range(2, 10)}
    # t large enough that ||tA||_1 is past the condition-(3.13) switch (~63)
    lo = math.log10(70.0 / nrm) if large else -2
    t = float(10 ** rng.uniform(lo, lo + 2.5))
    return nrm, d, t


# ----------------------------------------------------------- exact 1-norm

def _random_csr(rng, n, density):
    A = np.zeros((n, n), np.complex128)
    mask = rng.random((n, n)) < density
    A[mask] = rng.normal(size=mask.sum()) + 1j * rng.normal(size=mask.sum())
    if n > 2:
        A[1, :] = 0.0          # an empty row
        A[:, 2] = 0.0          # an empty column
    rows, cols = np.nonzero(A)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return native.CSR(n, rp, cols.astype(np.int32), A[rows, cols]), A


def test_norm1_hand_case():
    # [[1, -2i], [3+4i, 0]]: column sums |1| + |3+4i| = 6 and |-2i| = 2.
    A = native.CSR(2, np.array([0, 2, 3]), np.array([0, 1, 0], np.int32),
                   np.array([1.0, -2j, 3 + 4j]))
    assert A.norm1() == 6.0


@pytest.mark.parametrize("seed,n,density", [(1, 7, 0.5), (2, 40, 0.1), (3, 130, 0.03),
                                            (4, 64, 0.9)])
def test_norm1_matches_dense_column_sums(seed, n, density):
    rng = np.random.Generator(np.random.PCG64(seed))
    A, D = _random_csr(rng, n, density)
    want = np.abs(D).sum(axis=0).max()
    assert abs(A.norm1() - want) <= 1e-14 * want


def test_norm1_is_column_not_row_sum():
    # A single dense row: the largest column sum is one entry, the row sum is n.
    n = 9
    A = native.CSR(n, np.r_[0, np.full(n, n)].astype(np.int64),
                   np.arange(n, dtype=np.int32), np.full(n, 2.0 + 0j))
    assert A.norm1() == 2.0


def test_norm1_of_walk_superop_matches_dense():
    import oracle
    import workloads
    rng = np.random.Generator(np.random.PCG64(12))
    g = workloads.random_out_degree(9, 3, rng)
    A = oracle.walk_superop(g.dense(), 0.35)
    D = A.dense()
    assert abs(A.norm1() - np.abs(D).sum(axis=0).max()) <= 1e-14 * A.norm1()


# ---------------------------------------------------------- the alpha_p rule

@pytest.mark.parametrize("tol,m_max,p_max", [(oth.TOL_DOUBLE, oth.M_MAX, oth.P_MAX),
                                               (oth.TOL_SINGLE, 20, 5)])
def test_select_params_feasible_and_optimal(tol, m_max, p_max):
    th = oth.theta_table(tol)
    rng = np.random.Generator(np.random.PCG64(41))
    for _ in range(300):
        nrm, d, t = _random_case(rng)
        n0 = int(rng.integers(1, 5))
        if expmv.condition_3_13(t * nrm, n0, thetas=th, m_max=m_max, p_max=p_max):
            continue
        m, s = expmv.select_params(nrm, d, t, n0, thetas=th, m_max=m_max, p_max=p_max)
        assert m <= m_max
        # feasibility: the bound holds for some admissible p
        assert any(p * (p - 1) - 1 <= m and _alpha(d, p, t) / s <= th[m - 1]
                   for p in range(2, p_max + 1)), (nrm, t, m, s)
        # optimality over every admissible pair, smallest m among the best
        costs = [(mm * math.ceil(_alpha(d, p, t) / th[mm - 1]), mm)
                 for mm, p in _admissible_pairs(m_max, p_max)]
        best = min(c for c, _ in costs)
        assert m * s == best, (m, s, best)
        assert m == min(mm for c, mm in costs if c == best)


def test_select_params_uses_the_larger_of_consecutive_norms():
    # d_{p+1} far above d_p for every p: a rule that forgot max(d_p, d_{p+1})
    # would take s from d_p alone and break the bound.
    nrm = 10.0
    d = {p: (1.0 if p % 2 == 0 else 9.0) for p in range(2, 10)}
    t = 40.0
    m, s = expmv.select_params(nrm, d, t)
    assert t * 9.0 / s <= TH[m - 1]


def test_select_params_equal_norms_reduce_to_norm1_rule():
    # d_p = ||A||_1 for every p (e.g. A = c I): alpha_p = ||tA||_1 and p = 2
    # admits every m >= 1, so the rule is the plain 1-norm choice.
    for x in (64.0, 100.0, 1234.5, 5e4):
        d = {p: 3.0 for p in range(2, 10)}
        assert expmv.select_params(3.0, d, x / 3.0) == expmv.select_params_norm1(x)


@pytest.mark.parametrize("n0", [1, 2, 4])
def test_condition_3_13_boundary(n0):
    ell, pm, mm = 2, oth.P_MAX, oth.M_MAX
    thr = 2 * ell * pm * (pm + 3) * TH[mm - 1] / (n0 * mm)
    # theta_55 = 9.9 in the published table (two digits)
    lo = 2 * ell * pm * (pm + 3) * 9.85 / (n0 * mm)
    hi = 2 * ell * pm * (pm + 3) * 9.95 / (n0 * mm)
    assert lo <= thr <= hi
    nrm = 1.0
    d = {p: 1e-3 for p in range(2, 10)}            # far below ||A||_1
    below = thr * (1 - 1e-12)
    above = thr * (1 + 1e-12)
    assert expmv.condition_3_13(below, n0) and not expmv.condition_3_13(above, n0)
    assert expmv.select_params(nrm, d, below, n0) == expmv.select_params_norm1(below)
    m, s = expmv.select_params(nrm, d, above, n0)
    m1, s1 = expmv.select_params_norm1(above)
    assert m * s < m1 * s1                           # the d_p were used


def test_select_params_zero():
    d = {p: 1.0 for p in range(2, 10)}
    assert expmv.select_params(0.0, d, 5.0) == (0, 1)
    assert expmv.select_params(2.0, d, 0.0) == (0, 1)


def test_select_params_end_to_end_accuracy():
    """With exact d_p from dense powers of a walk generator, the chosen (m, s)
    give exp(tA) b to within a small multiple of the unit roundoff
    (backward-error bound), past the condition-(3.13) switch."""
    import oracle
    import workloads
    rng = np.random.Generator(np.random.PCG64(77))
    g = workloads.random_out_degree(8, 3, rng)
    A = oracle.walk_superop(g.dense(), 0.4)
    D = A.dense()
    nrm = np.abs(D).sum(0).max()
    d = {}
    P = D.copy()
    for p in range(2, 10):
        P = P @ D
        d[p] = np.abs(P).sum(0).max() ** (1.0 / p)
    rho0 = workloads.random_density(8, rng, rank=2).reshape(-1)
    for t in (70.0 / nrm * 1.5, 400.0 / nrm):
        assert not expmv.condition_3_13(t * nrm)
        m, s = expmv.select_params(nrm, d, t)
        assert m * s < np.prod(expmv.select_params_norm1(t * nrm))
        F, _ = native.taylor_expmv(A, rho0, t, m, s, oth.TOL_DOUBLE)
        ref = scipy.linalg.expm(t * D) @ rho0
        assert np.abs(F - ref).max() <= 1e-12, t


@pytest.mark.parametrize("tol,m_max,p_max", [(oth.TOL_DOUBLE, oth.M_MAX, oth.P_MAX),
                                               (oth.TOL_SINGLE, 20, 5)])
def test_select_params_without_switch_feasible_and_optimal(tol, m_max, p_max):
    """Without the condition-3.13 switch the alpha_p rule holds at every
    ||tA||_1, small ones included: feasible and optimal as above."""
    th = oth.theta_table(tol)
    rng = np.random.Generator(np.random.PCG64(43))
    for _ in range(300):
        nrm, d, t = _random_case(rng, large=False)
        m, s = expmv.select_params(nrm, d, t, thetas=th, m_max=m_max, p_max=p_max,
                                   switch=False)
        assert any(p * (p - 1) - 1 <= m and _alpha(d, p, t) / s <= th[m - 1]
                   for p in range(2, p_max + 1)), (nrm, t, m, s)
        costs = [(mm * math.ceil(_alpha(d, p, t) / th[mm - 1]), mm)
                 for mm, p in _admissible_pairs(m_max, p_max)]
        best = min(c for c, _ in costs)
        assert m * s == best and m == min(mm for c, mm in costs if c == best)
