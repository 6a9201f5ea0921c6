"""Pins for the oracle's theta_m constants (backward-error bound of the
truncated Taylor method the paper adopts in Section 3.1)."""
import math

import mpmath
import pytest

from oracle import theta as th


def test_theta_monotone_in_m():
    t = th.theta_table()
    assert len(t) == th.M_MAX
    assert all(b > a for a, b in zip(t, t[1:]))


def test_theta_1_closed_form():
    # m = 1: h_2(x) = log(1 + x) - x, so |c_k| = 1/k (k >= 2) and
    # h~_2(theta)/theta = sum_{k>=2} theta^(k-1)/k = theta/2 + theta^2/3 + ...
    # which equals tol at theta ~= 2 tol (1 - 4 tol/3 + ...).
    tol = th.TOL_DOUBLE
    expect = 2 * tol
    assert abs(th.theta(1) - expect) / expect < 1e-12


def test_theta_2_closed_form():
    # m = 2: log(1 + x + x^2/2) - x = -x^3/6 + 0 x^4 + x^5/40 - ...
    # so h~_3(theta)/theta ~= theta^2/6 for tiny theta: theta_2 ~= sqrt(6 tol).
    expect = math.sqrt(6 * th.TOL_DOUBLE)
    assert abs(th.theta(2) - expect) / expect < 1e-6


def test_coefficients_vanish_below_m_plus_1():
    # c_k = 0 for k <= m and c_{m+1} = -1/(m+1)!  (log(e^-x T_m(x)) is
    # O(x^{m+1}) because T_m matches e^x to degree m).
    for m in (3, 17, 55):
        c = th.log_taylor_coeffs(m, m + 40)
        for k in range(m + 1):
            assert abs(c[k]) < mpmath.mpf(10) ** -120
        with mpmath.workdps(120):
            rel = abs(c[m + 1] + 1 / mpmath.factorial(m + 1)) * mpmath.factorial(m + 1)
            assert rel < mpmath.mpf(10) ** -60


def test_coefficients_match_direct_series():
    # Independent check of the recurrence: mpmath.taylor of log(exp(-x) T_m(x)).
    m = 6
    f = lambda x: mpmath.log(mpmath.exp(-x) * sum(x ** k / mpmath.factorial(k)
                                                  for k in range(m + 1)))
    with mpmath.workdps(50):
        direct = mpmath.taylor(f, 0, 14)
    c = th.log_taylor_coeffs(m, 14)
    for k in range(15):
        assert abs(c[k] - direct[k]) < mpmath.mpf(10) ** -30


def test_series_truncation_is_converged():
    for m in (30, 55):
        K = th._series_length(m)
        t = th.theta(m)
        a = th.backward_error_ratio(m, t, K)
        b = th.backward_error_ratio(m, t, K + 600)
        assert abs(a - b) / b < 1e-12
        assert a <= th.TOL_DOUBLE


# Al-Mohy and Higham, "Computing the action of the matrix exponential",
# Table 3.1 (u = 2^-53), two significant digits as published.
PUBLISHED = {5: 2.4e-3, 10: 1.4e-1, 15: 6.4e-1, 20: 1.4, 25: 2.4, 30: 3.5,
             35: 4.7, 40: 6.0, 45: 7.2, 50: 8.5, 55: 9.9}


@pytest.mark.parametrize("m", sorted(PUBLISHED))
def test_theta_matches_published_table(m):
    got = th.theta(m)
    assert float(f"{got:.2g}") == pytest.approx(PUBLISHED[m], rel=1e-9), got


def test_theta_single_precision_smaller():
    # The unit roundoff of binary32 gives larger theta (looser tolerance).
    for m in (10, 30, 55):
        assert th.theta(m, th.TOL_SINGLE) > th.theta(m)
