"""Oracle: the theta_m constants of the truncated-Taylor backward-error bound.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file.

The paper evaluates exp(A)u by the scaling relation and a truncated Taylor
polynomial T_m (Section 3.1, scaling-and-squaring equations), choosing m and s
by the backward-error analysis of Al-Mohy and Higham, which it cites for its
`step` and `series` algorithms (their Algorithms 3.2 and 5.2).  That analysis
writes (T_m(s^-1 A))^s = exp(A + dA) and bounds dA through

    h_{m+1}(x) = log(exp(-x) T_m(x)) = sum_{k >= m+1} c_k x^k,
    h~_{m+1}(x) = sum_{k >= m+1} |c_k| x^k,

    theta_m = max{ theta : h~_{m+1}(theta) / theta <= tol }.

This module computes c_k in high-precision arithmetic straight from that
definition: the power series of log(T_m(x)) from the identity T_m * g' = T_m'
for g = log T_m, minus the series of x.  Nothing is taken from a printed table.
"""
from __future__ import annotations

import functools

import mpmath

M_MAX = 55          # largest Taylor degree considered (Al-Mohy and Higham)
P_MAX = 8           # largest power p in the alpha_p(A) bounds (norms of A^1..A^9)
TOL_DOUBLE = 2.0 ** -53
TOL_SINGLE = 2.0 ** -24

_DPS = 160          # working digits: c_{m+1} = -1/(m+1)! is ~1e-75 at m = 55


@functools.lru_cache(maxsize=None)
def log_taylor_coeffs(m: int, K: int) -> tuple:
    """Coefficients c_0..c_K of h_{m+1}(x) = log T_m(x) - x, as mpf.

    g = log T_m satisfies T_m g' = T_m'; with T_m = sum_{k<=m} f_k x^k,
    f_k = 1/k!, comparing x^{k-1} coefficients gives
        k g_k = k f_k - sum_{j=1}^{k-1} j g_j f_{k-j}.
    """
    with mpmath.workdps(_DPS):
        f = [mpmath.mpf(1) / mpmath.factorial(k) if k <= m else mpmath.mpf(0)
             for k in range(K + 1)]
        g = [mpmath.mpf(0)] * (K + 1)   # g_0 = log T_m(0) = log 1 = 0
        for k in range(1, K + 1):
            acc = k * f[k]
            for j in range(max(1, k - m), k):
                acc -= j * g[j] * f[k - j]
            g[k] = acc / k
        c = list(g)
        c[1] -= 1                       # subtract the series of x
        return tuple(c)


def backward_error_ratio(m: int, theta, K: int) -> mpmath.mpf:
    """h~_{m+1}(theta)/theta = sum_{k>m} |c_k| theta^{k-1}, truncated at K."""
    c = log_taylor_coeffs(m, K)
    with mpmath.workdps(40):
        th = mpmath.mpf(theta)
        s = mpmath.mpf(0)
        p = th ** m
        for k in range(m + 1, K + 1):
            s += abs(c[k]) * p
            p *= th
        return s


def _series_length(m: int) -> int:
    # The series of log T_m converges inside the smallest root of T_m, whose
    # modulus grows roughly linearly in m; theta_m sits well inside it.  The
    # length below keeps the dropped tail many orders under tol (checked by
    # comparing two lengths in the tests).
    return m + 600


@functools.lru_cache(maxsize=None)
def theta(m: int, tol: float = TOL_DOUBLE) -> float:
    """theta_m for unit roundoff tol, by bisection on the monotone ratio."""
    if m < 1:
        raise ValueError("m >= 1")
    K = _series_length(m)
    lo, hi = 0.0, 1.0
    while backward_error_ratio(m, hi, K) <= tol:
        lo, hi = hi, 2.0 * hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if backward_error_ratio(m, mid, K) <= tol:
            lo = mid
        else:
            hi = mid
    return lo


@functools.lru_cache(maxsize=None)
def theta_table(tol: float = TOL_DOUBLE, m_max: int = M_MAX) -> tuple:
    """(theta_1, ..., theta_{m_max}) as Python floats; index m-1."""
    return tuple(theta(m, tol) for m in range(1, m_max + 1))
