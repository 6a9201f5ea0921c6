"""Oracle: parameter selection and the time-grid drivers (step / series).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file.

The paper's `step` and `series` (Section 3.1) are Al-Mohy and Higham's
single-time algorithm and time-series algorithm, without balancing and
without the trace shift.  This module restates them:

* ``select_params``      - the choice of Taylor degree m* and scaling s from
  the 1-norm of tA, or from alpha_p(tA) = max(d_p, d_{p+1}) t with
  d_p = ||A^p||_1^(1/p) when ||tA||_1 is large (their condition 3.13).
* ``select_params_norm1``- the same choice using ||tA||_1 only.  Every
  alpha_p is at most ||A||_1, so this choice satisfies the same backward-error
  bound; it can only cost more products.  The oracle itself always uses it.
* ``expmv``              - exp(tA) b by one application of the single-time
  algorithm with the exact ||A||_1.
* ``propagate``          - rho(t0 + k dt), k = 0..n_steps: exp(t0 A) rho0 and
  then one single-time application per interval.  This is the plain
  definition of the grid (each point is exp(dt A) of the previous one).
* ``series``             - the time-series algorithm, with its reuse of the
  powers K_p = (h^p/p!) A^p Z across the points of a block, for small n.
* ``propagate_single_values`` - the reduced-storage variant: the same grid
  with every stored value of A rounded to complex64, theta_m and the stopping
  test at u = 2^-24 (Al-Mohy and Higham's single-precision choice), the
  1-norm and all vector arithmetic in double.
* ``propagate_fp32_products`` - the single-precision-products variant: values,
  terms and their products in complex64 (each term's row sums accumulated in
  complex64, scaled in double and rounded once), the accumulator exact (in
  double), the Taylor degree at most 20, u = 2^-24, and each output point
  scaled back to the input's trace.  It shows what that arithmetic costs in
  accuracy, so the GPU's single-precision path can be held to it.
"""
from __future__ import annotations

import math

import numpy as np

from . import native
from .theta import M_MAX, P_MAX, TOL_DOUBLE, TOL_SINGLE, theta_table


M_MAX_FP32 = 20     # Taylor degree cap of the single-precision products
P_MAX_FP32 = 5      # largest p with p(p-1)-1 <= 20


def select_params_norm1(norm_tA: float, thetas=None, m_max: int = M_MAX):
    """m* = smallest m minimising m * ceil(||tA||_1 / theta_m);
    s = ceil(||tA||_1 / theta_{m*}).  tA = 0 gives (0, 1)."""
    if thetas is None:
        thetas = theta_table()
    if norm_tA == 0.0:
        return 0, 1
    best_m, best_cost = None, None
    for m in range(1, m_max + 1):
        cost = m * math.ceil(norm_tA / thetas[m - 1])
        if best_cost is None or cost < best_cost:
            best_m, best_cost = m, cost
    s = max(1, math.ceil(norm_tA / thetas[best_m - 1]))
    return best_m, s


def condition_3_13(norm_tA: float, n0: int = 1, ell: int = 2,
                   thetas=None, m_max: int = M_MAX, p_max: int = P_MAX) -> bool:
    """||tA||_1 <= 2 ell p_max (p_max + 3) theta_{m_max} / (n0 m_max):
    the 1-norm alone is then used (estimating the d_p would cost more
    products than it can save)."""
    if thetas is None:
        thetas = theta_table()
    return norm_tA <= 2 * ell * p_max * (p_max + 3) * thetas[m_max - 1] / (n0 * m_max)


def select_params(norm1_A: float, d: dict, t: float, n0: int = 1, ell: int = 2,
                  thetas=None, m_max: int = M_MAX, p_max: int = P_MAX, switch: bool = True):
    """Full choice for tA given ||A||_1 and d[p] = ||A^p||_1^(1/p),
    p = 2..p_max+1.  Minimises m * ceil(alpha_p / theta_m) over
    2 <= p <= p_max and p(p-1)-1 <= m <= m_max, smallest m on ties.  With
    switch=False the alpha_p rule applies for every t (the norms are known
    already, so condition 3.13's saving does not arise)."""
    if thetas is None:
        thetas = theta_table()
    t = abs(t)
    norm_tA = t * norm1_A
    if norm_tA == 0.0:
        return 0, 1
    if switch and condition_3_13(norm_tA, n0, ell, thetas, m_max, p_max):
        return select_params_norm1(norm_tA, thetas, m_max)
    best = None  # (cost, m, s)
    for m in range(1, m_max + 1):
        s_m = None
        for p in range(2, p_max + 1):
            if p * (p - 1) - 1 > m:
                continue
            alpha = t * max(d[p], d[p + 1])
            s_p = math.ceil(alpha / thetas[m - 1])
            if s_m is None or s_p < s_m:
                s_m = s_p
        if s_m is None:
            continue
        cost = m * s_m
        if best is None or cost < best[0]:
            best = (cost, m, max(s_m, 1))
    return best[1], best[2]


def expmv(A: native.CSR, b: np.ndarray, t: float, tol: float = TOL_DOUBLE,
          norm1: float | None = None):
    """exp(tA) b; returns (result, (m, s), number of products)."""
    if norm1 is None:
        norm1 = A.norm1()
    m, s = select_params_norm1(abs(t) * norm1)
    F, k = native.taylor_expmv(A, b, t, m, s, tol)
    return F, (m, s), k


def propagate(A: native.CSR, rho0: np.ndarray, t0: float, dt: float,
              n_steps: int, tol: float = TOL_DOUBLE):
    """out[k] = exp((t0 + k dt) A) vec(rho0), k = 0..n_steps (row-major vec).
    Returns (out[n_steps+1, N, N], info)."""
    N = rho0.shape[0]
    norm1 = A.norm1()
    x = np.ascontiguousarray(rho0, np.complex128).reshape(-1)
    products = 0
    if t0 != 0.0:
        x, _, k = expmv(A, x, t0, tol, norm1)
        products += k
    out = np.empty((n_steps + 1, N * N), np.complex128)
    out[0] = x
    m, s = select_params_norm1(abs(dt) * norm1)
    for k in range(1, n_steps + 1):
        x, kk = native.taylor_expmv(A, x, dt, m, s, tol)
        products += kk
        out[k] = x
    return out.reshape(n_steps + 1, N, N), {"m": m, "s": s, "norm1": norm1,
                                            "products": products}


def series(A: native.CSR, rho0: np.ndarray, t0: float, tq: float, q: int,
           tol: float = TOL_DOUBLE):
    """The time-series algorithm on the grid t0 + k h, h = (tq - t0)/q.

    With (m*, s) chosen for (tq - t0) A: if q <= s each interval is one
    single-time application for hA; otherwise the points are taken in blocks
    of d = floor(q/s) steps from the block start Z, reusing the vectors
    K_p = (h/p) A K_{p-1} (K_0 = Z) so that point k of the block is
    sum_p k^p K_p, summed until the same two-term test as the single-time
    algorithm passes.
    """
    N = rho0.shape[0]
    norm1 = A.norm1()
    x = np.ascontiguousarray(rho0, np.complex128).reshape(-1)
    if t0 != 0.0:
        x, _, _ = expmv(A, x, t0, tol, norm1)
    h = (tq - t0) / q
    out = np.empty((q + 1, N * N), np.complex128)
    out[0] = x
    m, s = select_params_norm1(abs(tq - t0) * norm1)
    if q <= s:
        mh, sh = select_params_norm1(abs(h) * norm1)
        for k in range(1, q + 1):
            x, _ = native.taylor_expmv(A, x, h, mh, sh, tol)
            out[k] = x
        return out.reshape(q + 1, N, N), {"branch": "q<=s", "m": mh, "s": sh}
    d = q // s
    j = q // d
    r = q - d * j
    Z = x
    for i in range(1, j + 2):
        dd = d if i <= j else r
        if dd == 0:
            break
        Ks = [Z]
        for k in range(1, dd + 1):
            F = Z.copy()
            c1 = np.max(np.abs(Z))
            for p in range(1, m + 1):
                if p >= len(Ks):
                    Ks.append((h / p) * A.matvec(Ks[p - 1]))
                term = float(k) ** p * Ks[p]
                F = F + term
                c2 = np.max(np.abs(term))
                if c1 + c2 <= tol * np.max(np.abs(F)):
                    break
                c1 = c2
            out[(i - 1) * d + k] = F
        Z = out[(i - 1) * d + dd]
    return out.reshape(q + 1, N, N), {"branch": "q>s", "m": m, "s": s, "d": d}


def round_values_c64(A: native.CSR) -> native.CSR:
    """A with each real and imaginary part rounded to the nearest float32."""
    return native.CSR(A.n, A.row_ptr, A.col, A.val.astype(np.complex64).astype(np.complex128))


def propagate_single_values(A: native.CSR, rho0: np.ndarray, t0: float, dt: float,
                            n_steps: int):
    """out[k] = rho(t0 + k dt) through A rounded to complex64 values, with the
    single-precision theta table and tolerance.  (m, s) come from ||tA||_1 of
    the unrounded A, as in ``propagate``."""
    N = rho0.shape[0]
    norm1 = A.norm1()
    thetas = theta_table(TOL_SINGLE)
    A32 = round_values_c64(A)
    x = np.ascontiguousarray(rho0, np.complex128).reshape(-1)
    products = 0
    if t0 != 0.0:
        m0, s0 = select_params_norm1(abs(t0) * norm1, thetas)
        x, k = native.taylor_expmv(A32, x, t0, m0, s0, TOL_SINGLE)
        products += k
    out = np.empty((n_steps + 1, N * N), np.complex128)
    out[0] = x
    m, s = select_params_norm1(abs(dt) * norm1, thetas)
    for k in range(1, n_steps + 1):
        x, kk = native.taylor_expmv(A32, x, dt, m, s, TOL_SINGLE)
        products += kk
        out[k] = x
    return out.reshape(n_steps + 1, N, N), {"m": m, "s": s, "norm1": norm1,
                                            "products": products}


def single_values_bound(norm1: float, t: float, rho0: np.ndarray) -> float:
    """First-order bound on ||vec rho_single(t) - vec rho(t)||_1 (and so on the
    largest element error): rounding the values perturbs A by at most
    u ||A||_1 in the 1-norm, and truncating at the 2^-24 test adds a backward
    error of at most u ||tA||_1; with a semigroup of 1-norm at most one the
    two give 2 u |t| ||A||_1 ||vec rho0||_1."""
    return 2.0 * TOL_SINGLE * abs(t) * norm1 * float(np.abs(rho0).sum())


def _fp32_matvec(A32, x32: np.ndarray, alpha: float) -> np.ndarray:
    """round32(alpha * (A32 x32)) with the row sums in complex64 (scipy's CSR
    product accumulates in the operands' type, in storage order)."""
    y = A32 @ x32
    assert y.dtype == np.complex64
    return (alpha * y.astype(np.complex128)).astype(np.complex64)


def _fp32_taylor(A32, F: np.ndarray, t: float, m: int, s: int, tol: float):
    """T_m(tA/s)^s F with complex64 terms and an exact (double) accumulator;
    the stopping test of the single-time algorithm in double."""
    products = 0
    for _ in range(s):
        c1 = np.max(np.abs(F))
        b = F.astype(np.complex64)
        G = F.copy()
        for j in range(1, m + 1):
            b = _fp32_matvec(A32, b, t / (s * j))
            products += 1
            c2 = np.max(np.abs(b.astype(np.complex128)))
            G = G + b.astype(np.complex128)
            if c1 + c2 <= tol * np.max(np.abs(G)):
                break
            c1 = c2
        F = G
    return F, products


def propagate_fp32_products(A: native.CSR, rho0: np.ndarray, t0: float, dt: float,
                            n_steps: int):
    """rho(t0 + k dt), k = 0..n_steps, with single-precision values, terms and
    products (see the module header).  (m, s) from ||tA||_1 of the unrounded
    A with the single-precision theta table and m <= 20."""
    import scipy.sparse
    N = rho0.shape[0]
    norm1 = A.norm1()
    thetas = theta_table(TOL_SINGLE)
    A32 = scipy.sparse.csr_matrix((A.val.astype(np.complex64), A.col, A.row_ptr),
                                  shape=(A.n, A.n))
    x = np.ascontiguousarray(rho0, np.complex128).reshape(-1)
    diag = np.arange(N) * (N + 1)
    tr0 = float(x[diag].real.sum())
    products = 0

    def renormalise(v):
        tr = float(v[diag].real.sum())
        if tr != 0.0 and tr0 != 0.0 and abs(tr - tr0) <= 2.0 ** -10 * abs(tr0):
            return v * (tr0 / tr)
        return v

    if t0 != 0.0:
        m0, s0 = select_params_norm1(abs(t0) * norm1, thetas, M_MAX_FP32)
        x, k = _fp32_taylor(A32, x, t0, m0, s0, TOL_SINGLE)
        x = renormalise(x)
        products += k
    out = np.empty((n_steps + 1, N * N), np.complex128)
    out[0] = x
    m, s = select_params_norm1(abs(dt) * norm1, thetas, M_MAX_FP32)
    for k in range(1, n_steps + 1):
        x, kk = _fp32_taylor(A32, x, dt, m, s, TOL_SINGLE)
        x = renormalise(x)
        products += kk
        out[k] = x
    return out.reshape(n_steps + 1, N, N), {"m": m, "s": s, "norm1": norm1,
                                            "products": products}


def fp32_products_bound(norm1: float, t: float, steps: int, theta: float, r_max: int,
                        vec1: float) -> float:
    """First-order bound on max |rho_fp32(t) - rho(t)| for the single-precision
    products, u = 2^-24:

        u [ 2 |t| ||A||_1 + (r_max + 2) steps e^theta ] vec1

    * rounding the values perturbs A by at most u ||A||_1 and truncating at u
      adds a backward error of at most u ||tA||_1 (2 u |t| ||A||_1 together);
    * one scaling step of degree m sums terms b_j with sum_j ||b_j||_1 <=
      e^theta ||b_0||_1 (theta = ||A||_1 |t_step| / s); each term's row sums of
      at most r_max products, its scaling and its rounding add at most
      (r_max + 2) u of its size; the two-float accumulator adds O(u^2);
    * the evolution is completely positive and trace preserving, so it does
      not increase the trace norm of an error, and |X_ab| <= ||X||_tr <=
      ||vec X||_1: errors made at any step reach rho(t) at most as large;
    * vec1 bounds ||vec rho||_1 of the states along the way (the caller takes
      it from the oracle's double-precision solution)."""
    u = TOL_SINGLE
    return u * (2.0 * abs(t) * norm1 + (r_max + 2) * steps * math.exp(theta)) * vec1
