"""Oracle: dense matrix exponential for tiny superoperators.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file.

exp(A) is its Taylor series (Section 3.1, first equation).  For a dense A of
a few hundred rows it is evaluated by the scaling relation exp(A) =
exp(A / 2^j)^(2^j): the series of A / 2^j with ||A / 2^j||_1 <= 1/2 is summed
until the next term cannot change the sum, then squared j times.  Matrix
products are numpy's.
"""
from __future__ import annotations

import math

import numpy as np


def expm(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    nrm = np.abs(A).sum(axis=0).max() if n else 0.0
    j = 0 if nrm <= 0.5 else int(math.ceil(math.log2(nrm / 0.5)))
    B = A / (2.0 ** j)
    E = np.eye(n, dtype=np.complex128)
    T = np.eye(n, dtype=np.complex128)
    for k in range(1, 200):
        T = T @ B / k
        E_next = E + T
        if np.array_equal(E_next, E):
            break
        E = E_next
    for _ in range(j):
        E = E @ E
    return E


def expm_apply(A: np.ndarray, v: np.ndarray, t: float) -> np.ndarray:
    return expm(t * np.asarray(A)) @ v
