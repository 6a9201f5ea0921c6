"""CPU FP64 oracle for the L-QSW propagator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.
It shares no code with the GPU path: it has its own operator construction,
its own superoperator assembly (plain C, ``qsw_oracle.c``), its own theta_m
constants (``theta.py``), its own parameter selection and drivers
(``expmv.py``) and a dense brute-force path (``operators.superop_kron`` +
``dense.expm``) for tiny graphs.

Pins (each checked by the CPU tests):
* superop_kron (explicit Kronecker products, one L_k at a time) == the
  sparse analytic rows of qsw_oracle.c, N <= 16;
* dense.expm against closed forms and against scipy.linalg.expm;
* theta_m against the definition at two series lengths and against the
  published magnitudes of Al-Mohy and Higham's table;
* the omega = 0 closed form (CTQW and Liouville-von Neumann, Sections 2.3-2.4),
  the omega = 1 classical limit (CTRW, Section 2.2), the paper's printed
  three-vertex results (Section 4), density-matrix invariants (Section 2.4),
  the maximally mixed fixed point on regular graphs (Section 4), step vs
  series agreement (Section 5), and scipy's expm_multiply.
"""
from . import dense, expmv, native, operators, theta  # noqa: F401
from .native import CSR, superop_csr  # noqa: F401


def walk_superop(graph_dense, omega, h_mode="laplacian", r_mode="transition",
                 dephasing=False, gamma=1.0) -> "CSR":
    """Graph (dense, row = target) -> row-major CSR of the generator."""
    H, ML = operators.walk_operators(graph_dense, h_mode, r_mode, dephasing, gamma)
    return superop_csr(H, ML, omega)


def run_workload(wl, n_steps=None):
    """rho(t0 + k dt) for a workloads.Workload; out[k] is N x N row-major."""
    A = walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                     wl.dephasing, wl.gamma)
    steps = wl.n_steps if n_steps is None else n_steps
    return expmv.propagate(A, wl.rho0, wl.t0, wl.dt, steps)


def dense_csr(S):
    """Dense row-major generator -> oracle CSR (explicit zeros dropped)."""
    import numpy as np
    n = S.shape[0]
    rows, cols = np.nonzero(S)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return CSR(n, rp, cols.astype(np.int32), S[rows, cols])


def general_superop(H, Ls, omega, H_rot=None, Ls_free=()) -> "CSR":
    """Explicit operators (G-QSW, NM-G-QSW, channels) -> row-major CSR,
    through the dense Kronecker form (small N only)."""
    return dense_csr(operators.general_rowmajor(H, Ls, omega, H_rot, Ls_free))


def channel_superop(graph_dense, omega, sources, sinks, h_mode="laplacian",
                    r_mode="transition", dephasing=False, gamma=1.0) -> "CSR":
    """A walk on the augmented digraph (Section 2.5.1): the graph's H and
    L_k (omega-scaled) padded with the source and sink vertices, plus the
    channels outside omega.  Dense (small N only)."""
    import numpy as np
    Ga, chans = operators.augmented(np.asarray(graph_dense, float), sources, sinks)
    H, ML = operators.walk_operators(Ga, h_mode, r_mode, dephasing, gamma)
    Ls = operators.lindblad_ops(ML)
    return general_superop(H, Ls, omega, None, chans)
