"""The products with L^dagger that ||L||_1 and the 1-norm estimator need go
through the phase-split layout of L for walks with a real H: off the rows
(a, a) a row of L^dagger is the row of L with its Hamiltonian (imaginary)
entries negated and its diagonal conjugated, and a row (a, a) trades the
population transfers of L (omega R_aj on rho_jj) for the transposed ones
(omega R_ja).  No CSR or layout of L^dagger is then built.  ||L||_1 is the
same bit for bit as from the assembled L^dagger (QSW_ADJ_LAYOUT=1), and so
are the estimates, their unit columns and probe columns; a walk with a
complex H keeps the assembled L^dagger."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu

PS = range(2, 10)


def _info(monkeypatch, make, layout):
    if layout:
        monkeypatch.setenv("QSW_ADJ_LAYOUT", "1")
    op = make()
    monkeypatch.delenv("QSW_ADJ_LAYOUT", raising=False)
    inf = op.info()
    op.close()
    return (inf["norm1"], [inf["d"][p] for p in PS], [inf["d_index"][p] for p in PS],
            [inf["d_probe"][p] for p in PS], inf["norm_products"], inf["split"])


def _channels():
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(972))
    g = workloads.random_out_degree(40, 3, rng)
    return qsw.Superop.from_channels(g, 0.6, [(0, 1.5), (3, 0.4)], [(5, 2.0), (9, 0.7)])


def _operators(imag):
    """LQSW(omega, H, M_L) with a random real (or complex) Hermitian H and a
    random nonnegative M_L, plus channels outside omega."""
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(973 + imag))
    N = 33
    A = (rng.random((N, N)) < 0.15) * rng.random((N, N))
    H = A + A.T
    if imag:
        B = (rng.random((N, N)) < 0.1) * rng.random((N, N))
        H = H + 1j * (B - B.T)
    M = (rng.random((N, N)) < 0.12) * rng.random((N, N))
    F = np.zeros((N, N))
    F[4, 7] = 0.9
    return qsw.Superop.from_operators(H, M, 0.45, M_free=F)


CASES = {
    "cycle16": lambda: build_gpu(workloads.cycle16()),
    "rand2": lambda: build_gpu(random_workload(2, 1, 0.5, 7)),
    "rand9_dephasing": lambda: build_gpu(random_workload(9, 3, 0.6, 5, dephasing=True)),
    "rand37_colnorm": lambda: build_gpu(random_workload(37, 4, 0.3, 971, r_mode="colnorm",
                                                        dephasing=True)),
    "rand300_omega1": lambda: build_gpu(random_workload(300, 5, 1.0, 811)),
    "rand512_colnorm": lambda: build_gpu(random_workload(512, 4, 0.7, 812, r_mode="colnorm",
                                                         dephasing=True)),
    "er256": lambda: build_gpu(workloads.er256()),
    "outdeg1024": lambda: build_gpu(workloads.outdeg1024()),
    "channels": _channels,
    "operators_real_h": lambda: _operators(0),
    "operators_complex_h": lambda: _operators(1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_through_forward_layout_changes_nothing(monkeypatch, case):
    assembled = _info(monkeypatch, CASES[case], True)
    through = _info(monkeypatch, CASES[case], False)
    assert through == assembled, (case, through, assembled)
    assert np.isfinite(through[0]) and through[0] > 0.0
    print(f"{case}: ||L||_1 {through[0]!r}, d_2..9 {[round(x, 6) for x in through[1]]}, "
          f"products {through[4]}", flush=True)
