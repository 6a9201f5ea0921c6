"""The 1-norm estimates of ||L^p||_1 (p = 2..9, Section 4 footnote) with the
power chains of several p merged into one pass over the matrix per step equal
those of one estimate at a time, bit for bit: the same products in the same
order, the same decisions.  Groups of 8 (all at once), 3 (8 = 3 + 3 + 2) and
1 (one at a time) are compared, in the phase-split and the complex layouts."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu


def _estimates(monkeypatch, make, chains, split=True):
    monkeypatch.setenv("QSW_EST_CHAINS", str(chains))
    if not split:
        monkeypatch.setenv("QSW_SPLIT", "0")
    op = make()
    monkeypatch.delenv("QSW_EST_CHAINS", raising=False)
    monkeypatch.delenv("QSW_SPLIT", raising=False)
    inf = op.info()
    op.close()
    ps = range(2, 10)
    return ([inf["d"][p] for p in ps], [inf["d_index"][p] for p in ps],
            [inf["d_probe"][p] for p in ps], inf["norm_products"], inf["split"])


CASES = {
    "cycle16": workloads.cycle16,
    "rand9_dephasing": lambda: random_workload(9, 3, 0.6, 5, dephasing=True),
    "rand2": lambda: random_workload(2, 1, 0.5, 7),
    "rand300": lambda: random_workload(300, 5, 0.3, 811),
    "rand512_colnorm": lambda: random_workload(512, 4, 0.7, 812, r_mode="colnorm",
                                               dephasing=True),
    "er256": workloads.er256,
    "outdeg1024": workloads.outdeg1024,
}


@pytest.mark.parametrize("case", list(CASES))
def test_merged_chains_equal_one_at_a_time(monkeypatch, case):
    wl = CASES[case]()
    make = lambda: build_gpu(wl)  # noqa: E731
    one = _estimates(monkeypatch, make, 1)
    for chains in (3, 8):
        got = _estimates(monkeypatch, make, chains)
        assert got == one, (case, chains, got, one)
    d = one[0]
    assert all(np.isfinite(d)) and all(x >= 0 for x in d)
    print(f"{case}: d_2..9 = {[round(x, 6) for x in d]}, products {one[3]}", flush=True)


@pytest.mark.parametrize("case", ["rand300", "er256"])
def test_merged_chains_complex_layout(monkeypatch, case):
    wl = CASES[case]()
    make = lambda: build_gpu(wl)  # noqa: E731
    one = _estimates(monkeypatch, make, 1, split=False)
    got = _estimates(monkeypatch, make, 8, split=False)
    assert not one[4] and not got[4]
    assert got == one
    # and the complex layout's estimates are the phase-split layout's
    assert _estimates(monkeypatch, make, 8)[:4] == one[:4]
