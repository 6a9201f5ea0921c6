"""The 1-norm estimates of ||L^p||_1 (p = 2..9, Section 4 footnote) with the
power chains of several p merged into one pass over the matrix per step equal
those of one estimate at a time, bit for bit: the same products in the same
order, the same decisions.  Groups of 8 (all at once), 3 (8 = 3 + 3 + 2) and
1 (one at a time) are compared, in the phase-split and the complex layouts.
One estimate at a time keeps its unit-column chains for later estimates that
start from the same unit pair; with and without that the estimates are the
same, bit for bit, and it saves products on the 1024-vertex operator."""
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
        # estimates bit for bit; one at a time may take kept unit chains
        assert got[:3] == one[:3] and got[4] == one[4], (case, chains, got, one)
        assert one[3] <= got[3]
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
    assert got[:3] == one[:3] and one[3] <= got[3]
    # and the complex layout's estimates are the phase-split layout's
    assert _estimates(monkeypatch, make, 8)[:4] == got[:4]


@pytest.mark.parametrize("case", ["rand300", "rand512_colnorm", "er256", "outdeg1024"])
def test_kept_unit_chains_change_no_estimate(monkeypatch, case):
    """One estimate at a time with and without its kept unit-column chains
    (QSW_EST_SHARE=0 turns them off): the same estimates, bit for bit."""
    wl = CASES[case]()
    make = lambda: build_gpu(wl)  # noqa: E731
    kept = _estimates(monkeypatch, make, 1)
    monkeypatch.setenv("QSW_EST_SHARE", "0")
    plain = _estimates(monkeypatch, make, 1)
    monkeypatch.delenv("QSW_EST_SHARE")
    assert kept[:3] == plain[:3] and kept[4] == plain[4], (case, kept, plain)
    assert kept[3] <= plain[3]
    if case == "outdeg1024":
        # three pairs of powers start their second iteration from the same
        # unit pair (two of them with the columns exchanged)
        assert kept[3] < plain[3]
    print(f"{case}: products {kept[3]} with kept unit chains, {plain[3]} without", flush=True)
