"""The launch-configuration autotuner: any choice leaves results bitwise
unchanged, and a second handle with the same key reuses the first tuning."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, gpu_run, random_workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [lambda: workloads.er256(),
                                  lambda: random_workload(41, 4, 0.45, 91, n_steps=4, dt=0.6)])
def test_autotune_keeps_results_and_caches(make):
    wl = make()
    wl.n_steps = min(wl.n_steps, 6)
    before, op = gpu_run(wl)
    t = op.autotune()
    assert t["grid"] >= 1 and t["us_per_product"] > 0
    after, _ = gpu_run(wl, op)
    assert np.array_equal(before, after)
    op2 = build_gpu(wl)
    assert op2.autotune()["from_cache"]
    again, _ = gpu_run(wl, op2)
    assert np.array_equal(before, again)
    op.close()
    op2.close()


def test_autotune_single_precision():
    wl = workloads.er256()
    wl.n_steps = 4
    op = build_gpu(wl)
    op.set_precision(True)
    before, _ = gpu_run(wl, op)
    op.autotune()
    after, _ = gpu_run(wl, op)
    assert np.array_equal(before, after)
    op.close()
