"""Launch pacing: with a lookahead, qsw_propagate enqueues no further Taylor
terms of a scaling step once the device has reported that the step passed
its stopping test.  The terms it leaves out would have exited at once, so
the results are bitwise those of the unpaced call, with the same computed
products and fewer launches."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu


def _run(op, wl):
    import torch
    out = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), op.last_stats()


@pytest.mark.parametrize("lookahead", [1, 3, 16])
@pytest.mark.parametrize("case", ["er256", "rand512_t0", "rand300_single"])
def test_paced_equals_unpaced(case, lookahead):
    # one grid interval: always the single-time branch (paced)
    if case == "er256":
        wl = workloads.er256()
        wl.n_steps, wl.dt = 1, 6.0
    elif case == "rand512_t0":
        wl = random_workload(512, 6, 0.6, 820, n_steps=1, dt=2.0, t0=0.5)
    else:
        wl = random_workload(300, 4, 0.3, 821, n_steps=1, dt=3.0)
    op = build_gpu(wl)
    if case == "rand300_single":
        op.set_precision(True)
    ref, st0 = _run(op, wl)
    op.set_pacing(lookahead)
    got, st1 = _run(op, wl)
    again, st2 = _run(op, wl)
    op.set_pacing(0)
    off, st3 = _run(op, wl)
    assert st0["branch"] == 0
    for x, st in ((got, st1), (again, st2), (off, st3)):
        assert np.array_equal(x, ref)
        assert st["products"] == st0["products"]
    # never more launches than unpaced, at least the computed products; with
    # a short lookahead, fewer (a long one may cover what a step leaves)
    for st in (st1, st2):
        assert st0["products"] <= st["launched"] <= st0["launched"]
        if lookahead <= 3:
            assert st["launched"] < st0["launched"], (lookahead, st0["m"])
    assert st3["launched"] == st0["launched"]
    op.close()


def test_pacing_survives_set_omega():
    wl = random_workload(256, 5, 0.4, 822, n_steps=1, dt=2.5)
    op = build_gpu(wl)
    op.set_pacing(2)
    op.set_omega(0.7)
    got, st = _run(op, wl)
    fresh = build_gpu(random_workload(256, 5, 0.7, 822, n_steps=1, dt=2.5))
    ref, st0 = _run(fresh, wl)
    assert np.array_equal(got, ref)
    assert st["launched"] < st0["launched"] and st["products"] == st0["products"]
    op.close()
    fresh.close()
