"""Time-series blocks of one grid point (d = 1) run through the fused
single-time kernels with (m, 1) per interval: the same powers, sums, tests
and order as the stored-power kernels, so the results are bitwise those of
QSW_FUSE_SERIES=0, in both precisions, paced or not."""
import numpy as np
import pytest

import paper_2003_02450_amd as qsw
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu


def _one_point_blocks(op, single):
    """(n_steps, dt) for which the series branch takes d = 1 (s < q < 2 s):
    q/s is about theta_m / (dt alpha), so a dt in the right range is looked
    for along with q."""
    info = op.info()
    for dt in (0.35, 0.5, 0.7, 1.0, 1.4, 2.0, 2.8, 4.0, 0.25, 0.18, 0.12):
        for q in range(3, 60):
            m, s = qsw.select_params(info["norm1"], info["d"], q * dt, single=single,
                                     known_norms=True)
            if s < q < 2 * s:
                return q, dt
    raise AssertionError("no one-point block split for this operator")


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("pace", [0, 2])
def test_one_point_blocks_fused(monkeypatch, single, pace):
    wl = random_workload(256, 5, 0.45, 830, dt=0.35)
    op = build_gpu(wl)
    op.set_precision(single)
    op.set_pacing(pace)
    wl.n_steps, wl.dt = _one_point_blocks(op, single)
    import torch
    monkeypatch.setenv("QSW_FUSE_SERIES", "0")
    ref = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    st0 = op.last_stats()
    monkeypatch.delenv("QSW_FUSE_SERIES", raising=False)
    got = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    st1 = op.last_stats()
    torch.cuda.synchronize()
    assert st0["branch"] == 1 and st1["branch"] == 1
    assert np.isfinite(got).all()
    assert np.array_equal(got, ref)
    assert st1["products"] == st0["products"]
    op.close()
