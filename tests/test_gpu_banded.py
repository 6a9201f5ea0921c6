"""The XCD-banded traversal (each of the 8 XCDs takes one band of columns of
rho for the rho H gathers) changes only the order in which rows are visited,
so its results equal the default staged engine's bit for bit.  It is taken
when QSW_BANDS=1 is set at build time and the rho-row fits the LDS stage
(N = 512, 1024 or 2048)."""
import numpy as np
import pytest

from tests.gpu_util import build_gpu, gpu_run, random_workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,k,single", [(512, 6, False), (1024, 4, False), (1024, 4, True),
                                        (2048, 2, False)])
def test_banded_matches_staged(monkeypatch, N, k, single):
    wl = random_workload(N, k, 0.4, 700 + N, n_steps=2, dt=0.5)
    monkeypatch.delenv("QSW_BANDS", raising=False)
    op = build_gpu(wl)
    if single:
        op.set_precision(True)
    ref, _ = gpu_run(wl, op)
    op.close()
    monkeypatch.setenv("QSW_BANDS", "1")
    opb = build_gpu(wl)
    if single:
        opb.set_precision(True)
    got, _ = gpu_run(wl, opb)
    opb.close()
    assert np.isfinite(ref).all()
    assert np.array_equal(ref, got)
