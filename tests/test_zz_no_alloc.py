"""qsw_propagate_noalloc (static device scratch, no allocation) against
qsw_propagate (caller workspace) through the C ABI: the same kernels in the
same order, so the results are bitwise equal.  Two calls in a row, the second
on a smaller operator, and a call whose plan does not fit the scratch."""
import ctypes

import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu


def _noalloc(op, rho0, t0, dt, n_steps):
    import torch
    from paper_2003_02450_amd import _lib
    L = _lib.load()
    r = torch.from_numpy(np.ascontiguousarray(rho0, np.complex128)).cuda()
    out = torch.full((n_steps + 1, op.N, op.N), float("nan"), dtype=torch.complex128,
                     device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.qsw_propagate_noalloc(op._h, ctypes.c_void_p(r.data_ptr()), float(t0), float(dt),
                                 int(n_steps), ctypes.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    return st, out.cpu().numpy()


def _reference(op, wl):
    import torch
    out = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_workspace_path_twice_then_smaller():
    from paper_2003_02450_amd import _lib
    cases = [random_workload(41, 4, 0.45, 61, n_steps=5, dt=0.6, t0=0.4),   # larger first
             random_workload(13, 3, 0.8, 62, n_steps=7, dt=0.9)]            # then smaller
    for wl in cases:
        op = build_gpu(wl)
        print(f"noalloc: N={wl.graph.N} steps={wl.n_steps}", flush=True)
        ref = _reference(op, wl)
        assert op.workspace_bytes(wl.t0, wl.dt, wl.n_steps) <= _lib.NOALLOC_SCRATCH_BYTES
        st, got = _noalloc(op, wl.rho0, wl.t0, wl.dt, wl.n_steps)
        assert st == 0, _lib.STATUS_NAMES.get(st, st)
        assert np.array_equal(got, ref)
        stats = op.last_stats()
        assert stats["products"] > 0 and not stats["nonfinite"]
        op.close()


def test_noalloc_series_branch_and_benchmark_size():
    from paper_2003_02450_amd import _lib
    wl = workloads.cycle16()                 # time-series branch (stored powers)
    op = build_gpu(wl)
    ref = _reference(op, wl)
    assert op.last_stats()["branch"] == 1
    st, got = _noalloc(op, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    assert st == 0 and np.array_equal(got, ref)
    op.close()
    wl = workloads.outdeg1024(n_steps=2)     # N = 1024: four 16 MiB vectors fit
    op = build_gpu(wl)
    print("noalloc: outdeg1024, 2 steps", flush=True)
    ref = _reference(op, wl)
    st, got = _noalloc(op, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    assert st == 0 and np.array_equal(got, ref)
    op.close()


def test_noalloc_rejects_a_plan_beyond_the_scratch():
    from paper_2003_02450_amd import _lib
    wl = workloads.outdeg1024(n_steps=50)
    wl.dt = 0.02                             # q > s: m stored powers of 16 MiB each
    op = build_gpu(wl)
    need = op.workspace_bytes(wl.t0, wl.dt, wl.n_steps)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    st, got = _noalloc(op, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    assert _lib.STATUS_NAMES[st] == "QSW_ERR_SCRATCH"
    assert np.isnan(got).all()               # nothing was enqueued
    op.close()
