"""Single-precision products (QSW_PREC_FP32) on the GPU.

Each result is compared with the FP64 oracle at every grid point, against two
bars:
* the first-order bound of ``oracle.expmv.fp32_products_bound`` (value
  rounding and the 2^-24 truncation, plus (r_max + 2) u e^theta per scaling
  step for the single-precision terms, carried by the trace-norm contraction
  of the evolution);
* ten times the error of the oracle's own single-precision-products variant
  (same arithmetic precision, rounded in its own order) on the same input, so
  that the GPU path is no less accurate than the method it implements.
Each output point keeps the input's trace (the FP64 trace check), and the
double path is untouched by switching precision.
"""
import numpy as np
import pytest

import workloads
from oracle import expmv
from oracle import theta as otheta
from tests.gpu_util import build_gpu, oracle_superop, random_workload

pytestmark = pytest.mark.gpu

THETA20 = otheta.theta_table(otheta.TOL_SINGLE)[expmv.M_MAX_FP32 - 1]


def _run(op, wl):
    import torch
    out = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _steps(norm1, t0, s, k):
    s0 = 0
    if t0 != 0.0:
        th = otheta.theta_table(otheta.TOL_SINGLE)
        s0 = expmv.select_params_norm1(abs(t0) * norm1, th, expmv.M_MAX_FP32)[1]
    return max(1, k * s + s0)


def _check(wl, emulate=True):
    A = oracle_superop(wl)
    ref, info = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    op = build_gpu(wl)
    op.set_precision("fp32")
    got = _run(op, wl)
    st = op.last_stats()
    assert st["prec"] == "fp32" and st["branch"] == 0 and st["m"] <= 20
    rmax = int(np.diff(A.row_ptr).max())
    vec1 = max(float(np.abs(ref[k]).sum()) for k in range(wl.n_steps + 1))
    tr0 = np.trace(wl.rho0).real
    err = np.abs(got - ref).reshape(wl.n_steps + 1, -1).max(axis=1)
    s = expmv.select_params_norm1(abs(wl.dt) * info["norm1"],
                                  otheta.theta_table(otheta.TOL_SINGLE), expmv.M_MAX_FP32)[1]
    for k in range(wl.n_steps + 1):
        t = wl.t0 + k * wl.dt
        b = expmv.fp32_products_bound(info["norm1"], t, _steps(info["norm1"], wl.t0, s, k),
                                      THETA20, rmax, vec1)
        assert err[k] <= b, (wl.name, k, err[k], b)
        assert abs(np.trace(got[k]).real - tr0) <= 1e-12, (k, np.trace(got[k]))
    if emulate:
        emu, _ = expmv.propagate_fp32_products(A, wl.rho0, wl.t0, wl.dt, wl.n_steps)
        emu_err = np.abs(emu - ref).max()
        assert err.max() <= 10 * emu_err + 1e-12, (wl.name, err.max(), emu_err)
    print(f"fp32 {wl.name}: max |d rho| {err.max():.3e}, trace_dev {st['trace_dev']:.2e}, "
          f"m={st['m']} s={st['s']} products={st['products']}", flush=True)
    return op, got, st, err


def test_cycle16():
    op, _, st, err = _check(workloads.cycle16())
    assert err.max() > 1e-12          # the single-precision rounding is really there
    assert 0.0 < st["trace_dev"] < 1e-6
    op.close()


@pytest.mark.parametrize("omega", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("r_mode,dephasing", [("transition", False), ("colnorm", True)])
def test_random_digraphs(omega, r_mode, dephasing):
    for N, k, seed in ((7, 2, 51), (23, 3, 52)):
        wl = random_workload(N, k, omega, seed, r_mode=r_mode, dephasing=dephasing,
                             n_steps=6, dt=0.8)
        op, _, _, _ = _check(wl)
        op.close()


def test_ragged_size_start_time_and_negative_step():
    wl = random_workload(41, 4, 0.45, 53, n_steps=4, dt=0.6, t0=1.3)
    op, _, st, _ = _check(wl)
    assert st["m0"] > 0
    op.close()
    wl = random_workload(9, 2, 0.3, 54, n_steps=3, dt=-0.5)
    op, _, _, _ = _check(wl)
    op.close()


def test_zero_steps_and_empty_graph():
    import paper_2003_02450_amd as qsw
    wl = random_workload(6, 2, 0.5, 55, n_steps=0)
    op = build_gpu(wl)
    op.set_precision("fp32")
    got = _run(op, wl)
    assert got.shape == (1, 6, 6) and np.array_equal(got[0], wl.rho0)
    op.close()
    op = qsw.Superop.from_graph(5, np.zeros(6, np.int64), np.array([], np.int32),
                                np.array([], np.float64), 0.5)
    op.set_precision("fp32")
    rho0 = workloads.uniform_superposition(5)
    out = op.propagate(rho0, 0.0, 1.0, 3).cpu().numpy()
    for k in range(4):
        assert np.abs(out[k] - rho0).max() <= 2.0 ** -24
    op.close()


def test_er256_every_point():
    """ER N=256 (101 points) against the oracle's full FP64 grid."""
    wl = workloads.er256()
    op, got, st, err = _check(wl, emulate=False)
    assert err.max() < 1e-6
    op.close()


def test_parameters_rerun_and_double_untouched():
    import paper_2003_02450_amd as qsw
    wl = workloads.er256()
    wl.n_steps = 5
    op = build_gpu(wl)
    d64 = _run(op, wl)
    s64 = op.last_stats()
    op.set_precision("fp32")
    a = _run(op, wl)
    s32 = op.last_stats()
    b = _run(op, wl)
    assert np.array_equal(a, b)                       # reruns are bitwise identical
    inf = op.info()
    d = [inf["norm1"], inf["norm1"]] + [inf["d"][p] for p in range(2, 10)]
    assert (s32["m"], s32["s"]) == qsw.select_params(inf["norm1"], d, wl.dt, single="fp32",
                                                            known_norms=True)
    assert s32["products"] < s64["products"] and s32["bytes"] < s64["bytes"]
    op.set_precision(False)
    again = _run(op, wl)
    assert op.last_stats()["prec"] == "double"
    assert np.array_equal(again, d64)                 # the double path is untouched
    op.close()


def test_batch_engine_takes_fp32_handles():
    """A single-precision-products handle runs in the batch engine too,
    bitwise as qsw_propagate runs it (more in test_gpu_batch_fp32.py)."""
    import torch
    import paper_2003_02450_amd as qsw
    wl = random_workload(9, 2, 0.3, 56, n_steps=3)
    op = build_gpu(wl)
    op.set_precision("fp32")
    r0 = torch.from_numpy(wl.rho0[None]).cuda()
    out = torch.empty((4, 1, 9, 9), dtype=torch.complex128, device="cuda")
    st = qsw.batch_propagate([(op, r0, 0.0, wl.dt, 3, out, None)])
    torch.cuda.synchronize()
    assert st["live"] == 0 and st["trace_dev"] > 0.0
    assert np.array_equal(out.cpu().numpy()[:, 0], _run(op, wl))
    op.close()


def _fullgrid():
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(__file__), "golden", "make_fullgrid.py")
    spec = importlib.util.spec_from_file_location("make_fullgrid", here)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, mod.load("outdeg1024")


def test_outdeg1024_every_point():
    """The benchmark workload at full size (N = 1024, 51 points), in the
    benchmark's launch configuration (launch pacing 2), against the oracle's
    full-grid fixture at every point (populations, trace, 10^4 samples),
    within the first-order bound; the single-precision error is reported."""
    mod, (hdr, fx) = _fullgrid()
    wl = workloads.outdeg1024()
    op = build_gpu(wl)
    op.set_pacing(2)
    op.set_precision("fp32")
    got = _run(op, wl)
    st = op.last_stats()
    n = wl.graph.N ** 2
    flat = got.reshape(wl.n_steps + 1, n)
    # the bound's inputs from the oracle: ||L||_1, the longest row, ||vec rho||_1
    A = oracle_superop(wl)
    norm1 = hdr["oracle"]["norm1"]
    rmax = int(np.diff(A.row_ptr).max())
    s = expmv.select_params_norm1(wl.dt * norm1, otheta.theta_table(otheta.TOL_SINGLE),
                                  expmv.M_MAX_FP32)[1]
    vec1 = float(fx["vec1"].max())
    worst = 0.0
    for k in range(wl.n_steps + 1):
        e = max(np.abs(np.diag(got[k]).real - fx["pops"][k]).max(),
                np.abs(flat[k, mod.sample_indices(n, k)] - fx["samples"][k]).max())
        b = expmv.fp32_products_bound(norm1, k * wl.dt, max(1, k * s), THETA20, rmax, vec1)
        assert e <= b, (k, e, b)
        assert abs(np.trace(got[k]).real - 1.0) <= 1e-12
        worst = max(worst, e)
    assert worst < 1e-6
    print(f"fp32 outdeg1024: max |d rho| {worst:.3e} over the fixture, trace_dev "
          f"{st['trace_dev']:.2e}, m={st['m']} s={st['s']} products={st['products']}", flush=True)
    op.close()
