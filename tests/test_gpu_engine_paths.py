"""The product engines other than the default (wave layout, rho-row staged in
LDS) against it and against the oracle.

* Unstaged wave layout (QSW_STAGE=0; the engine every operator with N > 2048
  takes): the staging only moves where a gather reads from, so its results
  equal the staged engine's bit for bit.
* Plain CSR engines (QSW_ENGINE=3 stream, 16 vector): the complex CSR in row
  order, a different summation order, so they agree to rounding and, like
  the default, with the oracle within the FP64 bar.
* N = 2100 (beyond the LDS stage): the unstaged wave layout and the CSR
  stream engine, two independent product paths, agree to rounding; every
  point keeps the trace and is Hermitian.
* Wide groups (QSW_WIDE=1, engine 300: more positions per group at fewer
  waves per SIMD, taken by default for long rows): only the grouping of a
  row's positions changes, so the results equal the default's bit for bit,
  and both agree with the oracle within the FP64 bar.
* The CSR stream engine's workgroup count (QSW_CSR_GRID) only changes which
  workgroup takes which run of row blocks: the same results bit for bit.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, gpu_run, oracle_superop, random_workload
from oracle import expmv

pytestmark = pytest.mark.gpu

CASES = [(37, 3, 0.6, False), (300, 4, 0.25, True), (1024, 3, 0.5, False)]


def _run_with(monkeypatch, wl, **env):
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    op = build_gpu(wl)
    for k in env:
        monkeypatch.delenv(k, raising=False)
    out, _ = gpu_run(wl, op)
    op.close()
    return out


@pytest.mark.parametrize("N,k,omega,dephasing", CASES)
def test_unstaged_equals_staged(monkeypatch, N, k, omega, dephasing):
    wl = random_workload(N, k, omega, 900 + N, dephasing=dephasing, n_steps=3, dt=0.6)
    ref = _run_with(monkeypatch, wl)
    got = _run_with(monkeypatch, wl, QSW_STAGE="0")
    assert np.isfinite(ref).all()
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("engine", ["3", "16"])
@pytest.mark.parametrize("N,k,omega,dephasing", CASES[:2])
def test_csr_engines_match_default_and_oracle(monkeypatch, engine, N, k, omega, dephasing):
    wl = random_workload(N, k, omega, 910 + N, dephasing=dephasing, n_steps=3, dt=0.6)
    ref = _run_with(monkeypatch, wl)
    got = _run_with(monkeypatch, wl, QSW_ENGINE=engine)
    assert np.abs(got - ref).max() <= 1e-13
    A = oracle_superop(wl)
    orc, _ = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    assert np.abs(got - orc).max() <= 1e-10
    assert np.abs(ref - orc).max() <= 1e-10


def test_beyond_stage_two_engines_agree(monkeypatch):
    """A path digraph of 2100 vertices (superoperator of 4.41M rows): its
    rho-row does not fit the LDS stage, so the wave layout runs unstaged."""
    rng = np.random.Generator(np.random.PCG64(921))
    g = workloads.line_digraph(2100, rng)
    rho0 = np.zeros((g.N, g.N), dtype=np.complex128)
    rho0[0, 0] = 1.0
    wl = workloads.Workload("line2100", g, 0.5, "laplacian", "transition", False, rho0,
                            0.0, 0.5, 2)
    wave = _run_with(monkeypatch, wl)
    csr = _run_with(monkeypatch, wl, QSW_ENGINE="3")
    assert np.isfinite(wave).all()
    assert np.abs(wave - csr).max() <= 1e-13
    for k in range(wl.n_steps + 1):
        assert abs(np.trace(wave[k]) - 1.0) <= 1e-12
        assert np.abs(wave[k] - wave[k].conj().T).max() <= 1e-14
    # the walk has left vertex 0
    assert wave[-1][0, 0].real < 1.0 - 1e-3


@pytest.mark.parametrize("N,k,omega,dense", [(300, 4, 0.4, False), (1024, 3, 0.5, False),
                                              (64, 0, 0.3, True)])
def test_wide_groups_equal_default(monkeypatch, N, k, omega, dense):
    if dense:
        rng = np.random.Generator(np.random.PCG64(931))
        g = workloads.complete_digraph(N, rng)
        rho0 = workloads.random_density(N, rng, rank=2)
        wl = workloads.Workload("complete64", g, omega, "laplacian", "transition", False, rho0,
                                0.0, 0.05, 3)
    else:
        wl = random_workload(N, k, omega, 940 + N, n_steps=3, dt=0.6)
    ref = _run_with(monkeypatch, wl, QSW_WIDE="0")
    got = _run_with(monkeypatch, wl, QSW_WIDE="1")
    assert np.isfinite(ref).all()
    assert np.array_equal(ref, got)
    A = oracle_superop(wl)
    orc, _ = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    assert np.abs(got - orc).max() <= 1e-10
    # the engine each takes, and the default for long rows
    monkeypatch.setenv("QSW_WIDE", "1")
    op = build_gpu(wl)
    monkeypatch.delenv("QSW_WIDE")
    assert op.info()["engine"] == 310
    op.close()
    op = build_gpu(wl)
    per_row = op.info()["stream_entries"] / op.info()["n"]
    assert op.info()["engine"] == (310 if per_row >= 128 else 110)
    op.close()


@pytest.mark.parametrize("grid", ["1", "24"])
def test_stream_engine_grid_changes_nothing(monkeypatch, grid):
    wl = random_workload(300, 4, 0.25, 1210, dephasing=True, n_steps=3, dt=0.6)
    ref = _run_with(monkeypatch, wl, QSW_ENGINE="3")
    got = _run_with(monkeypatch, wl, QSW_ENGINE="3", QSW_CSR_GRID=grid)
    assert np.isfinite(ref).all()
    assert np.array_equal(ref, got)
