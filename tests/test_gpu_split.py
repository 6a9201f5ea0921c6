"""Phase-split values.  Every off-diagonal entry of a graph-built L-QSW
superoperator is real (rate terms) or imaginary (Hamiltonian terms), so the
product kernels read one real coefficient per entry, the phase in the column
index and the complex diagonal per row.  The complex value is rebuilt before
the same multiply-adds, so results equal the complex layout's (QSW_SPLIT=0)
element for element (np.array_equal: up to the sign of zeros), in both
precisions and both branches, and the 1-norm estimates are the same.  Block-
shared leading positions (stored once per 64-row block when every row has
the same offset and value there) keep each row's order of summation, so
they change nothing either (QSW_SHARED=0 turns them off)."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu, random_workload

pytestmark = pytest.mark.gpu


def _series(op, wl, single):
    import torch
    op.set_precision(single)
    out = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), op.last_stats()["branch"]


def _both_formats(monkeypatch, make):
    monkeypatch.delenv("QSW_SPLIT", raising=False)
    a = make()
    monkeypatch.setenv("QSW_SPLIT", "0")
    b = make()
    monkeypatch.delenv("QSW_SPLIT", raising=False)
    return a, b


@pytest.mark.parametrize("case", ["er256_branch0", "rand300_series", "rand512_dephasing_colnorm"])
def test_split_equals_complex_layout(monkeypatch, case):
    if case == "er256_branch0":
        wl = workloads.er256()
        wl.n_steps = 3
    elif case == "rand300_series":
        wl = random_workload(300, 5, 0.3, 811, n_steps=24, dt=0.05)
    else:
        wl = random_workload(512, 4, 0.7, 812, r_mode="colnorm", dephasing=True,
                             n_steps=3, dt=0.4)
    sp, cx = _both_formats(monkeypatch, lambda: build_gpu(wl))
    assert sp.info()["split"] and not cx.info()["split"]
    for k in ("norm1", "d"):
        assert sp.info()[k] == cx.info()[k]
    for single in (False, True):
        a, ba = _series(sp, wl, single)
        b, bb = _series(cx, wl, single)
        assert ba == bb
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), (case, single, float(np.abs(a - b).max()))
    if case == "rand300_series":
        assert ba == 1
    if case == "er256_branch0":
        assert ba == 0
    sp.close()
    cx.close()


def test_split_channels_and_demoralised(monkeypatch):
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(813))
    g = workloads.random_out_degree(40, 3, rng)
    rho_c = workloads.random_density(42, rng, rank=2)

    def ch():
        return qsw.Superop.from_channels(g, 0.4, sources=[(3, 0.5)], sinks=[(7, 0.8)])
    sp, cx = _both_formats(monkeypatch, ch)
    assert sp.info()["split"]
    import torch
    a = sp.propagate(rho_c, 0.0, 0.5, 4).cpu().numpy()
    b = cx.propagate(rho_c, 0.0, 0.5, 4).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b)
    sp.close()
    cx.close()

    def dm():
        return qsw.Superop.from_demoralised(g, 0.6)
    sp, cx = _both_formats(monkeypatch, dm)
    n = sp.info()["N"]
    rho_d = workloads.random_density(n, rng, rank=1)
    a = sp.propagate(rho_d, 0.0, 0.5, 4).cpu().numpy()
    b = cx.propagate(rho_d, 0.0, 0.5, 4).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b)
    sp.close()
    cx.close()


def test_complex_entries_fall_back():
    """A Hamiltonian with complex off-diagonal entries gives entries that are
    neither real nor imaginary: the complex layout is used."""
    import paper_2003_02450_amd as qsw
    H = np.array([[1.0, 0.5 + 0.5j, 0.0], [0.5 - 0.5j, 0.0, 0.2j], [0.0, -0.2j, 2.0]])
    op = qsw.Superop.from_general(H, [np.array([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]])], 0.5)
    assert not op.info()["split"]
    op.close()


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("dense", [False, True])
def test_shared_positions_change_nothing(monkeypatch, single, dense):
    """Shared leading positions (at most 64 per block: the dense graph's
    H rows have more neighbours, and the rest stay in the rows) give the
    unshared layout's sums."""
    import torch
    if dense:
        wl = random_workload(128, 40, 0.35, 816, n_steps=2, dt=0.2)
    else:
        wl = random_workload(256, 6, 0.35, 815, n_steps=3, dt=0.5)
    monkeypatch.delenv("QSW_SHARED", raising=False)
    sh = build_gpu(wl)
    monkeypatch.setenv("QSW_SHARED", "0")
    un = build_gpu(wl)
    monkeypatch.delenv("QSW_SHARED", raising=False)
    i_sh, i_un = sh.info(), un.info()
    assert i_sh["split"] and i_un["split"]
    assert i_sh["shared_entries"] > 0 and i_un["shared_entries"] == 0
    assert i_sh["shared_entries"] <= 64 * ((i_sh["n"] + 63) // 64)
    assert i_sh["stream_entries"] < i_un["stream_entries"] == i_un["nnz"]
    assert i_sh["d"] == i_un["d"] and i_sh["norm1"] == i_un["norm1"]
    for op in (sh, un):
        op.set_precision(single)
    a = sh.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    b = un.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)
    sh.close()
    un.close()


@pytest.mark.parametrize("single", [False, True])
def test_block_dedup_changes_nothing(monkeypatch, single):
    """Blocks whose stored rows are word for word equal (columns as offsets
    from the row) read one copy; QSW_DEDUP=0 gives each block its own."""
    import torch
    wl = random_workload(512, 5, 0.45, 816, n_steps=3, dt=0.4)
    monkeypatch.delenv("QSW_DEDUP", raising=False)
    dd = build_gpu(wl)
    monkeypatch.setenv("QSW_DEDUP", "0")
    own = build_gpu(wl)
    monkeypatch.delenv("QSW_DEDUP", raising=False)
    i_dd, i_own = dd.info(), own.info()
    assert i_dd["distinct_entries"] < i_dd["stream_entries"] == i_own["stream_entries"]
    assert i_own["distinct_entries"] == i_own["stream_entries"]
    assert i_dd["d"] == i_own["d"]
    for op in (dd, own):
        op.set_precision(single)
    a = dd.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    b = own.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)
    dd.close()
    own.close()
