"""Batched walks (qsw_engine_* / qsw_batch_propagate) on the GPU.

Each column of a walk must be bitwise what qsw_propagate gives for that
density matrix alone (same parameters, terms, sums and stopping decisions);
sampled walks are also compared with the oracle at the FP64 bar (1e-10)."""
import numpy as np
import pytest

import workloads
from oracle import expmv
from tests.gpu_util import build_gpu, oracle_superop

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _single(op, rho0, wl):
    import torch
    out = op.propagate(rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _mixed_walks():
    """Small walks covering both branches, t0 != 0, ragged sizes, 1..4
    right-hand sides, complex64 values and an operator with L = 0."""
    rng = np.random.Generator(np.random.PCG64(77))
    wls = []
    g = workloads.random_out_degree(9, 2, rng)
    wls.append(workloads.Workload("a", g, 0.3, "laplacian", "transition", False,
                                  np.stack([workloads.random_density(9, rng, 2) for _ in range(3)]),
                                  0.0, 0.7, 5))
    g = workloads.er_undirected(23, 0.3, rng)
    wls.append(workloads.Workload("b", g, 0.8, "laplacian", "colnorm", True,
                                  workloads.basis_states(23, [0, 5, 7, 22]), 1.1, 0.4, 6))
    wl = workloads.cycle16()              # series branch (q > s)
    wl.rho0 = np.stack([wl.rho0, workloads.maximally_mixed(16)])
    wls.append(wl)
    g = workloads.er_undirected(41, 0.15, rng)
    wls.append(workloads.Workload("d", g, 0.5, "adjacency", "transition", False,
                                  workloads.basis_states(41, [3]), 0.0, 2.5, 3))
    g = workloads.graph_from_arcs(5, [], [], [])  # no arcs: L = 0, m = 0
    wls.append(workloads.Workload("e", g, 0.5, "laplacian", "transition", False,
                                  workloads.basis_states(5, [1, 2]), 0.5, 1.0, 2))
    return wls


def _run_batch(wls, rhs=None, single=()):
    import torch
    import paper_2003_02450_amd as qsw
    dev = torch.device("cuda", 0)
    ops, items, outs, pops = [], [], [], []
    for i, wl in enumerate(wls):
        op = build_gpu(wl)
        if i in single:
            op.set_precision(True)
        r0 = torch.from_numpy(wl.rho0).to(dev)
        n0, N = r0.shape[0], wl.graph.N
        o = torch.full((wl.n_steps + 1, n0, N, N), float("nan"), dtype=torch.complex128, device=dev)
        p = torch.full((wl.n_steps + 1, n0, N), float("nan"), dtype=torch.float64, device=dev)
        ops.append(op)
        outs.append(o)
        pops.append(p)
        items.append((op, r0, wl.t0, wl.dt, wl.n_steps, o, p))
    st = qsw.batch_propagate(items, rhs=rhs)
    torch.cuda.synchronize()
    return ops, [o.cpu().numpy() for o in outs], [p.cpu().numpy() for p in pops], st


@pytest.mark.parametrize("rhs", [4, None])
def test_batch_is_bitwise_single_walks(rhs):
    wls = _mixed_walks()
    ops, outs, pops, st = _run_batch(wls, rhs=rhs, single=(1,))
    assert st["live"] == 0 and not st["nonfinite"]
    total = 0
    for i, (wl, op) in enumerate(zip(wls, ops)):
        for c in range(wl.rho0.shape[0]):
            ref = _single(op, wl.rho0[c], wl)
            total += op.last_stats()["products"]
            assert np.array_equal(outs[i][:, c], ref), (wl.name, c)
            assert np.array_equal(pops[i][:, c], np.real(np.einsum("kaa->ka", ref))), (wl.name, c)
    assert st["products"] <= total   # the matrix is read once for all columns
    for op in ops:
        op.close()


def test_batch_matches_oracle_and_invariants():
    wls = workloads.batch64(count=6, n_steps=12)
    ops, outs, _, st = _run_batch(wls)
    assert st["live"] == 0
    for i, wl in enumerate(wls):
        A = oracle_superop(wl)
        for c in (0, wl.rho0.shape[0] - 1):
            ref, _ = expmv.propagate(A, wl.rho0[c], wl.t0, wl.dt, wl.n_steps)
            assert np.abs(outs[i][:, c] - ref).max() <= TOL, (wl.name, c)
        for k in range(wl.n_steps + 1):
            for c in range(wl.rho0.shape[0]):
                assert abs(np.trace(outs[i][k, c]) - 1) < 1e-12
    for op in ops:
        op.close()


def test_engine_admission_and_reuse():
    """An arena with room for two walks admits two, refuses the third until
    one finishes, and every result is bitwise that of the one-shot batch."""
    import torch
    import paper_2003_02450_amd as qsw
    from paper_2003_02450_amd import _lib
    dev = torch.device("cuda", 0)
    wls = workloads.batch64(count=3, n_steps=8, n_lo=20, n_hi=24)
    ops = [build_gpu(wl) for wl in wls]
    need = [qsw.Engine.walk_bytes(op, wl.rho0.shape[0], wl.t0, wl.dt, wl.n_steps, 4)
            for op, wl in zip(ops, wls)]
    L = _lib.load()
    pair = (_lib.Walk * 2)(*[_lib.Walk(ops[i]._h, wls[i].rho0.shape[0], 1, 0.0, wls[i].dt,
                                      wls[i].n_steps, None, None) for i in range(2)])
    arena = (int(L.qsw_batch_workspace_bytes(pair, 2, 4)) - int(L.qsw_engine_table_bytes(2))
             + int(L.qsw_engine_table_bytes(4)))
    eng = qsw.Engine(4, 4, arena)
    outs = [torch.empty((wl.n_steps + 1,) + wl.rho0.shape, dtype=torch.complex128, device=dev)
            for wl in wls]
    r0 = [torch.from_numpy(wl.rho0).to(dev) for wl in wls]
    t = [eng.submit(ops[i], r0[i], 0.0, wls[i].dt, wls[i].n_steps, out=outs[i]) for i in range(2)]
    assert None not in t
    if need[2] > max(need[0], need[1]):
        pytest.skip("third walk larger than both others")
    assert eng.submit(ops[2], r0[2], 0.0, wls[2].dt, wls[2].n_steps, out=outs[2]) is None
    assert eng.run() == 0
    assert sorted(eng.poll()) == sorted(t)
    t3 = eng.submit(ops[2], r0[2], 0.0, wls[2].dt, wls[2].n_steps, out=outs[2])
    assert t3 is not None
    assert eng.run() == 0 and eng.poll() == [t3]
    eng.close()
    _, ref, _, _ = _run_batch(wls)
    for i in range(3):
        assert np.array_equal(outs[i].cpu().numpy(), ref[i])
    for op in ops:
        op.close()


def test_single_rhs_engine_and_zero_steps():
    wls = _mixed_walks()
    for wl in wls:
        wl.rho0 = wl.rho0[:1]
    wls[0].n_steps = 0
    ops, outs, _, st = _run_batch(wls, rhs=1)
    for i, (wl, op) in enumerate(zip(wls, ops)):
        ref = _single(op, wl.rho0[0], wl)
        assert np.array_equal(outs[i][:, 0], ref), wl.name
    for op in ops:
        op.close()


@pytest.mark.parametrize("graph,tune", [("0", "0"), ("1", "0"), ("1", "1")])
def test_graph_chunks_and_tuned_shapes_change_nothing(graph, tune, monkeypatch):
    """Chunk graphs (captured once per set of running walks, replayed per
    chunk) and every tuned launch shape give bitwise the results of direct
    launches with the default shape."""
    monkeypatch.setenv("QSW_BATCH_GRAPH", graph)
    monkeypatch.setenv("QSW_BATCH_TUNE", tune)
    wls = workloads.batch64(count=8, n_steps=40)
    ops, outs, pops, st = _run_batch(wls)
    assert st["live"] == 0 and not st["nonfinite"]
    if graph == "1":
        assert st["graph_launches"] > 0 and 1 <= st["graphs"] <= st["graph_launches"]
    else:
        assert st["graph_launches"] == 0
    assert st["bytes"] > 0
    monkeypatch.setenv("QSW_BATCH_GRAPH", "0")
    monkeypatch.setenv("QSW_BATCH_TUNE", "0")
    _, ref, rpops, _ = _run_batch(wls)
    for i in range(len(wls)):
        assert np.array_equal(outs[i], ref[i]) and np.array_equal(pops[i], rpops[i])
    for op in ops:
        op.close()


def test_tuned_shape_is_remembered_for_the_key(monkeypatch):
    monkeypatch.setenv("QSW_BATCH_TUNE", "1")
    wls = workloads.batch64(count=6, n_steps=60)
    ops1, a, _, st1 = _run_batch(wls)
    ops2, b, _, st2 = _run_batch(wls)              # same key: the shape is taken, not tuned
    assert (st1["rounds"], st1["staged"]) == (st2["rounds"], st2["staged"])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for op in ops1 + ops2:
        op.close()
