"""Single-precision products (QSW_PREC_FP32) in the batch engine.

Each column of such a walk must be bitwise what qsw_propagate with
single-precision products gives for that density matrix alone: complex64
terms, the hi + lo accumulation, the stopping decisions in double, one
single-time application per interval and the FP64 trace check at every
point.  Walks of every precision share one engine, each bitwise its own
single path; chunk graphs and tuned launch shapes change nothing; the
engine's largest trace deviation is that of the single paths.  (The single
path itself is held to the FP64 oracle within the stated bound in
test_gpu_fp32.py.)"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import build_gpu
from tests.test_gpu_batch import _mixed_walks, _single

pytestmark = pytest.mark.gpu


def _run(wls, precs, rhs=None):
    import torch
    import paper_2003_02450_amd as qsw
    dev = torch.device("cuda", 0)
    ops, items, outs, pops = [], [], [], []
    for wl, prec in zip(wls, precs):
        op = build_gpu(wl)
        op.set_precision(prec)
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


def _check_single(wls, ops, outs, pops):
    tdev = 0.0
    for i, (wl, op) in enumerate(zip(wls, ops)):
        for c in range(wl.rho0.shape[0]):
            ref = _single(op, wl.rho0[c], wl)
            st = op.last_stats()
            if st["prec"] == "fp32":
                tdev = max(tdev, st["trace_dev"])
            assert np.array_equal(outs[i][:, c], ref), (wl.name, c, st["prec"])
            assert np.array_equal(pops[i][:, c], np.real(np.einsum("kaa->ka", ref))), (wl.name, c)
    return tdev


@pytest.mark.parametrize("rhs", [4, None])
def test_fp32_batch_is_bitwise_single_walks(rhs):
    wls = _mixed_walks()
    ops, outs, pops, st = _run(wls, ["fp32"] * len(wls), rhs=rhs)
    assert st["live"] == 0 and not st["nonfinite"]
    tdev = _check_single(wls, ops, outs, pops)
    assert st["trace_dev"] == tdev and 0.0 < tdev < 1e-6
    for op in ops:
        op.close()


def test_precisions_mixed_in_one_engine():
    wls = _mixed_walks()
    precs = ["fp32", "double", "fp32", "single", "fp32"]
    ops, outs, pops, st = _run(wls, precs)
    assert st["live"] == 0 and not st["nonfinite"]
    tdev = _check_single(wls, ops, outs, pops)
    assert st["trace_dev"] == tdev
    for op in ops:
        op.close()


def test_fp32_single_rhs_and_zero_steps():
    wls = _mixed_walks()
    for wl in wls:
        wl.rho0 = wl.rho0[:1]
    wls[0].n_steps = 0
    ops, outs, pops, st = _run(wls, ["fp32"] * len(wls), rhs=1)
    _check_single(wls, ops, outs, pops)
    for op in ops:
        op.close()


@pytest.mark.parametrize("graph,tune", [("0", "0"), ("1", "1")])
def test_fp32_graph_chunks_and_tuned_shapes_change_nothing(graph, tune, monkeypatch):
    monkeypatch.setenv("QSW_BATCH_GRAPH", graph)
    monkeypatch.setenv("QSW_BATCH_TUNE", tune)
    wls = workloads.batch64(count=8, n_steps=40)
    precs = ["fp32"] * 6 + ["double"] * 2
    ops, outs, pops, st = _run(wls, precs)
    assert st["live"] == 0 and not st["nonfinite"]
    assert 0.0 < st["trace_dev"] < 1e-6
    monkeypatch.setenv("QSW_BATCH_GRAPH", "0")
    monkeypatch.setenv("QSW_BATCH_TUNE", "0")
    _, ref, rpops, _ = _run(wls, precs)
    for i in range(len(wls)):
        assert np.array_equal(outs[i], ref[i]) and np.array_equal(pops[i], rpops[i])
    # sampled: the first and the last walk against their single paths
    _check_single([wls[0], wls[-1]], [ops[0], ops[-1]], [outs[0], outs[-1]],
                  [pops[0], pops[-1]])
    for op in ops:
        op.close()


def test_fp32_walk_bytes_are_half():
    import paper_2003_02450_amd as qsw
    wl = workloads.batch64(count=1, n_steps=10)[0]
    op = build_gpu(wl)
    b64 = qsw.Engine.walk_bytes(op, 4, 0.0, wl.dt, wl.n_steps, 4)
    op.set_precision("fp32")
    b32 = qsw.Engine.walk_bytes(op, 4, 0.0, wl.dt, wl.n_steps, 4)
    assert 0 < b32 < b64 and b32 * 2 <= b64 + 6 * 256
    op.close()


def test_fp32_complex_valued_operator():
    """An explicit operator with complex entries (complex layout, no
    phase-split values) as a single-precision-products walk, next to a
    graph walk: each column bitwise its single-walk result."""
    import torch
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(91))
    N = 12
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    H = (A + A.conj().T) / 2
    Ls = [np.outer(rng.standard_normal(N) + 1j * rng.standard_normal(N), np.eye(N)[k])
          for k in range(3)]
    op_c = qsw.Superop.from_general(H, Ls, 0.4)
    assert not op_c.info()["split"]
    op_c.set_precision("fp32")
    wl_g = _mixed_walks()[0]
    op_g = build_gpu(wl_g)
    op_g.set_precision("fp32")
    dev = torch.device("cuda", 0)
    rho_c = np.stack([workloads.random_density(N, rng, rank=2) for _ in range(2)])
    items, outs = [], []
    for op, r0, t0, dt, q in ((op_c, rho_c, 0.3, 0.5, 6), (op_g, wl_g.rho0, wl_g.t0, wl_g.dt,
                                                             wl_g.n_steps)):
        r = torch.from_numpy(r0).to(dev)
        o = torch.empty((q + 1,) + r0.shape, dtype=torch.complex128, device=dev)
        items.append((op, r, t0, dt, q, o, None))
        outs.append(o)
    st = qsw.batch_propagate(items)
    torch.cuda.synchronize()
    assert st["live"] == 0 and not st["nonfinite"]
    for (op, r, t0, dt, q, _, _), o in zip(items, outs):
        got = o.cpu().numpy()
        for c in range(r.shape[0]):
            ref = op.propagate(r[c], t0, dt, q)
            torch.cuda.synchronize()
            assert np.array_equal(got[:, c], ref.cpu().numpy()), c
    op_c.close()
    op_g.close()
