"""Continuous-batching server on the GPU: results are bitwise those of each
walk alone (and of qsw_propagate), the operator cache and admission work, and
a sampled walk matches the oracle at the FP64 bar."""
import numpy as np
import pytest

import workloads
from oracle import expmv
from tests.gpu_util import oracle_superop

pytestmark = pytest.mark.gpu

GB = 1 << 30


def _requests(k, seed, n_hi=60):
    return workloads.served_requests(k, seed=seed, n_lo=12, n_hi=n_hi, t_end=4.0)


def _serve(reqs, arena=2 * GB, cache=2 * GB, max_walks=64, cycles=8):
    import torch
    import paper_2003_02450_amd as qsw
    srv = qsw.Server(arena, cache, max_walks)
    ids = [srv.submit(r["graph"], r["omega"], 0.0, r["dt"], r["n_steps"]) for r in reqs]
    results = {}
    seen_pending = False
    for _ in range(100000):
        running, pending = srv.step(cycles)
        seen_pending |= pending > 0
        for rid, lat, pops, _ in srv.poll():
            results[rid] = pops.cpu().numpy()
            assert lat >= 0
        if running == 0 and pending == 0 and len(results) == len(ids):
            break
    torch.cuda.synchronize()
    st = srv.stats()
    srv.close()
    return [results[i] for i in ids], st, seen_pending


def test_mix_is_bitwise_each_walk_alone_and_single_path():
    import torch
    import paper_2003_02450_amd as qsw
    reqs = _requests(7, 501)
    mixed, st, _ = _serve(reqs)
    assert st["completed"] == 7 and st["cache_misses"] == 7
    for r, got in zip(reqs, mixed):
        alone, _, _ = _serve([r])
        assert np.array_equal(got, alone[0])
        g = r["graph"]
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, r["omega"])
        rho0 = workloads.basis_state(g.N, 0)
        ref = op.propagate(rho0, 0.0, r["dt"], r["n_steps"])
        pref = op.populations(ref)
        torch.cuda.synchronize()
        assert np.array_equal(got, pref.cpu().numpy())
        op.close()


def test_matches_oracle():
    r = _requests(1, 502, n_hi=30)[0]
    got, _, _ = _serve([r])
    wl = workloads.Workload("s", r["graph"], r["omega"], "laplacian", "transition", False,
                            workloads.basis_state(r["graph"].N, 0), 0.0, r["dt"], r["n_steps"])
    ref, _ = expmv.propagate(oracle_superop(wl), wl.rho0, 0.0, wl.dt, wl.n_steps)
    pops = np.real(np.einsum("kaa->ka", ref))
    assert np.abs(got[0] - pops).max() <= 1e-10


def test_benchmark_stream_walks_match_oracle_fixture():
    """The sampled walks of the serving benchmark's request stream, served in
    a mix with their neighbours of the stream, against the oracle's committed
    populations (tests/golden/make_served.py) at the FP64 bar."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(__file__), "golden", "make_served.py")
    spec = importlib.util.spec_from_file_location("make_served", here)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    hdr, pops = mod.load()
    reqs = workloads.served_requests(mod.MIN_COUNT)
    last = max(pops) + 1
    small = [i for i in range(last) if reqs[i]["graph"].N <= 256]   # the mix, kept small
    got, st, _ = _serve([reqs[i] for i in small])
    for i, p in pops.items():
        err = np.abs(got[small.index(i)] - p).max()
        assert err <= 1e-10, (i, err)
    print(f"served sampled walks {sorted(pops)}: max |d pops| vs oracle "
          f"{max(np.abs(got[small.index(i)] - p).max() for i, p in pops.items()):.2e}",
          flush=True)


def test_cache_hits_and_evictions():
    reqs = _requests(4, 503)
    again = [reqs[0], reqs[1], reqs[0]]
    res, st, _ = _serve(reqs + again)
    assert st["cache_hits"] == 3 and st["cache_misses"] == 4
    assert np.array_equal(res[0], res[4]) and np.array_equal(res[0], res[6])
    # a budget below one operator: every unused operator is evicted
    res2, st2, _ = _serve(reqs + again, cache=1)
    assert st2["evictions"] > 0
    for a, b in zip(res, res2):
        assert np.array_equal(a, b)


def _largest_walk_bytes(reqs):
    import paper_2003_02450_amd as qsw
    best = 0
    for r in reqs:
        g = r["graph"]
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, r["omega"])
        best = max(best, qsw.Engine.walk_bytes(op, 1, 0.0, r["dt"], r["n_steps"], 1))
        op.close()
    return best


def test_admission_waits_for_space():
    """Walks wait when no slot or not enough arena is free; all finish with
    unchanged results; a walk that can never fit is refused at submit."""
    import paper_2003_02450_amd as qsw
    from paper_2003_02450_amd import _lib
    reqs = _requests(5, 504, n_hi=40)
    full, _, _ = _serve(reqs)
    slots, st, seen_pending = _serve(reqs, max_walks=2)
    assert seen_pending and st["completed"] == 5
    big = _largest_walk_bytes(reqs)
    arena = int(_lib.load().qsw_engine_table_bytes(64)) + (big * 3) // 2 + (64 << 10)
    tight, st, seen_pending = _serve(reqs, arena=arena)
    assert seen_pending and st["completed"] == 5
    for a, b, c in zip(full, slots, tight):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    # an arena too small for any walk: the operator is built off the serving
    # loop, and the step that sees the build finish refuses the walk
    srv = qsw.Server(64 << 10, 1 << 30, 4)
    rid = srv.submit(reqs[0]["graph"], reqs[0]["omega"], 0.0, reqs[0]["dt"], reqs[0]["n_steps"])
    with pytest.raises(qsw.QswError, match="QSW_ERR_OOM"):
        for _ in range(20000):
            srv.step(1)
    assert [d[0] for d in srv.poll()] == [rid]
    srv.close()


def test_builds_overlap_running_walks():
    """A walk that arrives while others run has its operator built off the
    serving loop: the running walks keep stepping (the step calls return while
    the build is in flight) and every result is bitwise that of the walk alone."""
    import paper_2003_02450_amd as qsw
    reqs = _requests(6, 505, n_hi=48)
    srv = qsw.Server(2 * GB, 2 * GB, 64)
    first = [srv.submit(r["graph"], r["omega"], 0.0, r["dt"], r["n_steps"]) for r in reqs[:3]]
    steps_before_late = 0
    results = {}
    late = None
    for _ in range(100000):
        running, pending = srv.step(2)
        for rid, lat, pops, _ in srv.poll():
            results[rid] = pops.cpu().numpy()
        if late is None and running > 0:
            late = [srv.submit(r["graph"], r["omega"], 0.0, r["dt"], r["n_steps"])
                    for r in reqs[3:]]
        elif late is not None and len(results) < 6:
            steps_before_late += 1
        if late is not None and len(results) == 6 and running == 0 and pending == 0:
            break
    st = srv.stats()
    srv.close()
    assert st["completed"] == 6 and st["cache_misses"] == 6 and st["build_ms"] > 0
    alone = [_serve([r])[0][0] for r in reqs]
    for rid, a in zip(first + late, alone):
        assert np.array_equal(results[rid], a)


def test_direct_lane_and_engine_lane_mix(monkeypatch):
    """With the direct lane taking every walk of order 30 or more, walks run
    in both lanes at once; every result is bitwise that of qsw_propagate
    alone."""
    import torch
    import paper_2003_02450_amd as qsw
    monkeypatch.setenv("QSW_SERVER_DIRECT_N", "30")
    reqs = _requests(8, 506, n_hi=60)
    assert any(r["graph"].N >= 30 for r in reqs) and any(r["graph"].N < 30 for r in reqs)
    mixed, st, _ = _serve(reqs)
    assert st["completed"] == 8
    for r, got in zip(reqs, mixed):
        g = r["graph"]
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, r["omega"])
        ref = op.populations(op.propagate(workloads.basis_state(g.N, 0), 0.0, r["dt"],
                                          r["n_steps"]))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), g.N
        op.close()
