"""Paper variants on the GPU (same product kernels, other assemblies):
explicit operators (G-QSW, rotating Hamiltonian), absorption / emission
channels, and set_omega; each against the oracle at the FP64 bar."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import expmv, operators

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run(op, rho0, t0, dt, q):
    import torch
    out = op.propagate(rho0, t0, dt, q)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _rand_ops(N, seed, n_ops=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    H = X + X.conj().T
    H[np.abs(H) < 0.8] = 0  # some sparsity, still Hermitian
    Y = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    Hr = 0.3 * (Y + Y.conj().T)
    Ls = []
    for _ in range(n_ops):
        L = 0.5 * (rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
        L[rng.random((N, N)) < 0.5] = 0
        Ls.append(L)
    rho0 = workloads.random_density(N, rng, rank=2)
    return H, Ls, Hr, rho0


@pytest.mark.parametrize("omega", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("with_rot", [False, True])
def test_general_operators_match_oracle(omega, with_rot):
    import paper_2003_02450_amd as qsw
    H, Ls, Hr, rho0 = _rand_ops(5, 71)
    op = qsw.Superop.from_general(H, Ls, omega, H_rot=Hr if with_rot else None)
    A = oracle.general_superop(H, Ls, omega, Hr if with_rot else None)
    rp, col, val = op.csr()
    D = np.zeros((op.n, op.n), complex)
    for r in range(op.n):
        D[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
    assert np.abs(D - A.dense()).max() < 1e-14
    assert abs(op.info()["norm1"] - A.norm1()) <= 1e-13 * A.norm1()
    got = _run(op, rho0, 0.0, 0.6, 5)
    ref, _ = expmv.propagate(A, rho0, 0.0, 0.6, 5)
    assert np.abs(got - ref).max() <= TOL
    op.close()


def test_gqsw_three_vertex_example():
    import paper_2003_02450_amd as qsw
    gold = json.load(open(os.path.join(GOLDEN, "gqsw_example.json")))
    G = np.zeros((3, 3))
    for i, j in gold["graph_arcs_target_source"]:
        G[i, j] = 1.0
    H = operators.transition_matrix(1.0, operators.undirected(G))
    op = qsw.Superop.from_general(H, [G], gold["omega"])
    got = _run(op, np.diag([1.0, 0.0, 0.0]).astype(complex), 0.0, gold["t"], 1)
    assert np.abs(np.real(np.diag(got[1])) - gold["populations"]).max() < 1e-10
    op.close()


@pytest.mark.parametrize("omega", [0.0, 0.5, 1.0])
def test_channels_match_oracle(omega):
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(72))
    g = workloads.random_out_degree(7, 2, rng)
    sources, sinks = [(0, 1.5), (3, 0.4)], [(5, 2.0)]
    op = qsw.Superop.from_channels(g, omega, sources, sinks)
    assert op.N == 10
    A = oracle.channel_superop(g.dense(), omega, sources, sinks)
    rho0 = np.zeros((10, 10), complex)
    rho0[7, 7] = 0.5          # half in the first source
    rho0[2, 2] = 0.5
    got = _run(op, rho0, 0.0, 0.5, 6)
    ref, _ = expmv.propagate(A, rho0, 0.0, 0.5, 6)
    assert np.abs(got - ref).max() <= TOL
    for k in range(7):
        assert abs(np.trace(got[k]) - 1) < 1e-12
    op.close()


def test_open_operators_match_channels():
    """build_open with M_free is the same generator as build_channels."""
    import paper_2003_02450_amd as qsw
    G = np.array([[0.0, 1.0], [1.0, 0.0]])
    g = workloads.graph_from_arcs(2, [0, 1], [1, 0], [1.0, 1.0])
    a = qsw.Superop.from_channels(g, 0.4, [(0, 2.0)], [(1, 3.0)])
    Ga, chans = operators.augmented(G, [(0, 2.0)], [(1, 3.0)])
    H, ML = operators.walk_operators(Ga)
    F = sum(np.real(c) for c in chans)
    b = qsw.Superop.from_operators(H, ML, 0.4, M_free=F)
    rho0 = np.diag([0, 0, 1.0, 0]).astype(complex)
    ra = _run(a, rho0, 0.0, 0.8, 10)
    rb = _run(b, rho0, 0.0, 0.8, 10)
    assert np.abs(ra - rb).max() < 1e-13
    assert np.real(ra[-1][3, 3]) > 0.3   # the sink fills
    a.close()
    b.close()


@pytest.mark.parametrize("kind", ["graph", "general", "channels"])
def test_set_omega_equals_fresh_build(kind):
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(73))
    g = workloads.random_out_degree(9, 2, rng)
    H, Ls, Hr, _ = _rand_ops(4, 74)

    def make(omega):
        if kind == "graph":
            return qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, omega)
        if kind == "general":
            return qsw.Superop.from_general(H, Ls, omega, H_rot=Hr)
        return qsw.Superop.from_channels(g, omega, [(1, 0.8)], [(4, 1.1)])
    op = make(0.2)
    op.set_precision(True)
    op.set_omega(0.85)
    assert abs(op.omega - 0.85) < 1e-15 and op.last_stats is not None
    fresh = make(0.85)
    fresh.set_precision(True)
    rho0 = workloads.random_density(op.N, rng, rank=1)
    a = _run(op, rho0, 0.0, 0.5, 4)
    b = _run(fresh, rho0, 0.0, 0.5, 4)
    assert np.array_equal(a, b)
    op.set_precision(False)
    fresh.set_precision(False)
    assert np.array_equal(_run(op, rho0, 0.0, 0.5, 4), _run(fresh, rho0, 0.0, 0.5, 4))
    op.close()
    fresh.close()


@pytest.mark.parametrize("omega", [0.0, 0.6, 1.0])
def test_demoralised_matches_oracle(omega):
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(75))
    g = workloads.random_out_degree(5, 2, rng)
    op = qsw.Superop.from_demoralised(g, omega)
    d, HD, LD, Hr = operators.demoralise(g.dense())
    assert (op.copies == d).all() and op.N == int(d.sum())
    A = oracle.general_superop(HD, [LD], omega, Hr)
    rho0 = qsw.demoralised_state(workloads.random_density(5, rng, rank=2), op.copies)
    got = _run(op, rho0, 0.0, 0.7, 5)
    ref, _ = expmv.propagate(A, rho0, 0.0, 0.7, 5)
    assert np.abs(got - ref).max() <= TOL
    pops = qsw.demoralised_populations(np.real(np.einsum("kaa->ka", got)), op.copies)
    assert np.abs(pops.sum(axis=1) - 1).max() < 1e-12
    op.close()


def test_nm_gqsw_example_through_gpu():
    import paper_2003_02450_amd as qsw
    gold = json.load(open(os.path.join(GOLDEN, "nm_gqsw_example.json")))
    g = workloads.graph_from_arcs(3, [2, 2], [0, 1], [1.0, 1.0])
    for omega, key in ((1.0, "omega_1"), (0.0, "omega_0")):
        op = qsw.Superop.from_demoralised(g, omega)
        rho0 = qsw.demoralised_state(np.diag([1.0, 0.0, 0.0]).astype(complex), op.copies)
        got = _run(op, rho0, 0.0, gold["t"], 1)
        p = qsw.demoralised_populations(np.real(np.diag(got[1])), op.copies)[0]
        printed = np.array(gold["printed_populations"][key])
        assert np.abs(p - printed).max() < 5e-9, (key, p)
        if omega == 1.0:
            assert abs(p[0] - np.exp(-100.0)) < 1e-6 * np.exp(-100.0)
        op.close()
