"""Pins for the oracle's variant generators: the G-QSW of eq. L_global
(paper's printed three-vertex result), the general Kronecker form against
the analytic L-QSW rows, and the absorption / emission channels of eq.
qsw_ss against closed forms and invariants."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from oracle import expmv, operators

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gqsw_three_vertex_printed():
    gold = json.load(open(os.path.join(GOLDEN, "gqsw_example.json")))
    G = np.zeros((3, 3))
    for i, j in gold["graph_arcs_target_source"]:
        G[i, j] = 1.0
    H = operators.transition_matrix(1.0, operators.undirected(G))
    A = oracle.general_superop(H, [G], gold["omega"])
    out, _ = expmv.propagate(A, np.diag([1.0, 0.0, 0.0]).astype(complex), 0.0, gold["t"], 1)
    # the |-> = (|0> - |1>)/sqrt 2 component is dark (G|-> = 0): populations
    # reach exactly 1/4, 1/4 and 1/2
    assert np.abs(np.real(np.diag(out[1])) - gold["populations"]).max() < 1e-12


@pytest.mark.parametrize("omega", [0.0, 0.35, 1.0])
@pytest.mark.parametrize("r_mode,dephasing", [("transition", False), ("colnorm", True)])
def test_general_form_equals_local_rows(omega, r_mode, dephasing):
    rng = np.random.Generator(np.random.PCG64(61))
    g = workloads.random_out_degree(6, 2, rng).dense()
    H, ML = operators.walk_operators(g, "laplacian", r_mode, dephasing)
    A = oracle.walk_superop(g, omega, "laplacian", r_mode, dephasing).dense()
    B = oracle.general_superop(H, operators.lindblad_ops(ML), omega).dense()
    assert np.abs(A - B).max() < 1e-14


def test_general_form_is_trace_preserving_and_hermiticity_preserving():
    rng = np.random.Generator(np.random.PCG64(62))
    N = 4
    X = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    H = X + X.conj().T
    Y = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    Hr = Y + Y.conj().T
    Ls = [rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)) for _ in range(2)]
    S = operators.general_rowmajor(H, Ls, 0.6, Hr)
    trace_row = np.eye(N).reshape(-1)
    assert np.abs(trace_row @ S).max() < 1e-12          # d tr(rho)/dt = 0
    rho = workloads.random_density(N, rng, rank=2)
    d = (S @ rho.reshape(-1)).reshape(N, N)
    assert np.abs(d - d.conj().T).max() < 1e-12          # stays Hermitian
    E = scipy.linalg.expm(0.7 * S)
    r = (E @ rho.reshape(-1)).reshape(N, N)
    assert np.linalg.eigvalsh(0.5 * (r + r.conj().T)).min() > -1e-12  # positive


def test_sink_closed_form():
    """One vertex drained by a sink at rate Theta: p(t) = exp(-Theta t)."""
    A = oracle.channel_superop(np.zeros((1, 1)), 0.3, [], [(0, 0.7)])
    out, _ = expmv.propagate(A, np.diag([1.0, 0.0]).astype(complex), 0.0, 0.5, 6)
    for k in range(7):
        p = np.real(out[k][0, 0])
        assert abs(p - np.exp(-0.35 * k)) < 1e-14
        assert abs(np.real(out[k][1, 1]) - (1 - np.exp(-0.35 * k))) < 1e-14


def test_source_into_graph_closed_form():
    """A source at rate Gamma feeding vertex 0 of an edgeless pair: the source
    population is exp(-Gamma t) and vertex 0 receives the rest."""
    A = oracle.channel_superop(np.zeros((2, 2)), 0.5, [(0, 1.3)], [])
    rho0 = np.zeros((3, 3), complex)
    rho0[2, 2] = 1.0
    out, _ = expmv.propagate(A, rho0, 0.0, 0.4, 5)
    for k in range(6):
        assert abs(np.real(out[k][2, 2]) - np.exp(-1.3 * 0.4 * k)) < 1e-14
        assert abs(np.real(out[k][0, 0]) - (1 - np.exp(-1.3 * 0.4 * k))) < 1e-14


def test_dimer_with_source_and_sink_invariants():
    """The dimer of the augmented-digraph figure (Section 2.5.1): source at
    rate 2 into v1, sink at rate 3 out of v2; trace one, populations
    non-negative, the sink fills monotonically and ends with everything."""
    G = np.array([[0.0, 1.0], [1.0, 0.0]])
    A = oracle.channel_superop(G, 0.5, [(0, 2.0)], [(1, 3.0)])
    rho0 = np.zeros((4, 4), complex)
    rho0[2, 2] = 1.0   # the walker starts in the source
    out, _ = expmv.propagate(A, rho0, 0.0, 1.0, 40)
    sink = [np.real(out[k][3, 3]) for k in range(41)]
    for k in range(41):
        assert abs(np.trace(out[k]) - 1) < 1e-12
        assert np.real(np.diag(out[k])).min() > -1e-12
    assert all(b >= a - 1e-14 for a, b in zip(sink, sink[1:]))
    assert sink[-1] > 1 - 1e-8


# ------------------------------------------------------------- demoralisation

def _nm_example():
    gold = json.load(open(os.path.join(GOLDEN, "nm_gqsw_example.json")))
    G = np.zeros((3, 3))
    for i, j in gold["graph_arcs_target_source"]:
        G[i, j] = 1.0
    return gold, G


def _nm_run(G, omega, t):
    d, HD, LD, Hr = operators.demoralise(G)
    A = oracle.general_superop(HD, [LD], omega, Hr)
    rho0 = operators.demoralised_state(np.diag([1.0, 0.0, 0.0]).astype(complex), d)
    out, _ = expmv.propagate(A, rho0, 0.0, t, 1)
    return d, operators.demoralised_populations(out[1], d)


def test_nm_gqsw_omega1_printed():
    """At omega = 1 nothing flows into v0, which loses population at the rate
    ||L_D |v0>||^2 = 1: p0 = e^-100, the printed 3.72007598e-44; v2 ends with
    everything (no spontaneous moralisation into v1)."""
    gold, G = _nm_example()
    d, p = _nm_run(G, 1.0, gold["t"])
    assert list(d) == [1, 1, 2]
    printed = gold["printed_populations"]["omega_1"]
    assert abs(p[0] - np.exp(-100.0)) < 1e-8 * np.exp(-100.0)
    assert abs(p[0] - printed[0]) < 5e-9 * printed[0]
    assert abs(p[1]) < 1e-30 and abs(p[2] - 1.0) < 1e-12


def test_nm_gqsw_omega0_closed_form_and_printed():
    """At omega = 0 the expanded graph's Laplacian has a uniform diagonal and
    v0, v1 couple to the symmetric copy of v2 with strength 1: populations are
    those of the CTQW on the star (cos^4, sin^4, sin^2(sqrt2 t)/2)."""
    gold, G = _nm_example()
    _, p = _nm_run(G, 0.0, gold["t"])
    t = gold["t"]
    closed = np.array([np.cos(t / np.sqrt(2)) ** 4, np.sin(t / np.sqrt(2)) ** 4,
                       0.5 * np.sin(np.sqrt(2) * t) ** 2])
    assert np.abs(p - closed).max() < 5e-12
    printed = np.array(gold["printed_populations"]["omega_0"])
    assert np.abs(p - printed).max() < 5e-9


def test_demoralised_operators_structure():
    rng = np.random.Generator(np.random.PCG64(63))
    G = workloads.random_out_degree(6, 2, rng).dense()
    d, HD, LD, Hr = operators.demoralise(G)
    indeg = (G != 0).sum(axis=1)
    assert (d == np.maximum(1, indeg)).all()
    assert np.abs(HD - HD.conj().T).max() < 1e-14
    assert np.abs(Hr - Hr.conj().T).max() < 1e-14
    # each parent w of v reaches v's copies through its own Fourier column:
    # the images of two different parents are orthogonal (no moralisation)
    off = np.concatenate([[0], np.cumsum(d)])
    for v in range(G.shape[0]):
        par = np.nonzero(G[v])[0]
        cols = [LD[off[v]:off[v + 1], off[w]] for w in par]
        for a in range(len(cols)):
            for b in range(a + 1, len(cols)):
                assert abs(np.vdot(cols[a], cols[b])) < 1e-12
    rho = workloads.random_density(6, rng, rank=2)
    rd = operators.demoralised_state(rho, d)
    assert abs(np.trace(rd) - 1) < 1e-14
    assert np.abs(operators.demoralised_populations(rd, d) - np.real(np.diag(rho))).max() < 1e-14


def test_library_host_maps_match_oracle():
    """The library's host-only demoralisation maps (no GPU needed)."""
    import paper_2003_02450_amd as qsw
    rng = np.random.Generator(np.random.PCG64(64))
    g = workloads.random_out_degree(7, 2, rng)
    d_lib = qsw.demoralised_copies(g)
    d, *_ = operators.demoralise(g.dense())
    assert (d_lib == d).all()
    rho = workloads.random_density(7, rng, rank=3)
    assert np.abs(qsw.demoralised_state(rho, d_lib) - operators.demoralised_state(rho, d)).max() < 1e-15
    pd = rng.random((3, int(d.sum())))
    ref = np.stack([operators.demoralised_populations(np.diag(x), d) for x in pd])
    assert np.abs(qsw.demoralised_populations(pd, d_lib) - ref).max() < 1e-14
