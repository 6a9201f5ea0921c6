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
    """The dimer of the augmented-digraph figure (Section 2.4.2): source at
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
