"""Oracle: graph -> walk operators (H, Lindblad rates, superoperator), dense.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file.

Everything here is plain dense numpy in float64/complex128, written to be
checked against the paper by eye:

* ``transition_matrix``   - eq. generator_matrix (Section 2.2): M_ij = -gamma G_ij
  for i != j, M_jj = gamma OutDeg(j), OutDeg(v_j) = sum_i G_ij (eq. out_degree).
* ``undirected``          - G^u_ij = max(G_ij, G_ji) (Section 2.1).
* ``walk_operators``      - H and the Lindblad operators of the L-QSW
  (Section 2.5.1, eq. lindblad): L_k = sqrt(|M_ij|) |v_i><v_j|.
* ``lindblad_ops``        - the explicit list of L_k matrices.
* ``superop_kron``        - the vectorised generator of eq. qsw built literally
  from the Kronecker mappings of eq. vec_mappings with column stacking
  (vec(XYZ) = (Z^T kron X) vec(Y)), one explicit L_k at a time.
* ``superop_kron_general``- the same for explicit operators: any list of
  L_k scaled by omega (the G-QSW of eq. L_global has one, L = G), the
  rotating Hamiltonian term omega i[H_rot, rho] of eq. nm_gqsw, and L_k
  outside omega (the absorption / emission channels of eq. qsw_ss).
* ``augmented``           - the augmented digraph of Section 2.5.1 (eq.
  dimer_aug): source and sink vertices appended after the graph's.

Conventions (readings of the paper, listed in the design notes):
* G[i, j] is the weight of the arc j -> i (row = target, column = source).
* ``h_mode``: "laplacian" -> H = transition matrix of G^u (= weighted graph
  Laplacian for gamma = 1); "adjacency" -> H = G^u (used by the paper's
  three-vertex example, which passes H = GU).
* ``r_mode``: "transition" -> L_k = sqrt(gamma G_ij) |i><j| for every arc;
  "colnorm" -> the column-normalised transition matrix, L_k = sqrt(G_ij /
  OutDeg(j)) |i><j| (eq. markov_chain rates).
* ``dephasing``: also keep the diagonal L_k = sqrt(|M_jj|) |j><j| that the
  sum over all N^2 indices k of eq. qsw contains.
"""
from __future__ import annotations

import numpy as np


def undirected(G: np.ndarray) -> np.ndarray:
    return np.maximum(G, G.T)


def out_degree(G: np.ndarray) -> np.ndarray:
    """OutDeg(v_j) = sum over i of G_ij (column sums)."""
    return G.sum(axis=0)


def transition_matrix(gamma: float, G: np.ndarray) -> np.ndarray:
    """eq. generator_matrix: off-diagonal -gamma G_ij, diagonal gamma OutDeg(j)."""
    N = G.shape[0]
    M = -gamma * G.astype(np.float64)
    M[np.arange(N), np.arange(N)] = gamma * out_degree(G)
    return M


def colnorm_transition_matrix(G: np.ndarray) -> np.ndarray:
    """CTRW transition matrix with unit total outflow from every vertex that
    has out-arcs: off-diagonal -G_ij / OutDeg(j), diagonal 1 (0 for sinks)."""
    N = G.shape[0]
    od = out_degree(G)
    M = np.zeros((N, N))
    for j in range(N):
        if od[j] > 0:
            M[:, j] = -G[:, j] / od[j]
            M[j, j] = 1.0
    return M


def walk_operators(G: np.ndarray, h_mode: str = "laplacian",
                   r_mode: str = "transition", dephasing: bool = False,
                   gamma: float = 1.0):
    """Return (H, ML) with H real symmetric N x N and ML the condensed
    Lindblad matrix (eq. condensed_lindblads): ML_ij = sqrt(|M_ij|) for every
    (i, j) that carries an L_k."""
    G = np.asarray(G, dtype=np.float64)
    N = G.shape[0]
    if np.any(np.diag(G) != 0):
        raise ValueError("simple graphs only (Tr G = 0)")
    if np.any(G < 0):
        raise ValueError("weights must be positive")
    Gu = undirected(G)
    if h_mode == "laplacian":
        H = transition_matrix(gamma, Gu)
    elif h_mode == "adjacency":
        H = Gu.copy()
    else:
        raise ValueError(h_mode)
    if r_mode == "transition":
        M = transition_matrix(gamma, G)
    elif r_mode == "colnorm":
        M = colnorm_transition_matrix(G)
    else:
        raise ValueError(r_mode)
    ML = np.sqrt(np.abs(M))
    if not dephasing:
        ML[np.arange(N), np.arange(N)] = 0.0
    return H, ML


def lindblad_ops(ML: np.ndarray):
    """The explicit list of L_k = ML_ij |v_i><v_j| for every nonzero ML_ij,
    k = N(j-1)+i order (column-major over (i, j))."""
    N = ML.shape[0]
    ops = []
    for j in range(N):
        for i in range(N):
            if ML[i, j] != 0:
                L = np.zeros((N, N), np.complex128)
                L[i, j] = ML[i, j]
                ops.append(L)
    return ops


def superop_kron(H: np.ndarray, ML: np.ndarray, omega: float) -> np.ndarray:
    """Dense N^2 x N^2 generator of eq. qsw acting on the COLUMN-STACKED
    vec(rho) (index i + N j <-> rho_ij), from eq. vec_mappings:

      -i(1-omega) (I kron H - H^T kron I)
      + omega sum_k [ conj(L_k) kron L_k
                      - 1/2 (I kron L_k^dag L_k + (L_k^dag L_k)^T kron I) ]
    """
    N = H.shape[0]
    I = np.eye(N)
    Hc = np.asarray(H, dtype=np.complex128)
    S = -1j * (1.0 - omega) * (np.kron(I, Hc) - np.kron(Hc.T, I))
    for L in lindblad_ops(ML):
        LdL = L.conj().T @ L
        S = S + omega * (np.kron(L.conj(), L)
                         - 0.5 * (np.kron(I, LdL) + np.kron(LdL.T, I)))
    return S


def colstack_to_rowmajor(N: int) -> np.ndarray:
    """perm[r] = column-stacked index of the row-major index r = a N + b,
    i.e. rho_ab: rowmajor a N + b  <->  colstack a + N b."""
    r = np.arange(N * N)
    a, b = r // N, r % N
    return a + N * b


def superop_kron_rowmajor(H, ML, omega) -> np.ndarray:
    """superop_kron permuted to act on the row-major vec(rho) (index a N + b)."""
    N = H.shape[0]
    S = superop_kron(H, ML, omega)
    p = colstack_to_rowmajor(N)
    return S[np.ix_(p, p)]


def dissipator_kron(L: np.ndarray) -> np.ndarray:
    """D[L] rho = L rho L^dag - 1/2 {L^dag L, rho} on the column-stacked vec."""
    N = L.shape[0]
    I = np.eye(N)
    LdL = L.conj().T @ L
    return np.kron(L.conj(), L) - 0.5 * (np.kron(I, LdL) + np.kron(LdL.T, I))


def commutator_kron(M: np.ndarray) -> np.ndarray:
    """[M, rho] on the column-stacked vec."""
    N = M.shape[0]
    I = np.eye(N)
    return np.kron(I, M) - np.kron(M.T, I)


def superop_kron_general(H, Ls, omega, H_rot=None, Ls_free=()) -> np.ndarray:
    """-i(1-omega)[H, .] + omega (i[H_rot, .] + sum_k D[L_k]) + sum_f D[F_f],
    column-stacked, dense."""
    Hc = np.asarray(H, dtype=np.complex128)
    S = -1j * (1.0 - omega) * commutator_kron(Hc)
    if H_rot is not None:
        S = S + 1j * omega * commutator_kron(np.asarray(H_rot, dtype=np.complex128))
    for L in Ls:
        S = S + omega * dissipator_kron(np.asarray(L, dtype=np.complex128))
    for F in Ls_free:
        S = S + dissipator_kron(np.asarray(F, dtype=np.complex128))
    return S


def general_rowmajor(H, Ls, omega, H_rot=None, Ls_free=()) -> np.ndarray:
    N = np.asarray(H).shape[0]
    S = superop_kron_general(H, Ls, omega, H_rot, Ls_free)
    p = colstack_to_rowmajor(N)
    return S[np.ix_(p, p)]


def augmented(G: np.ndarray, sources, sinks):
    """(G_aug on N + len(sources) + len(sinks) vertices with the graph's arcs
    only, the list of channel operators).  Source k is vertex N + k and feeds
    sources[k] = (vertex, Gamma) through L = sqrt(Gamma)|vertex><N + k|; sink k
    is vertex N + len(sources) + k and drains sinks[k] = (vertex, Theta)
    through L = sqrt(Theta)|sink><vertex|."""
    N = G.shape[0]
    M = N + len(sources) + len(sinks)
    Ga = np.zeros((M, M))
    Ga[:N, :N] = G
    chans = []
    for k, (v, rate) in enumerate(sources):
        L = np.zeros((M, M), np.complex128)
        L[v, N + k] = np.sqrt(rate)
        chans.append(L)
    for k, (v, rate) in enumerate(sinks):
        L = np.zeros((M, M), np.complex128)
        L[N + len(sources) + k, v] = np.sqrt(rate)
        chans.append(L)
    return Ga, chans


def demoralise(G: np.ndarray, gamma: float = 1.0):
    """The non-moralising construction of Section 2.5.2 (graph demoralisation),
    dense: returns (copies, H_D, L_D, H_rot) on the expanded vertex set.

    * Vertex v keeps d_v = max(1, number of arcs into v) copies, numbered
      consecutively (vertex v's copies after those of vertices < v).
    * Two copies are joined when their vertices are (G^u for H_D, the arcs of
      G for L_D), with weight G_vw / sqrt(d_v d_w) (eq. nm_weight, the number
      of joined copy pairs being d_v d_w).
    * H_D is the transition matrix of that weighted graph (eq. generator_matrix).
    * L_D takes copy u of a parent w of v to copy k of v with coefficient
      F_v[k, m] G^D_vw, m the rank of w among v's parents and F_v the Fourier
      matrix exp(2 pi i k m / d_v) (unit-modulus entries) (eq. dm_lind).
    * H_rot couples consecutive copies of one vertex: +i from copy k to k+1,
      -i back (eq. H_rot), cyclically when d_v > 2.
    """
    G = np.asarray(G, dtype=float)
    N = G.shape[0]
    parents = [np.nonzero(G[v, :])[0] for v in range(N)]
    d = np.array([max(1, len(p)) for p in parents])
    off = np.concatenate([[0], np.cumsum(d)])
    M = int(off[-1])
    Gu = undirected(G)
    A = np.zeros((M, M))
    for v in range(N):
        for w in range(N):
            if Gu[v, w] != 0:
                A[off[v]:off[v + 1], off[w]:off[w + 1]] = Gu[v, w] / np.sqrt(d[v] * d[w])
    H_D = transition_matrix(gamma, A)
    L_D = np.zeros((M, M), np.complex128)
    for v in range(N):
        F = np.exp(2j * np.pi * np.outer(np.arange(d[v]), np.arange(d[v])) / d[v])
        for m, w in enumerate(parents[v]):
            g = G[v, w] / np.sqrt(d[v] * d[w])
            for k in range(d[v]):
                for u in range(d[w]):
                    L_D[off[v] + k, off[w] + u] = F[k, m] * g
    H_rot = np.zeros((M, M), np.complex128)
    for v in range(N):
        if d[v] < 2:
            continue
        links = [(k, k + 1) for k in range(d[v] - 1)]
        if d[v] > 2:
            links.append((d[v] - 1, 0))
        for k, l in links:
            H_rot[off[v] + l, off[v] + k] = 1j
            H_rot[off[v] + k, off[v] + l] = -1j
    return d, H_D, L_D, H_rot


def demoralised_state(rho: np.ndarray, copies) -> np.ndarray:
    """rho on the graph -> V rho V^dag with V|v> = d_v^(-1/2) sum_k |v^k>:
    trace and positivity kept, populations spread evenly over the copies."""
    N = rho.shape[0]
    d = np.asarray(copies)
    off = np.concatenate([[0], np.cumsum(d)])
    V = np.zeros((int(off[-1]), N))
    for v in range(N):
        V[off[v]:off[v + 1], v] = 1.0 / np.sqrt(d[v])
    return V @ rho @ V.T


def demoralised_populations(rho_d: np.ndarray, copies) -> np.ndarray:
    """p(v) = sum over the copies of v of the diagonal (eq. nm_rho_map)."""
    d = np.asarray(copies)
    off = np.concatenate([[0], np.cumsum(d)])
    diag = np.real(np.diag(rho_d))
    return np.array([diag[off[v]:off[v + 1]].sum() for v in range(d.size)])
