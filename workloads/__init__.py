"""Seeded synthetic inputs for the quantum-stochastic-walk propagator.

This module only draws graphs, weights and initial states.  It holds none of
the walk's arithmetic (no transition matrices, no superoperator, no
exponential), so both the CPU oracle and the GPU path can consume its output
without sharing any of the method.

Graph convention (Section 2.1, adjacency equation): a digraph on N vertices is
a CSR matrix G with ``G[i, j] = w(v_i, v_j) > 0`` meaning an arc from source
vertex j to target vertex i (row = target, column = source); the diagonal is
empty (simple graphs only).  Every generator returns ``Graph`` with int64
``row_ptr``, int32 ``col_idx`` (sorted within each row, no duplicates) and
float64 ``w``.

Every instance draws from one ``numpy.random.Generator(PCG64(seed))``; the
base seed of the named workloads is 2003 plus the instance index.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2003


@dataclasses.dataclass
class Graph:
    N: int
    row_ptr: np.ndarray  # int64 [N+1]
    col_idx: np.ndarray  # int32 [nnz]
    w: np.ndarray        # float64 [nnz]

    @property
    def n_arcs(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        """Dense N x N adjacency (row = target, column = source)."""
        A = np.zeros((self.N, self.N))
        for i in range(self.N):
            lo, hi = self.row_ptr[i], self.row_ptr[i + 1]
            A[i, self.col_idx[lo:hi]] = self.w[lo:hi]
        return A


@dataclasses.dataclass
class Workload:
    """One propagation job: graph, walk options, initial state and time grid."""
    name: str
    graph: Graph
    omega: float
    h_mode: str          # "laplacian" | "adjacency"
    r_mode: str          # "transition" | "colnorm"
    dephasing: bool
    rho0: np.ndarray     # complex128 N x N
    t0: float
    dt: float
    n_steps: int
    gamma: float = 1.0


def graph_from_arcs(N: int, tgt, src, w) -> Graph:
    """Build the CSR of G from arc lists (target, source, weight)."""
    tgt = np.asarray(tgt, dtype=np.int64)
    src = np.asarray(src, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    if tgt.size:
        if np.any(tgt == src):
            raise ValueError("self-loops are not allowed")
        key = tgt * N + src
        order = np.argsort(key, kind="stable")
        key, w = key[order], w[order]
        if np.any(key[1:] == key[:-1]):
            raise ValueError("duplicate arcs")
        tgt, src = key // N, key % N
    counts = np.bincount(tgt, minlength=N) if tgt.size else np.zeros(N, np.int64)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(N, row_ptr, src.astype(np.int32), w.copy())


def _unit_interval_open_low(rng, size):
    """U(0, 1] draws: arc weights must be strictly positive."""
    return 1.0 - rng.random(size)


def _undirected(N, pairs_i, pairs_j, weights):
    tgt = np.concatenate([pairs_i, pairs_j])
    src = np.concatenate([pairs_j, pairs_i])
    w = np.concatenate([weights, weights])
    return graph_from_arcs(N, tgt, src, w)


# ---------------------------------------------------------------------------
# Graph families
# ---------------------------------------------------------------------------

def cycle_graph(N: int, weight: float = 1.0) -> Graph:
    """Undirected cycle C_N (arcs both ways), unit weights by default."""
    i = np.arange(N)
    j = (i + 1) % N
    return _undirected(N, i, j, np.full(N, weight))


def er_undirected(N: int, p: float, rng, wlo=1.0, whi=1.0) -> Graph:
    """Erdos-Renyi G(N, p), symmetric weights U(wlo, whi) (constant if equal)."""
    iu, ju = np.triu_indices(N, k=1)
    keep = rng.random(iu.size) < p
    iu, ju = iu[keep], ju[keep]
    if whi > wlo:
        w = rng.uniform(wlo, whi, size=iu.size)
    else:
        w = np.full(iu.size, float(wlo))
    return _undirected(N, iu, ju, w)


def random_out_degree(N: int, k: int, rng) -> Graph:
    """Each vertex j sends arcs to k distinct uniform targets != j, w ~ U(0,1]."""
    tgt = np.empty(N * k, np.int64)
    for j in range(N):
        cand = rng.choice(N - 1, size=k, replace=False)
        cand = cand + (cand >= j)  # skip j itself
        tgt[j * k:(j + 1) * k] = cand
    src = np.repeat(np.arange(N, dtype=np.int64), k)
    w = _unit_interval_open_low(rng, N * k)
    return graph_from_arcs(N, tgt, src, w)


def er_mixed_direction(N: int, mean_degree: float, p_directed: float, rng) -> Graph:
    """ER graph with p = mean_degree/(N-1); each edge is one random arc with
    probability p_directed, else arcs both ways; unit weights."""
    p = min(1.0, mean_degree / max(N - 1, 1))
    iu, ju = np.triu_indices(N, k=1)
    keep = rng.random(iu.size) < p
    iu, ju = iu[keep], ju[keep]
    directed = rng.random(iu.size) < p_directed
    flip = rng.random(iu.size) < 0.5
    a = np.where(flip, ju, iu)
    b = np.where(flip, iu, ju)
    tgt = np.concatenate([a[directed], iu[~directed], ju[~directed]])
    src = np.concatenate([b[directed], ju[~directed], iu[~directed]])
    return graph_from_arcs(N, tgt, src, np.ones(tgt.size))


def line_digraph(N: int, rng) -> Graph:
    """Directed path v0 -> v1 -> ... -> v_{N-1}, w ~ U(0,1]."""
    src = np.arange(N - 1)
    return graph_from_arcs(N, src + 1, src, _unit_interval_open_low(rng, N - 1))


def lattice_digraph(side: int, rng) -> Graph:
    """side x side square lattice, each lattice edge one arc of random
    orientation, w ~ U(0,1]."""
    N = side * side
    idx = np.arange(N).reshape(side, side)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    flip = rng.random(a.size) < 0.5
    src = np.where(flip, b, a)
    tgt = np.where(flip, a, b)
    return graph_from_arcs(N, tgt, src, _unit_interval_open_low(rng, a.size))


def er_digraph_nlogn(N: int, rng) -> Graph:
    """Directed ER graph with floor(N ln N) distinct arcs, w ~ U(0,1]."""
    m = int(math.floor(N * math.log(N)))
    chosen = rng.choice(N * (N - 1), size=m, replace=False)
    src = chosen // (N - 1)
    r = chosen % (N - 1)
    tgt = r + (r >= src)
    return graph_from_arcs(N, tgt, src, _unit_interval_open_low(rng, m))


def complete_digraph(N: int, rng) -> Graph:
    """All N(N-1) arcs, w ~ U(0,1]."""
    i, j = np.nonzero(~np.eye(N, dtype=bool))
    return graph_from_arcs(N, i, j, _unit_interval_open_low(rng, i.size))


# ---------------------------------------------------------------------------
# Initial states
# ---------------------------------------------------------------------------

def basis_state(N: int, v: int = 0) -> np.ndarray:
    rho = np.zeros((N, N), np.complex128)
    rho[v, v] = 1.0
    return rho


def uniform_superposition(N: int) -> np.ndarray:
    """Pure state |s><s| with |s> = (1/sqrt N) sum_v |v>."""
    return np.full((N, N), 1.0 / N, np.complex128)


def maximally_mixed(N: int) -> np.ndarray:
    return np.eye(N, dtype=np.complex128) / N


def random_density(N: int, rng, rank: int = 2) -> np.ndarray:
    """A random mixed state of the given rank (Hermitian, PSD, unit trace)."""
    X = rng.standard_normal((N, rank)) + 1j * rng.standard_normal((N, rank))
    rho = X @ X.conj().T
    return rho / np.trace(rho).real


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def cycle16() -> Workload:
    """Cycle N=16, unit weights, omega=0.5, Laplacian H, column-normalised
    rates, rho0=|0><0|, t = 0..10 (11 points)."""
    g = cycle_graph(16)
    return Workload("cycle16", g, 0.5, "laplacian", "colnorm", False,
                    basis_state(16), 0.0, 1.0, 10)


def er256(seed: int = BASE_SEED + 1) -> Workload:
    """ER undirected N=256, p=0.05, w~U(0.5,1.5), omega=0.1, uniform
    superposition, t = 0..100 (101 points)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = er_undirected(256, 0.05, rng, 0.5, 1.5)
    return Workload("er256", g, 0.1, "laplacian", "transition", False,
                    uniform_superposition(256), 0.0, 1.0, 100)


def outdeg1024(seed: int = BASE_SEED + 2, N: int = 1024, k: int = 10,
               n_steps: int = 50) -> Workload:
    """Directed N=1024, out-degree 10 to uniform targets, w~U(0,1),
    omega=0.5, rho0=|0><0|, t = 0..50 (51 points)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = random_out_degree(N, k, rng)
    return Workload(f"outdeg{N}", g, 0.5, "laplacian", "transition", False,
                    basis_state(N), 0.0, 1.0, n_steps)


def paper_shaped(kind: str, seed: int = BASE_SEED + 10) -> Workload:
    """The four benchmark digraph shapes of Section 5 (about 1.28e8
    superoperator non-zeros each): line N=5050, 62x62 lattice, ER N=2020
    with floor(N ln N) arcs, complete N=400; w ~ U(0,1); maximally mixed
    rho0; omega=0.5 (the paper does not state it); one step to t=100."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "line":
        g = line_digraph(5050, rng)
    elif kind == "lattice":
        g = lattice_digraph(62, rng)
    elif kind == "er":
        g = er_digraph_nlogn(2020, rng)
    elif kind == "complete":
        g = complete_digraph(400, rng)
    else:
        raise ValueError(kind)
    return Workload(f"paper_{kind}", g, 0.5, "laplacian", "transition", False,
                    maximally_mixed(g.N), 0.0, 100.0, 1)


def two_sources_one_sink() -> tuple[Graph, Graph]:
    """The 3-vertex digraph of the demoralisation walkthrough (Section 4):
    arcs v0 -> v2 and v1 -> v2, unit weights; returns (G, G^u)."""
    G = graph_from_arcs(3, [2, 2], [0, 1], [1.0, 1.0])
    Gu = graph_from_arcs(3, [0, 1, 2, 2], [2, 2, 0, 1], [1.0] * 4)
    return G, Gu


def basis_states(N: int, vertices) -> np.ndarray:
    """[len(vertices), N, N] stack of |v><v|."""
    out = np.zeros((len(vertices), N, N), np.complex128)
    for i, v in enumerate(vertices):
        out[i, v, v] = 1.0
    return out


def batch64(seed: int = BASE_SEED + 20, count: int = 64, n0: int = 4, n_steps: int = 100,
            dt: float = 0.2, n_lo: int = 32, n_hi: int = 512) -> list:
    """Many small walks: `count` undirected ER graphs with
    N = round(exp(U(ln n_lo, ln n_hi))), p = 8 / N, unit weights, omega ~ U(0, 1),
    `n0` distinct basis states |v><v| per graph, t = 0 .. n_steps dt.
    Each item is a Workload whose rho0 is the [n0, N, N] stack."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        g = er_undirected(N, min(1.0, 8.0 / N), rng)
        omega = float(rng.uniform(0.0, 1.0))
        verts = rng.choice(N, size=min(n0, N), replace=False)
        out.append(Workload(f"batch{i}_N{N}", g, omega, "laplacian", "transition", False,
                            basis_states(N, verts), 0.0, dt, n_steps))
    return out


def served_requests(count: int, seed: int = BASE_SEED + 30, n_lo: int = 16, n_hi: int = 2048,
                    t_end: float = 10.0) -> list:
    """Walks for the serving workload: N = round(exp(U(ln n_lo, ln n_hi))),
    ER with mean degree 6 where each edge is one random arc with probability
    0.1 (else arcs both ways), unit weights, omega ~ U(0, 1), n_points ~
    U{10..200} grid steps over t in [0, t_end], rho0 = |0><0|.  Each item is a
    dict with graph, omega, n_steps, dt."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        g = er_mixed_direction(N, 6.0, 0.1, rng)
        omega = float(rng.uniform(0.0, 1.0))
        steps = int(rng.integers(10, 201))
        out.append({"graph": g, "omega": omega, "n_steps": steps, "dt": t_end / steps})
    return out


def poisson_arrivals(count: int, qps: float, seed: int = BASE_SEED + 31) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
