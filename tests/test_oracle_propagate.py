"""Pins for the oracle's propagation: closed forms at omega = 0 and 1, the
paper's printed three-vertex results, density-matrix invariants, the
maximally mixed fixed point, step vs series, dense expm and scipy."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import oracle
import workloads
from oracle import dense, expmv, native, operators

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cycle_wl(omega, r_mode="colnorm", N=16):
    g = workloads.cycle_graph(N)
    return workloads.Workload("c", g, omega, "laplacian", r_mode, False,
                              workloads.basis_state(N), 0.0, 1.0, 10)


# ---------------------------------------------------------------- omega = 0

def test_cycle_omega0_matches_ctqw_closed_form():
    """omega = 0: rho(t) = |psi(t)><psi(t)| with psi = exp(-iHt)|0> (eq. CTQW).
    For the cycle Laplacian the eigenvectors are Fourier modes with
    lambda_k = 2 - 2 cos(2 pi k / N)."""
    N = 16
    wl = _cycle_wl(0.0, N=N)
    out, _ = oracle.run_workload(wl)
    k = np.arange(N)
    lam = 2 - 2 * np.cos(2 * np.pi * k / N)
    for step in range(wl.n_steps + 1):
        t = step * wl.dt
        a = np.arange(N)
        psi = (np.exp(-1j * lam[None, :] * t)
               * np.exp(2j * np.pi * np.outer(a, k) / N)).sum(axis=1) / N
        rho = np.outer(psi, psi.conj())
        assert np.abs(out[step] - rho).max() < 1e-12


def test_random_graph_omega0_matches_eigh():
    rng = np.random.Generator(np.random.PCG64(5))
    g = workloads.er_undirected(12, 0.4, rng, 0.5, 1.5)
    H, ML = operators.walk_operators(g.dense())
    lam, V = np.linalg.eigh(H)
    A = native.superop_csr(H, ML, 0.0)
    rho0 = workloads.random_density(12, rng, rank=3)
    out, _ = expmv.propagate(A, rho0, 0.0, 0.7, 6)
    for k in range(7):
        U = (V * np.exp(-1j * lam * 0.7 * k)) @ V.conj().T
        assert np.abs(out[k] - U @ rho0 @ U.conj().T).max() < 1e-12


# ---------------------------------------------------------------- omega = 1

def test_cycle_omega1_matches_ctrw_closed_form():
    """omega = 1: populations obey dp/dt = -M p (eq. CTRW) with the
    column-normalised rates 1/2: p_a(t) = (1/N) sum_k exp(-(1 - cos(2 pi k/N)) t)
    cos(2 pi k a / N); coherences stay zero for diagonal rho0."""
    N = 16
    wl = _cycle_wl(1.0, N=N)
    out, _ = oracle.run_workload(wl)
    k = np.arange(N)
    lam = 1 - np.cos(2 * np.pi * k / N)
    for step in range(wl.n_steps + 1):
        t = step * wl.dt
        p = (np.exp(-lam[None, :] * t)
             * np.cos(2 * np.pi * np.outer(np.arange(N), k) / N)).sum(axis=1) / N
        assert np.abs(np.diag(out[step]).real - p).max() < 1e-12
        off = out[step] - np.diag(np.diag(out[step]))
        assert np.abs(off).max() < 1e-15


def test_directed_omega1_matches_classical_generator():
    rng = np.random.Generator(np.random.PCG64(9))
    g = workloads.random_out_degree(10, 3, rng)
    G = g.dense()
    H, ML = operators.walk_operators(G)
    A = native.superop_csr(H, ML, 1.0)
    M = operators.transition_matrix(1.0, G)
    p0 = rng.random(10)
    p0 /= p0.sum()
    out, _ = expmv.propagate(A, np.diag(p0).astype(complex), 0.0, 0.5, 8)
    for k in range(9):
        p = scipy.linalg.expm(-0.5 * k * M) @ p0
        assert np.abs(np.diag(out[k]).real - p).max() < 1e-13


# ------------------------------------------------- the paper's printed example

def _three_vertex(omega):
    spec = json.load(open(os.path.join(GOLDEN, "three_vertex_example.json")))
    G, _ = workloads.two_sources_one_sink()
    A = oracle.walk_superop(G.dense(), omega, h_mode="adjacency")
    out, _ = expmv.propagate(A, workloads.basis_state(3), 0.0, spec["t"], 1)
    return spec, np.diag(out[1]).real


def test_three_vertex_omega0_printed_and_closed_form():
    spec, p = _three_vertex(0.0)
    t = spec["t"]
    # CTQW on the star with centre v2: p = [cos^4(t/sqrt2), sin^4(t/sqrt2),
    # sin^2(sqrt2 t)/2]
    closed = np.array([math.cos(t / math.sqrt(2)) ** 4,
                       math.sin(t / math.sqrt(2)) ** 4,
                       0.5 * math.sin(math.sqrt(2) * t) ** 2])
    assert np.abs(p - closed).max() < 1e-12
    printed = np.array(spec["printed_populations"]["omega_0"])
    # printed to 9 significant digits; the paper's own value differs from the
    # closed form by 5.7e-14 in the first entry
    assert np.abs(p - printed).max() < 5e-9
    assert abs(p[0] - printed[0]) < 1e-13


def test_three_vertex_omega1_printed_and_closed_form():
    spec, p = _three_vertex(1.0)
    t = spec["t"]
    closed = np.array([math.exp(-t), 0.0, 1 - math.exp(-t)])
    assert np.abs(p - closed).max() < 1e-12
    printed = np.array(spec["printed_populations"]["omega_1"])
    assert np.abs(p - printed).max() < 1e-12


# ------------------------------------------------------------- invariants

def _check_density(rho, pure=False):
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))
    assert ev.min() > -1e-12
    pur = np.trace(rho @ rho).real
    assert pur <= 1 + 1e-12
    if pure:
        assert abs(pur - 1) < 1e-12


@pytest.mark.parametrize("omega", [0.0, 0.3, 0.9, 1.0])
def test_invariants_random_directed(omega):
    rng = np.random.Generator(np.random.PCG64(21))
    g = workloads.random_out_degree(9, 3, rng)
    A = oracle.walk_superop(g.dense(), omega)
    rho0 = workloads.random_density(9, rng, rank=2)
    out, _ = expmv.propagate(A, rho0, 0.0, 1.5, 6)
    for k in range(7):
        _check_density(out[k])
    rho_pure = workloads.uniform_superposition(9)
    out, _ = expmv.propagate(A, rho_pure, 0.0, 1.5, 4)
    for k in range(5):
        _check_density(out[k], pure=(omega == 0.0))


@pytest.mark.parametrize("omega", [0.0, 0.5, 1.0])
def test_maximally_mixed_is_fixed_on_regular_graph(omega):
    """Section 4: on regular graphs the stationary state shows no coherence;
    I/N is a fixed point of eq. qsw for symmetric rates."""
    N = 16
    wl = _cycle_wl(omega, r_mode="transition", N=N)
    A = oracle.walk_superop(wl.graph.dense(), omega)
    out, _ = expmv.propagate(A, workloads.maximally_mixed(N), 0.0, 10.0, 3)
    for k in range(4):
        assert np.abs(out[k] - np.eye(N) / N).max() < 1e-14


def test_linearity_mixed_equals_sum_of_pure():
    rng = np.random.Generator(np.random.PCG64(4))
    g = workloads.random_out_degree(8, 2, rng)
    A = oracle.walk_superop(g.dense(), 0.4)
    X = rng.standard_normal((8, 2)) + 1j * rng.standard_normal((8, 2))
    X /= np.linalg.norm(X, axis=0)
    p = np.array([0.3, 0.7])
    parts = [np.outer(X[:, i], X[:, i].conj()) for i in range(2)]
    mixed = p[0] * parts[0] + p[1] * parts[1]
    out_m, _ = expmv.propagate(A, mixed, 0.0, 1.0, 3)
    out_0, _ = expmv.propagate(A, parts[0], 0.0, 1.0, 3)
    out_1, _ = expmv.propagate(A, parts[1], 0.0, 1.0, 3)
    assert np.abs(out_m - (p[0] * out_0 + p[1] * out_1)).max() < 1e-14


# ------------------------------------------------------- step vs series

def test_series_both_branches_match_step():
    """Section 5 reports step vs series agreement to 1e-14 or below."""
    wl = workloads.cycle16()
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode)
    step, info = expmv.propagate(A, wl.rho0, 0.0, 1.0, 10)
    ser, sinfo = expmv.series(A, wl.rho0, 0.0, 10.0, 10)
    assert sinfo["branch"] == "q>s"
    assert np.abs(step - ser).max() < 1e-13
    # a long grid with few points: q <= s
    ser2, sinfo2 = expmv.series(A, wl.rho0, 0.0, 40.0, 2)
    step2, _ = expmv.propagate(A, wl.rho0, 0.0, 20.0, 2)
    assert sinfo2["branch"] == "q<=s"
    assert np.abs(step2 - ser2).max() < 1e-13


def test_series_with_start_time_and_resume():
    wl = workloads.cycle16()
    A = oracle.walk_superop(wl.graph.dense(), 0.7)
    full, _ = expmv.propagate(A, wl.rho0, 0.0, 0.5, 12)
    tail, _ = expmv.propagate(A, wl.rho0, 2.0, 0.5, 8)
    assert np.abs(full[4:] - tail).max() < 1e-13
    resumed, _ = expmv.propagate(A, full[6], 3.0 - 3.0, 0.5, 6)
    assert np.abs(full[6:] - resumed).max() < 1e-13


# -------------------------------------------------- dense and library checks

def test_dense_expm_rotation_closed_form():
    for a in (0.1, 1.0, 7.5, 40.0):
        A = np.array([[0.0, -a], [a, 0.0]])
        E = dense.expm(A)
        assert np.abs(E - np.array([[math.cos(a), -math.sin(a)],
                                    [math.sin(a), math.cos(a)]])).max() < 1e-13


def test_dense_expm_and_taylor_agree_with_scipy_on_cycle16():
    wl = workloads.cycle16()
    H, ML = operators.walk_operators(wl.graph.dense(), wl.h_mode, wl.r_mode)
    S = operators.superop_kron_rowmajor(H, ML, wl.omega)
    out, _ = oracle.run_workload(wl)
    v0 = wl.rho0.reshape(-1)
    for k in (1, 5, 10):
        E = dense.expm(k * S)
        assert np.abs(E - scipy.linalg.expm(k * S)).max() < 1e-13
        assert np.abs(E @ v0 - out[k].reshape(-1)).max() < 1e-13


def test_expmv_agrees_with_scipy_expm_multiply():
    rng = np.random.Generator(np.random.PCG64(12))
    g = workloads.er_undirected(48, 0.1, rng, 0.5, 1.5)
    A = oracle.walk_superop(g.dense(), 0.1)
    rho0 = workloads.uniform_superposition(48)
    out, _ = expmv.propagate(A, rho0, 0.0, 1.0, 5)
    S = scipy.sparse.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    ref = scipy.sparse.linalg.expm_multiply(S, rho0.reshape(-1), start=0.0,
                                            stop=5.0, num=6, endpoint=True)
    assert np.abs(out.reshape(6, -1) - ref).max() < 1e-12


# -------------------------------------------------- parameter selection

def test_select_params_norm1_properties():
    th = oracle.theta.theta_table()
    for x in (1e-3, 0.5, 3.0, 30.0, 63.0, 500.0):
        m, s = expmv.select_params_norm1(x)
        assert 1 <= m <= 55 and s >= 1
        assert x / s <= th[m - 1] * (1 + 1e-15)
        # no (m', s') with m' s' < m s satisfies the bound
        for mm in range(1, 56):
            assert mm * math.ceil(x / th[mm - 1]) >= m * s
    assert expmv.select_params_norm1(0.0) == (0, 1)


def test_select_params_alpha_never_worse_than_norm1():
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(200):
        nrm = float(rng.uniform(0.1, 50))
        d = {p: nrm * float(rng.uniform(0.05, 1.0)) for p in range(2, 10)}
        t = float(10 ** rng.uniform(-1, 2.5))
        m, s = expmv.select_params(nrm, d, t)
        m1, s1 = expmv.select_params_norm1(t * nrm)
        assert m * s <= m1 * s1


# ------------------------------------------- complex64-stored values variant

def test_single_values_rounding_is_componentwise_nearest():
    rng = np.random.Generator(np.random.PCG64(31))
    g = workloads.er_undirected(10, 0.5, rng, 0.5, 1.5)
    A = oracle.walk_superop(g.dense(), 0.37)
    A32 = expmv.round_values_c64(A)
    assert (A32.row_ptr == A.row_ptr).all() and (A32.col == A.col).all()
    for part in (np.real, np.imag):
        d = np.abs(part(A32.val) - part(A.val))
        assert (d <= 2.0 ** -24 * np.abs(part(A.val))).all()
        assert (part(A32.val) == part(A32.val).astype(np.float32)).all()
    assert (A32.val != A.val).any()


def test_single_values_exact_storage_reduces_to_truncation_error():
    """The 16-cycle with unit weights, rates equal to the weights and
    omega = 0.5 has only dyadic superoperator entries, so complex64 storage
    is exact and the variant differs from exp(tA) (scipy's dense expm) only
    by the 2^-24 truncation: at most u |t| ||A||_1 ||vec rho0||_1."""
    wl = _cycle_wl(0.5, r_mode="transition")
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                            wl.dephasing, wl.gamma)
    assert (expmv.round_values_c64(A).val == A.val).all()
    out, info = expmv.propagate_single_values(A, wl.rho0, 0.0, wl.dt, wl.n_steps)
    S = A.dense()
    v0 = wl.rho0.reshape(-1)
    for k in (1, 4, 10):
        ref = scipy.linalg.expm(k * wl.dt * S) @ v0
        err = np.abs(out[k].reshape(-1) - ref).max()
        assert err <= 2.0 ** -24 * k * wl.dt * info["norm1"] * np.abs(v0).sum()
    _, info64 = expmv.propagate(A, wl.rho0, 0.0, wl.dt, wl.n_steps)
    assert info["m"] < info64["m"]   # theta_m at 2^-24 is larger


@pytest.mark.parametrize("omega,t0", [(0.0, 0.0), (0.4, 0.0), (0.9, 0.6)])
def test_single_values_within_first_order_bound(omega, t0):
    rng = np.random.Generator(np.random.PCG64(32))
    g = workloads.random_out_degree(14, 3, rng)
    A = oracle.walk_superop(g.dense(), omega)
    rho0 = workloads.random_density(14, rng, rank=2)
    out, info = expmv.propagate_single_values(A, rho0, t0, 0.9, 4)
    S = A.dense()
    for k in range(5):
        t = t0 + 0.9 * k
        ref = scipy.linalg.expm(t * S) @ rho0.reshape(-1)
        err = np.abs(out[k].reshape(-1) - ref).max()
        assert err <= max(expmv.single_values_bound(info["norm1"], t, rho0), 1e-15), (k, err)
        assert err > 1e-12 or t == 0.0   # the rounding is really there


def test_fullgrid_fixture_is_the_oracles():
    """The committed N = 1024 full-grid fixture (tests/golden/make_fullgrid.py)
    holds the oracle's own values: its first interval recomputed here agrees
    bit for bit, and every stored point has unit trace."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_fullgrid", os.path.join(GOLDEN, "make_fullgrid.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    hdr, fx = mod.load("outdeg1024")
    pops, samples, trace = fx["pops"], fx["samples"], fx["trace"]
    wl = workloads.outdeg1024()
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                            wl.dephasing, wl.gamma)
    out, info = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, 1)
    n = wl.graph.N ** 2
    assert (hdr["oracle"]["m"], hdr["oracle"]["s"]) == (info["m"], info["s"])
    for k in (0, 1):
        assert np.array_equal(np.diag(out[k]).real, pops[k])
        assert np.array_equal(out[k].reshape(-1)[mod.sample_indices(n, k)], samples[k])
    assert np.abs(trace - 1).max() < 1e-12
    assert fx["vec1"][0] == 1.0 and abs(fx["vec1"][1] - np.abs(out[1]).sum()) < 1e-12
    assert len(np.unique(mod.sample_indices(n, 3))) == mod.SAMPLES


def test_served_fixture_is_the_oracles():
    """The committed serving-workload fixture (tests/golden/make_served.py)
    holds the oracle's populations of the sampled walks of the serving stream:
    the smallest one recomputed here agrees bit for bit; every point's
    populations sum to 1 and lie in [0, 1]."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_served", os.path.join(GOLDEN, "make_served.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    hdr, pops = mod.load()
    assert len(pops) == mod.SAMPLES
    reqs = workloads.served_requests(mod.MIN_COUNT)
    for w in hdr["walks"]:
        r = reqs[w["index"]]
        assert r["graph"].N == w["N"] <= mod.N_MAX and r["n_steps"] == w["n_steps"]
        p = pops[w["index"]]
        assert p.shape == (r["n_steps"] + 1, r["graph"].N)
        assert np.abs(p.sum(axis=1) - 1).max() < 1e-12
        assert p.min() > -1e-12 and p.max() < 1 + 1e-12
    w = min(hdr["walks"], key=lambda w: w["N"])
    r = reqs[w["index"]]
    A = oracle.walk_superop(r["graph"].dense(), r["omega"], "laplacian", "transition", False, 1.0)
    out, _ = expmv.propagate(A, workloads.basis_state(r["graph"].N, 0), 0.0, r["dt"], r["n_steps"])
    assert np.array_equal(np.real(np.einsum("kaa->ka", out)), pops[w["index"]])


# ------------------------------------------- single-precision products variant

def _vec1_max(ref):
    return max(float(np.abs(ref[k]).sum()) for k in range(ref.shape[0]))


def _fp32_check(A, rho0, t0, dt, n):
    out, info = expmv.propagate_fp32_products(A, rho0, t0, dt, n)
    S = A.dense()
    rmax = int(np.diff(A.row_ptr).max())
    th = oracle.theta.theta_table(oracle.theta.TOL_SINGLE)
    theta = th[expmv.M_MAX_FP32 - 1]     # every step has ||A||_1 |t_step| / s <= theta_20
    s0 = expmv.select_params_norm1(abs(t0) * info["norm1"], th, expmv.M_MAX_FP32)[1] \
        if t0 != 0.0 else 0
    errs = []
    refs = [scipy.linalg.expm((t0 + dt * k) * S) @ rho0.reshape(-1) for k in range(n + 1)]
    vec1 = max(float(np.abs(r).sum()) for r in refs)
    for k in range(n + 1):
        t = t0 + dt * k
        err = np.abs(out[k].reshape(-1) - refs[k]).max()
        steps = k * info["s"] + s0
        bound = expmv.fp32_products_bound(info["norm1"], t, max(steps, 1), theta, rmax, vec1)
        assert err <= bound, (k, err, bound)
        errs.append(err)
        assert abs(np.trace(out[k]).real - np.trace(rho0).real) < 1e-13
    assert info["m"] <= expmv.M_MAX_FP32
    return errs, info


def test_fp32_products_dyadic_cycle_within_bound():
    """Cycle with dyadic entries (float storage exact): only the products'
    rounding and the 2^-24 truncation remain; within the first-order bound and
    clearly above double rounding."""
    wl = _cycle_wl(0.5, r_mode="transition")
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                            wl.dephasing, wl.gamma)
    errs, info = _fp32_check(A, wl.rho0, 0.0, wl.dt, wl.n_steps)
    assert max(errs) > 1e-12


@pytest.mark.parametrize("omega,t0", [(0.0, 0.0), (0.4, 0.0), (0.9, 0.6), (1.0, 0.0)])
def test_fp32_products_random_digraphs_within_bound(omega, t0):
    rng = np.random.Generator(np.random.PCG64(33))
    g = workloads.random_out_degree(12, 3, rng)
    A = oracle.walk_superop(g.dense(), omega)
    rho0 = workloads.random_density(12, rng, rank=2)
    errs, info = _fp32_check(A, rho0, t0, 0.9, 4)
    assert max(errs) > 1e-12


def test_fp32_products_degree_cap_and_parameters():
    """The degree never exceeds 20 and (m, s) is the 1-norm rule at u = 2^-24
    restricted to m <= 20: theta_m s covers ||tA||_1 with the least m s."""
    th = oracle.theta.theta_table(oracle.theta.TOL_SINGLE)
    for x in (0.3, 3.0, 23.09, 150.0):
        m, s = expmv.select_params_norm1(x, th, expmv.M_MAX_FP32)
        assert 1 <= m <= 20 and x / s <= th[m - 1]
        assert all(mm * math.ceil(x / th[mm - 1]) >= m * s for mm in range(1, 21))
