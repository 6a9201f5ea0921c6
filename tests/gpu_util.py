"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np

import oracle
import workloads


def build_gpu(wl, **kw):
    import paper_2003_02450_amd as qsw
    g = wl.graph
    return qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, wl.omega, gamma=wl.gamma,
                                  h_mode=wl.h_mode, r_mode=wl.r_mode,
                                  dephasing=wl.dephasing, **kw)


def oracle_superop(wl):
    return oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                               wl.dephasing, wl.gamma)


def random_workload(N, k, omega, seed, h_mode="laplacian", r_mode="transition",
                    dephasing=False, n_steps=5, dt=0.7, t0=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = workloads.random_out_degree(N, k, rng)
    rho0 = workloads.random_density(N, rng, rank=2)
    return workloads.Workload(f"rand{N}", g, omega, h_mode, r_mode, dephasing, rho0,
                              t0, dt, n_steps)


def gpu_run(wl, op=None):
    import torch
    if op is None:
        op = build_gpu(wl)
    out = op.propagate(wl.rho0, wl.t0, wl.dt, wl.n_steps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), op
