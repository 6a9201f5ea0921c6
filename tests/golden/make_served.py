"""Write the oracle populations of sampled walks of the serving workload.

    python tests/golden/make_served.py

Calls only ``oracle/`` (and the seeded generators of ``workloads/``).  The
serving benchmark submits ``workloads.served_requests(count)`` (the same
seeded stream at every rate, at least its first MIN_COUNT walks); this file
stores, for the first SAMPLES walks of that prefix with N <= N_MAX, the
oracle's populations Re rho_k[a][a] at every grid point (FP64, exact 1-norm,
one single-time application per interval), so that the served results can be
checked against the oracle at the FP64 bar (Section 5 compares against an
independent code to at most 1e-10).  The walk: the ER graph with 10 %
one-way edges, H = Laplacian, one L_k per arc, rho0 = |0><0|, t = 0 .. 10.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MIN_COUNT = 24   # walks every serving rate submits at least
SAMPLES = 3
N_MAX = 32
PATH = os.path.join(HERE, "served_pops.npz")


def write() -> str:
    import oracle
    import workloads
    from oracle import expmv
    reqs = workloads.served_requests(MIN_COUNT)
    picked = [i for i, r in enumerate(reqs) if r["graph"].N <= N_MAX][:SAMPLES]
    arrays, meta = {}, []
    for i in picked:
        r = reqs[i]
        g = r["graph"]
        A = oracle.walk_superop(g.dense(), r["omega"], "laplacian", "transition", False, 1.0)
        rho0 = workloads.basis_state(g.N, 0)
        out, info = expmv.propagate(A, rho0, 0.0, r["dt"], r["n_steps"])
        arrays[f"pops_{i}"] = np.real(np.einsum("kaa->ka", out))
        meta.append({"index": i, "N": g.N, "omega": r["omega"], "n_steps": r["n_steps"],
                     "dt": r["dt"], "m": info["m"], "s": info["s"]})
    header = {"requests": "workloads.served_requests(%d)" % MIN_COUNT, "walks": meta,
              "source": "oracle.expmv.propagate (FP64); written by tests/golden/make_served.py"}
    np.savez(PATH, header=np.frombuffer(json.dumps(header).encode(), np.uint8), **arrays)
    print(f"{PATH}: walks {picked}", flush=True)
    return PATH


def load():
    """(header, {request index: populations [n_steps + 1, N]})."""
    z = np.load(PATH, allow_pickle=False)
    header = json.loads(bytes(z["header"]).decode())
    return header, {w["index"]: z[f"pops_{w['index']}"] for w in header["walks"]}


if __name__ == "__main__":
    write()
