"""Write the full-grid oracle fixture of the N = 1024 benchmark workload.

    python tests/golden/make_fullgrid.py [outdeg1024]

Calls only ``oracle/`` (and the seeded generators of ``workloads/``).  For
every grid point k of the workload it stores, from the oracle's FP64
propagation (one single-time application per interval, exact 1-norm):

* ``pops[k]``    - every population Re rho_k[a][a];
* ``samples[k]`` - rho_k at SAMPLES flat row-major indices given by
  ``sample_indices(n, k)`` below (a fixed odd-stride walk over the n = N^2
  elements, offset per point, so different points cover different elements);
* ``trace[k]``   - Tr rho_k;
* ``vec1[k]``    - ||vec rho_k||_1 (sum of the element moduli), for error bounds.

The files hold plain arrays (numpy .npz, no pickled objects) and a JSON
header.  Section 5 of the paper compares against an independent code at every
reported grid point, to at most 1e-10; the GPU tests do the same against
these fixtures.  (The N = 256 workload is small enough for the GPU test to
run the oracle's full grid itself; ``write("er256")`` still works.)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SAMPLES = 10_000
STRIDE = 0x9E3779B1        # odd: i -> (STRIDE i + offset) mod n is a bijection for n = 2^k


def sample_indices(n: int, k: int) -> np.ndarray:
    """SAMPLES distinct flat indices in [0, n) for grid point k (n a power of two)."""
    assert n & (n - 1) == 0 and n >= SAMPLES
    i = np.arange(SAMPLES, dtype=np.int64)
    off = (k * 0x5851F42D) % n
    return (STRIDE * i + off) % n


def fixture_path(name: str) -> str:
    return os.path.join(HERE, f"fullgrid_{name}.npz")


def write(name: str) -> str:
    import oracle
    import workloads
    from oracle import expmv
    wl = getattr(workloads, name)()
    t = time.time()
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                            wl.dephasing, wl.gamma)
    out, info = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, wl.n_steps)
    secs = time.time() - t
    N = wl.graph.N
    n = N * N
    K = wl.n_steps + 1
    flat = out.reshape(K, n)
    pops = np.stack([np.diag(out[k]).real for k in range(K)])
    samples = np.stack([flat[k, sample_indices(n, k)] for k in range(K)])
    trace = np.array([np.trace(out[k]) for k in range(K)])
    vec1 = np.abs(flat).sum(axis=1)
    header = {
        "workload": name, "N": N, "n": n, "points": K, "t0": wl.t0, "dt": wl.dt,
        "omega": wl.omega, "samples_per_point": SAMPLES,
        "sample_indices": "(0x9E3779B1 i + (k 0x5851F42D mod n)) mod n, i < samples",
        "oracle": {"m": info["m"], "s": info["s"], "norm1": info["norm1"],
                   "products": info["products"], "seconds": round(secs, 1)},
        "source": "oracle.expmv.propagate (FP64, exact 1-norm, one single-time "
                  "application per interval); written by tests/golden/make_fullgrid.py",
    }
    path = fixture_path(name)
    np.savez(path, pops=pops, samples=samples, trace=trace, vec1=vec1,
             header=np.frombuffer(json.dumps(header).encode(), np.uint8))
    print(f"{path}: {K} points, {secs:.1f} s", flush=True)
    return path


def load(name: str):
    """(header, arrays): arrays holds pops, samples, trace and vec1."""
    z = np.load(fixture_path(name), allow_pickle=False)
    header = json.loads(bytes(z["header"]).decode())
    return header, {k: z[k] for k in ("pops", "samples", "trace", "vec1")}


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["outdeg1024"]):
        write(nm)
