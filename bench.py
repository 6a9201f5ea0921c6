"""Benchmark: L-QSW time-series propagation on one MI355X.

One step = one pass of the whole hot path over the N = 1024 directed
workload (each vertex sends arcs to 10 uniform targets, w ~ U(0,1],
omega = 0.5, rho0 = |0><0|, t = 0..50 in 50 intervals): operators from the
graph, device assembly of the 1,048,576-dimensional superoperator CSR
(4.28e7 entries), its 1-norm series, parameter selection and the Taylor
propagation to all 51 grid points.  The graph, rho0, the output series and
the workspace are resident before the timed region starts.

Prints one JSON line.  `value` is rho(t) grid steps per second of the whole
pass.  `roofline` rates the fused Taylor-term product kernel: algorithmic
bytes of the products it computed (20 nnz + 8 (n+1) + 64 n per product)
over the device time of the timed propagate calls, measured with HIP events
on the stream the kernels run on.  `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_term_kernel_outdeg1024.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2003_02450_amd", "csrc", "kernels.hip")


def measured_traffic():
    """HBM bytes per computing Taylor-term product from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None when the kernel source
    has changed since those counters were taken."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
        h = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()[:16]
        if fields.get("kernels_sha256_16") != h:
            return None
        return float(fields["traffic_bytes_per_product"])
    except (OSError, KeyError, ValueError):
        return None


def term_bytes(n: int, nnz: int) -> float:
    """Algorithmic HBM bytes of one Taylor-term product: values and column
    indices (16 + 4 per entry), row pointers, x gathered once, the new term
    written, the accumulator read and written."""
    return 20.0 * nnz + 8.0 * (n + 1) + 64.0 * n


def cpu_baseline(wl, sample_steps: int) -> dict:
    """The oracle (plain C, OpenMP over rows) on the host cores: build the
    superoperator and propagate `sample_steps` intervals, then scale to the
    full grid."""
    import oracle
    from oracle import expmv

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode,
                            wl.dephasing, wl.gamma)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, sample_steps)
    t_steps = time.perf_counter() - t0
    per_step = t_steps / sample_steps
    full = t_build + wl.n_steps * per_step
    return {"value": wl.n_steps / full, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle superoperator build ({t_build:.2f} s) + {sample_steps} of "
                       f"{wl.n_steps} intervals ({t_steps:.2f} s, {info['products']} products); "
                       f"rate = {wl.n_steps} / (build + {wl.n_steps} x mean interval)")}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched and "
              "served workloads shard by instance and one instance does not span GPUs here.",
              file=sys.stderr)
        return 2

    import torch

    import paper_2003_02450_amd as qsw
    import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = workloads.outdeg1024()
    g = wl.graph
    N, q = g.N, wl.n_steps
    rho0 = torch.from_numpy(wl.rho0).to(dev)
    out = torch.empty((q + 1, N, N), dtype=torch.complex128, device=dev)

    def build():
        return qsw.Superop.from_graph(N, g.row_ptr, g.col_idx, g.w, wl.omega, gamma=wl.gamma,
                                      h_mode=wl.h_mode, r_mode=wl.r_mode,
                                      dephasing=wl.dephasing)

    probe = build()
    ws = torch.empty(probe.workspace_bytes(wl.t0, wl.dt, q) + 256, dtype=torch.uint8, device=dev)
    n, nnz = probe.n, probe.nnz
    probe.close()

    def one_pass():
        op = build()
        op.propagate(rho0, wl.t0, wl.dt, q, out=out, workspace=ws)
        st = op.last_stats()        # waits for the pass on the library stream
        info = op.info()
        op.close()
        return st, info

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        stats.append(one_pass())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    prop_ms = sum(s["ms"] for s, _ in stats)
    products = sum(s["products"] for s, _ in stats)
    launched = sum(s["launched"] for s, _ in stats)
    build_ms = sum(i["build_ms"] for _, i in stats) / len(stats)
    bytes_total = products * term_bytes(n, nnz)
    achieved = bytes_total / (prop_ms * 1e-3) / 1e9
    st0 = stats[0][0]

    result = {
        "metric": "rho(t) steps/s",
        "value": args.steps * q / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "outdeg1024: directed N=1024, 10 uniform out-arcs per vertex, "
                               "w~U(0,1], omega=0.5, H=Laplacian(G^u), one L_k per arc, "
                               "rho0=|0><0|, t=0..50 (51 points)",
                   "n": n, "nnz": nnz, "m": st0["m"], "s": st0["s"],
                   "branch": "single-time per interval" if st0["branch"] == 0 else "series",
                   "build_ms": round(build_ms, 3),
                   "propagate_ms": round(prop_ms / args.steps, 3),
                   "products_per_step": products // args.steps,
                   "term_launches_per_step": launched // args.steps},
        "roofline": {"bound": "hbm", "kernel": "term_kernel (CSR product + Taylor epilogue)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(),
                     "bytes_per_product": term_bytes(n, nnz),
                     "avg_launch_us": 1e3 * prop_ms / max(launched, 1),
                     "avg_product_us": 1e3 * prop_ms / max(products, 1)},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
