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
bytes of the products it computed (per product 12 e + 16 s + 8 (n+1) +
16 n + 64 n with phase-split values: one real coefficient and a column per
stored entry e, the entries shared by the 64 rows of a block s, row data,
the complex diagonal per row, x, the term and the accumulator; 20 nnz +
8 (n+1) + 64 n with complex values) over the device time of the timed
propagate calls, measured with HIP events on the stream the kernels run
on.  `single_values` repeats the pass with
the superoperator values stored as complex64 and the 2^-24 tolerance
(vectors and sums stay double) and reports its rate, its product kernel's
bandwidth and its largest deviation from the double pass.  `batched` runs 64
small walks with 4 density matrices each through one engine, against the same
walks one density matrix at a time.  `served` drives the continuous-batching
server with Poisson arrivals at several rates and reports walks/s and
p50/p99 latency.  `cpu_baseline`
times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

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


def term_bytes(info: dict, single: bool, series: bool = False) -> float:
    """Algorithmic HBM bytes of one Taylor-term product (the library's own
    qsw_stats_t.bytes per product): column index and value per stored entry
    (4 + 8 phase-split double, 4 + 4 phase-split single, 4 + 16 / 4 + 8
    complex), 16 bytes per block-shared entry (stored once for the 64 rows of
    a block), row data 8 (n+1), the diagonal per row with phase-split values
    (16 or 8 n), x gathered once, the new term written, the accumulator read
    and written (the time-series branch writes the power and accumulates in
    a second pass: 16 n more)."""
    n, split = info["n"], info["split"]
    entry = (8.0 if single else 12.0) if split else (12.0 if single else 20.0)
    diag = (8.0 if single else 16.0) if split else 0.0
    return (entry * info["stream_entries"] + 16.0 * info["shared_entries"] + 8.0 * (n + 1) +
            (diag + (80.0 if series else 64.0)) * n)


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


def single_leg(args, one_pass, out64, torch, n, nnz, q, wl) -> dict:
    """The same pass with complex64 superoperator values and the 2^-24
    tolerance (vectors and sums in double), timed the same way, and its
    largest element difference from the double pass over all 51 points."""
    out32 = torch.empty_like(out64)
    for _ in range(args.warmup):
        one_pass(True, out32)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        stats.append(one_pass(True, out32))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prop_ms = sum(s["ms"] for s, _ in stats)
    products = sum(s["products"] for s, _ in stats)
    launched = sum(s["launched"] for s, _ in stats)
    st0, info0 = stats[0]
    # the library's count (one-point series blocks run fused: no separate
    # accumulation pass)
    per = sum(s["bytes"] for s, _ in stats) / max(products, 1)
    achieved = products * per / (prop_ms * 1e-3) / 1e9
    diff = float((out32 - out64).abs().max().item())
    bound = 2.0 * 2.0 ** -24 * (q * wl.dt) * info0["norm1"] * float(abs(wl.rho0).sum())
    return {"value": args.steps * q / elapsed, "unit": "steps/s",
            "ms_per_step": 1e3 * elapsed / args.steps, "dtype": "c64 values, f64 vectors",
            "m": st0["m"], "s": st0["s"],
            "branch": "single-time per interval" if st0["branch"] == 0 else "series",
            "values": "phase-split f32" if info0["split"] else "complex64",
            "propagate_ms": round(prop_ms / args.steps, 3),
            "products_per_step": products // args.steps,
            "term_launches_per_step": launched // args.steps,
            "achieved": achieved, "frac": achieved / HBM_PEAK_GBPS,
            "bytes_per_product": per,
            "avg_product_us": 1e3 * prop_ms / max(products, 1),
            "max_abs_diff_vs_double": diff, "first_order_bound_t50": bound}


def batch_leg(torch, qsw, workloads, reps: int, compare: bool = True) -> dict:
    """Batched walks: 64 ER graphs (N log-uniform in [32, 512], p = 8/N,
    unit weights, omega ~ U(0,1)), 4 basis states each, t = 0..20 in 100
    steps, all walks in one engine (4 right-hand sides per walk).  Timed
    against the same walks through qsw_propagate one density matrix at a
    time; every batched result is bitwise that of its single walk."""
    dev = torch.device("cuda", 0)
    wls = workloads.batch64()
    t0 = time.perf_counter()
    ops = [qsw.Superop.from_graph(w.graph.N, w.graph.row_ptr, w.graph.col_idx, w.graph.w,
                                  w.omega) for w in wls]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    r0 = [torch.from_numpy(w.rho0).to(dev) for w in wls]
    outs = [torch.empty((w.n_steps + 1,) + w.rho0.shape, dtype=torch.complex128, device=dev)
            for w in wls]
    items = [(op, r, w.t0, w.dt, w.n_steps, o, None) for op, r, w, o in zip(ops, r0, wls, outs)]
    st = qsw.batch_propagate(items)  # warm-up, sizes the workspace
    ws = torch.empty(st["workspace_bytes"] + 256, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = qsw.batch_propagate(items, workspace=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    points = sum(w.n_steps * w.rho0.shape[0] for w in wls)
    # the same walks one density matrix at a time
    t0 = time.perf_counter()
    equal = True
    for i, (op, w, r) in enumerate(zip(ops, wls, r0) if compare else []):
        one = torch.empty((w.n_steps + 1, w.graph.N, w.graph.N), dtype=torch.complex128,
                          device=dev)
        wsp = torch.empty(op.workspace_bytes(0.0, w.dt, w.n_steps) + 256, dtype=torch.uint8,
                          device=dev)
        for c in range(r.shape[0]):
            op.propagate(r[c], 0.0, w.dt, w.n_steps, out=one, workspace=wsp)
            if i % 16 == 0:
                equal = equal and bool(torch.equal(one, outs[i][:, c]))
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t0
    for op in ops:
        op.close()
    value = reps * points / elapsed
    single = {"single_walk_path": {"value": points / single_s, "ms": 1e3 * single_s},
              "speedup_vs_single_walks": value / (points / single_s),
              "bitwise_equal_to_single_walks_sampled": equal} if compare else {}
    return {"metric": "instance-points/s", "value": value, "unit": "points/s",
            "workload": "64 ER walks, N~logU[32,512], p=8/N, 4 basis states each, "
                        "t=0..20 in 100 steps", "walks": len(wls), "rhs": 4, "points": points,
            "ms_per_batch": 1e3 * elapsed / reps, "build_ms": 1e3 * build_s,
            "cycles": st["cycles"], "products": st["products"],
            "workspace_gb": st["workspace_bytes"] / 1e9, **single}


def served_leg(torch, qsw, workloads, qps_list, count: int) -> dict:
    """Continuous batching: `count` walks (N log-uniform in [16, 2048], ER
    mean degree 6 with 10 % one-way edges, omega ~ U(0,1), 10..200 steps over
    t in [0, 10], rho0 = |0><0|, populations out) arrive as a Poisson process
    at each rate in qps_list.  Latency runs from a walk's arrival time to the
    moment its populations are ready (operator build, queueing and
    propagation included)."""
    GB = 1 << 30
    reqs = workloads.served_requests(count)
    points = []
    for qps in qps_list:
        arrivals = workloads.poisson_arrivals(count, qps)
        srv = qsw.Server(96 * GB, 48 * GB, 4096)
        t_arr = {}
        lat = []
        i = 0
        t0 = time.perf_counter()
        while len(lat) < count:
            now = time.perf_counter() - t0
            while i < count and arrivals[i] <= now:
                r = reqs[i]
                rid = srv.submit(r["graph"], r["omega"], 0.0, r["dt"], r["n_steps"])
                t_arr[rid] = arrivals[i]
                i += 1
            running, pending = srv.step(8)
            t_ready = time.perf_counter() - t0
            for rid, _, _, _ in srv.poll():
                lat.append(t_ready - t_arr.pop(rid))
            if running == 0 and pending == 0 and i < count and len(lat) < count:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat_ms = 1e3 * np.array(lat)
        points.append({"qps": qps, "walks_per_s": count / wall,
                       "p50_ms": float(np.percentile(lat_ms, 50)),
                       "p99_ms": float(np.percentile(lat_ms, 99)),
                       "mean_ms": float(lat_ms.mean()), "cycles": st["cycles"],
                       "build_ms": st["build_ms"]})
    return {"metric": "walks/s", "workload": "N~logU[16,2048] ER deg 6 (10% one-way), "
            "omega~U(0,1), 10..200 steps over t=0..10, rho0=|0><0|, populations out",
            "walks_per_point": count, "points": points}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pace", type=int, default=2,
                    help="launch pacing lookahead of the single-walk passes (0: off)")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the complex64-values leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-walks leg")
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batched-walks leg (for profiling) and print it")
    ap.add_argument("--no-batch-compare", action="store_true",
                    help="skip timing the batched walks one density matrix at a time")
    ap.add_argument("--no-serve", action="store_true", help="skip the continuous-batching leg")
    ap.add_argument("--serve-qps", default="2,4,8", help="arrival rates of the serving leg")
    ap.add_argument("--serve-count", type=int, default=32, help="walks per serving rate")
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
    if args.only_batch:
        print(json.dumps(batch_leg(torch, qsw, workloads, args.steps, not args.no_batch_compare)),
              flush=True)
        return 0
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

    def one_pass(single=False, dst=out):
        op = build()
        op.set_pacing(args.pace)
        if single:
            op.set_precision(True)
        op.propagate(rho0, wl.t0, wl.dt, q, out=dst, workspace=ws)
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
    info0 = stats[0][1]
    split = info0["split"]
    per_product = term_bytes(info0, False)
    bytes_total = products * per_product
    assert abs(bytes_total - sum(s["bytes"] for s, _ in stats)) <= 1e-6 * bytes_total
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
                   "values": "phase-split" if split else "complex",
                   "stream_entries": info0["stream_entries"],
                   "shared_entries": info0["shared_entries"],
                   "launch_pacing": args.pace,
                   "build_ms": round(build_ms, 3),
                   "propagate_ms": round(prop_ms / args.steps, 3),
                   "products_per_step": products // args.steps,
                   "term_launches_per_step": launched // args.steps},
        "roofline": {"bound": "hbm",
                     "kernel": (f"term_kernel<{110 if split else 100}> (CSR product + Taylor "
                                "epilogue, rho-row staged in LDS, "
                                f"{'phase-split' if split else 'complex'} values)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(),
                     "bytes_per_product": per_product,
                     "avg_launch_us": 1e3 * prop_ms / max(launched, 1),
                     "avg_product_us": 1e3 * prop_ms / max(products, 1)},
    }
    if not args.no_single:
        result["single_values"] = single_leg(args, one_pass, out, torch, n, nnz, q, wl)
    if not args.no_batch:
        result["batched"] = batch_leg(torch, qsw, workloads, args.steps,
                                      not args.no_batch_compare)
    if not args.no_serve:
        result["served"] = served_leg(torch, qsw, workloads,
                                      [float(x) for x in args.serve_qps.split(",")],
                                      args.serve_count)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
