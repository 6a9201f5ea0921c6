"""Benchmark: L-QSW time-series propagation on one MI355X.

One step = one pass of the whole hot path over the N = 1024 directed
workload (each vertex sends arcs to 10 uniform targets, w ~ U(0,1],
omega = 0.5, rho0 = |0><0|, t = 0..50 in 50 intervals): operators from the
graph, device assembly of the 1,048,576-dimensional superoperator CSR
(4.28e7 entries), its 1-norm series, parameter selection and the Taylor
propagation to all 51 grid points.  The graph, rho0, the output series and
the workspace are resident before the timed region starts.

Prints one JSON line.  `value` is rho(t) grid steps per second of the whole
pass.  `roofline` rates the fused Taylor-term product kernel over the device
time of the timed propagate calls (HIP events on the stream the kernels run
on).  Its `achieved` counts the layout bytes: every word the kernel reads or
writes per product (12 e + 16 s + 8 (n+1) + 16 n + 64 n with phase-split
values: one real coefficient and a column per stored entry e, the entries
shared by the 64 rows of a block s, row data, the complex diagonal per row, x,
the term and the accumulator), whether the HBM or a cache serves it; blocks
with equal rows read one cached copy, so the HBM traffic (`traffic`, from
rocprofv3 counters) is lower.  `csr_equivalent_gbps` divides the complex CSR's
bytes (20 nnz + 8 (n+1) + 64 n) by the same time.  `csr_engine` times the
plain CSR stream engine on the same pass, whose reads are exactly those CSR
bytes.  `fp32` repeats the pass with single-precision products (complex64
values, vectors and terms, two-float accumulation, FP64 norms, parameters and
trace check) and reports its rate, its kernel's bandwidth and its largest
deviation from the FP64 oracle at every point (the committed full-grid
fixture); `single_values` does the same with only the values in complex64.
`configs` reports the rate of the N = 16 cycle and N = 256 ER workloads.
`batched` runs 64 small walks with 4 density matrices each through one
engine, against the same walks one density matrix at a time, and again with
single-precision values and with single-precision products.  `served` drives
the continuous-batching server with Poisson arrivals at several rates and
reports walks/s and p50/p99 latency.  `cpu_baseline` times the CPU oracle on
a bounded sample of the same workload, with all host threads and with one.
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


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def measured_traffic(key: str = "traffic_bytes_per_product"):
    """HBM bytes per computing Taylor-term product from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (key: the FP64 kernel's, or
    "traffic_bytes_per_product_fp32"), or None when the kernel source has
    changed since those counters were taken."""
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
        return float(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def csr_bytes(n: int, nnz: int) -> float:
    """Algorithmic bytes of one Taylor-term product through the complex CSR:
    column and value per entry, row pointers, x, the term, the accumulator."""
    return 20.0 * nnz + 8.0 * (n + 1) + 64.0 * n


def term_bytes(info: dict, single: bool, series: bool = False, fp32: bool = False) -> float:
    """Algorithmic HBM bytes of one Taylor-term product (the library's own
    qsw_stats_t.bytes per product): column index and value per stored entry
    (4 + 8 phase-split double, 4 + 4 phase-split single, 4 + 16 / 4 + 8
    complex), 16 bytes per block-shared entry (stored once for the 64 rows of
    a block), row data 8 (n+1), the diagonal per row with phase-split values
    (16 or 8 n), x gathered once, the new term written, the accumulator read
    and written (the time-series branch writes the power and accumulates in
    a second pass: 16 n more)."""
    n, split = info["n"], info["split"]
    single = single or fp32
    entry = (8.0 if single else 12.0) if split else (12.0 if single else 20.0)
    diag = (8.0 if single else 16.0) if split else 0.0
    vec = 48.0 if fp32 else (80.0 if series else 64.0)
    return (entry * info["stream_entries"] + 16.0 * info["shared_entries"] + 8.0 * (n + 1) +
            (diag + vec) * n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle, workloads
from oracle import expmv
wl = workloads.outdeg1024()
t0 = time.perf_counter()
A = oracle.walk_superop(wl.graph.dense(), wl.omega, wl.h_mode, wl.r_mode, wl.dephasing, wl.gamma)
t_build = time.perf_counter() - t0
k = int(sys.argv[2])
t0 = time.perf_counter()
_, info = expmv.propagate(A, wl.rho0, wl.t0, wl.dt, k)
print(json.dumps({"build": t_build, "seconds": time.perf_counter() - t0, "intervals": k,
                  "products": info["products"]}))
"""


def cpu_baseline(wl, sample_steps: int, one_thread_steps: int) -> dict:
    """The oracle (plain C, OpenMP over rows) on the host cores: build the
    superoperator and propagate `sample_steps` intervals, then scale to the
    full grid.  Then the same on one thread (a child process with
    OMP_NUM_THREADS=1) for `one_thread_steps` intervals."""
    import subprocess

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
    out = {"value": wl.n_steps / full, "unit": "steps/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": (f"oracle superoperator build ({t_build:.2f} s) + {sample_steps} of "
                      f"{wl.n_steps} intervals ({t_steps:.2f} s, {info['products']} products); "
                      f"rate = {wl.n_steps} / (build + {wl.n_steps} x mean interval)")}
    if one_thread_steps > 0:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, str(one_thread_steps)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            per_step = one["seconds"] / one["intervals"]
            out["single_thread"] = {
                "value": wl.n_steps / (one["build"] + wl.n_steps * per_step), "unit": "steps/s",
                "cores": 1, "kind": "oracle",
                "sample": (f"oracle on one thread: build ({one['build']:.2f} s) + "
                           f"{one['intervals']} of {wl.n_steps} intervals ({one['seconds']:.2f} s, "
                           f"{one['products']} products); rate = {wl.n_steps} / (build + "
                           f"{wl.n_steps} x mean interval)")}
    return out


def timed_passes(args, one_pass, dst):
    for _ in range(args.warmup):
        one_pass(dst)
    import torch
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        stats.append(one_pass(dst))
    torch.cuda.synchronize()
    return stats, time.perf_counter() - t_start


def fixture_error(got) -> float:
    """Largest |rho - rho_oracle| of a [51, 1024, 1024] device series over the
    committed full-grid oracle fixture (all populations, the trace and 10^4
    sampled elements per point)."""
    import importlib.util
    path = os.path.join(ROOT, "tests", "golden", "make_fullgrid.py")
    spec = importlib.util.spec_from_file_location("make_fullgrid", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    _, fx = mod.load("outdeg1024")
    g = got.cpu().numpy()
    K, N = g.shape[0], g.shape[1]
    flat = g.reshape(K, N * N)
    worst = 0.0
    for k in range(K):
        worst = max(worst, float(np.abs(np.diag(g[k]).real - fx["pops"][k]).max()),
                    float(np.abs(flat[k, mod.sample_indices(N * N, k)] - fx["samples"][k]).max()),
                    float(abs(np.trace(g[k]) - fx["trace"][k])))
    return worst


def precision_leg(args, make_pass, out64, torch, q, mode) -> dict:
    """The same pass at another precision ("single": complex64 values,
    complex128 vectors; "fp32": single-precision products), timed the same
    way, its largest element difference from the double pass and from the
    FP64 oracle's full-grid fixture over all 51 points."""
    out = torch.empty_like(out64)
    stats, elapsed = timed_passes(args, make_pass(mode), out)
    prop_ms = sum(s["ms"] for s, _ in stats)
    products = sum(s["products"] for s, _ in stats)
    launched = sum(s["launched"] for s, _ in stats)
    st0, info0 = stats[0]
    # the library's count (one-point series blocks run fused: no separate
    # accumulation pass)
    per = sum(s["bytes"] for s, _ in stats) / max(products, 1)
    achieved = products * per / (prop_ms * 1e-3) / 1e9
    diff = float((out - out64).abs().max().item())
    res = {"value": args.steps * q / elapsed, "unit": "steps/s",
           "ms_per_step": 1e3 * elapsed / args.steps,
           "dtype": "c64 values, f64 vectors" if mode == "single" else
                    "c64 values, vectors and products; hi+lo c64 accumulator; f64 norms",
           "m": st0["m"], "s": st0["s"],
           "branch": "single-time per interval" if st0["branch"] == 0 else "series",
           "values": "phase-split f32" if info0["split"] else "complex64",
           "propagate_ms": round(prop_ms / args.steps, 3),
           "products_per_step": products // args.steps,
           "term_launches_per_step": launched // args.steps,
           "kernel": "term32_kernel<111>" if mode == "fp32" else "term_kernel<111>",
           "achieved": achieved, "unit_bw": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
           "bytes_per_product": per,
           "avg_product_us": 1e3 * prop_ms / max(products, 1),
           "max_abs_diff_vs_double": diff}
    try:
        res["max_abs_err_vs_fp64_oracle"] = fixture_error(out)
    except (OSError, KeyError, ValueError):
        res["max_abs_err_vs_fp64_oracle"] = None
    if mode == "fp32":
        res["trace_dev_max"] = max(s["trace_dev"] for s, _ in stats)
        traffic = measured_traffic("traffic_bytes_per_product_fp32")
        res["traffic"] = traffic
        if traffic is not None:
            res["measured_hbm_frac"] = traffic / (res["avg_product_us"] * 1e3) / HBM_PEAK_GBPS
    return res


def csr_leg(args, make_pass, out64, torch, q, n, nnz) -> dict:
    """The plain CSR stream engine (the paper's format: row_ptr, columns,
    complex128 values, read once per product) on the same pass.  Its reads
    are the complex CSR's bytes, 20 nnz + 8 (n+1) + 64 n per product."""
    out = torch.empty_like(out64)
    os.environ["QSW_ENGINE"] = "3"
    try:
        stats, elapsed = timed_passes(args, make_pass("double"), out)
    finally:
        os.environ.pop("QSW_ENGINE", None)
    prop_ms = sum(s["ms"] for s, _ in stats)
    products = sum(s["products"] for s, _ in stats)
    per = csr_bytes(n, nnz)
    achieved = products * per / (prop_ms * 1e-3) / 1e9
    return {"kernel": "term_kernel<3> (CSR stream engine)", "value": args.steps * q / elapsed,
            "unit": "steps/s", "propagate_ms": round(prop_ms / args.steps, 3),
            "avg_product_us": 1e3 * prop_ms / max(products, 1),
            "achieved": achieved, "unit_bw": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
            "bytes_per_product": per,
            "max_abs_diff_vs_wave_layout": float((out - out64).abs().max().item())}


def configs_leg(torch, qsw, workloads, reps: int) -> dict:
    """The N = 16 cycle (11 points, time-series branch) and the N = 256 ER
    workload (101 points): propagate-only rates (operators built once, inputs
    resident), device time from HIP events, effective GB/s from the library's
    byte count of the products."""
    res = {}
    dev = torch.device("cuda", 0)
    for wl in (workloads.cycle16(), workloads.er256()):
        g = wl.graph
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, wl.omega, gamma=wl.gamma,
                                    h_mode=wl.h_mode, r_mode=wl.r_mode, dephasing=wl.dephasing)
        rho0 = torch.from_numpy(wl.rho0).to(dev)
        out = torch.empty((wl.n_steps + 1, g.N, g.N), dtype=torch.complex128, device=dev)
        ws = torch.empty(op.workspace_bytes(wl.t0, wl.dt, wl.n_steps) + 256, dtype=torch.uint8,
                         device=dev)
        op.propagate(rho0, wl.t0, wl.dt, wl.n_steps, out=out, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = bytes_ = 0.0
        for _ in range(reps):
            op.propagate(rho0, wl.t0, wl.dt, wl.n_steps, out=out, workspace=ws)
            st = op.last_stats()
            ms += st["ms"]
            bytes_ += st["bytes"]
        elapsed = time.perf_counter() - t0
        res[wl.name] = {"steps_per_s": reps * wl.n_steps / elapsed,
                        "device_steps_per_s": reps * wl.n_steps / (ms * 1e-3),
                        "ms_per_propagate": ms / reps, "build_ms": op.info()["build_ms"],
                        "m": st["m"], "s": st["s"],
                        "branch": "single-time per interval" if st["branch"] == 0 else "series",
                        "products": st["products"],
                        "effective_gbps": bytes_ / (ms * 1e-3) / 1e9,
                        "note": "L2/Infinity-Cache resident operator: effective, not HBM"}
        op.close()
    return res


def batch_leg(torch, qsw, workloads, reps: int, compare: bool = True) -> dict:
    """Batched walks: 64 ER graphs (N log-uniform in [32, 512], p = 8/N,
    unit weights, omega ~ U(0,1)), 4 basis states each, t = 0..20 in 100
    steps, all walks in one engine (4 right-hand sides per walk; chunks of
    cycles replayed as HIP graphs, launch shape tuned on the first run).
    Timed against the same walks through qsw_propagate one density matrix at
    a time; every batched result is bitwise that of its single walk.  Then
    the same batch with single-precision values (`single_values`) and with
    single-precision products (`fp32`), each with its largest difference from
    the double batch."""
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
    st = qsw.batch_propagate(items)  # warm-up (tunes the launch shape), sizes the workspace
    ws = torch.empty(st["workspace_bytes"] + 256, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def timed(its):
        t_0 = time.perf_counter()
        dev_ms = byts = 0.0
        for k in range(reps):
            progress(f"batched: batch {k + 1} of {reps}")
            s_ = qsw.batch_propagate(its, workspace=ws)
            dev_ms += s_["ms"]
            byts += s_["bytes"]
        torch.cuda.synchronize()
        return time.perf_counter() - t_0, dev_ms, byts, s_

    elapsed, dev_ms, byts, st = timed(items)
    points = sum(w.n_steps * w.rho0.shape[0] for w in wls)
    achieved = byts / (dev_ms * 1e-3) / 1e9
    # the same walks one density matrix at a time
    progress("batched: the same walks one density matrix at a time")
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
    value = reps * points / elapsed
    single = {"single_walk_path": {"value": points / single_s, "ms": 1e3 * single_s},
              "speedup_vs_single_walks": value / (points / single_s),
              "bitwise_equal_to_single_walks_sampled": equal} if compare else {}
    # single-precision values, same batch
    outs32 = [torch.empty_like(o) for o in outs]
    for op in ops:
        op.set_precision(True)
    items32 = [(op, r, w.t0, w.dt, w.n_steps, o, None)
               for op, r, w, o in zip(ops, r0, wls, outs32)]
    qsw.batch_propagate(items32, workspace=ws)
    e32, ms32, by32, s32 = timed(items32)
    diff = max(float((a - b).abs().max().item()) for a, b in zip(outs32, outs))
    # single-precision products, same batch: against the double batch (itself
    # within 1e-10 of the oracle in the tests) and, sampled, bitwise against
    # the same walks' single-precision single-walk path
    progress("batched: single-precision products")
    outsp = [torch.empty_like(o) for o in outs]
    for op in ops:
        op.set_precision("fp32")
    itemsp = [(op, r, w.t0, w.dt, w.n_steps, o, None)
              for op, r, w, o in zip(ops, r0, wls, outsp)]
    qsw.batch_propagate(itemsp, workspace=ws)
    ep, msp, byp, sp = timed(itemsp)
    diffp = max(float((a - b).abs().max().item()) for a, b in zip(outsp, outs))
    eqp = True
    for i in range(0, len(wls), 16):
        w = wls[i]
        for c in range(r0[i].shape[0]):
            one = ops[i].propagate(r0[i][c], 0.0, w.dt, w.n_steps)
            eqp = eqp and bool(torch.equal(one, outsp[i][:, c]))
    achp = byp / (msp * 1e-3) / 1e9
    for op in ops:
        op.close()
    return {"metric": "instance-points/s", "value": value, "unit": "points/s",
            "workload": "64 ER walks, N~logU[32,512], p=8/N, 4 basis states each, "
                        "t=0..20 in 100 steps", "walks": len(wls), "rhs": 4, "points": points,
            "ms_per_batch": 1e3 * elapsed / reps, "device_ms_per_batch": dev_ms / reps,
            "build_ms": 1e3 * build_s, "cycles": st["cycles"], "products": st["products"],
            "graphs": st["graphs"], "graph_launches": st["graph_launches"],
            "launch_shape": {"rounds_of_resident_workgroups": st["rounds"],
                             "staged": st["staged"]},
            "roofline": {"bound": "hbm", "kernel": "batch_work_kernel<4>",
                         "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBPS,
                         "bytes_basis": "layout bytes of every product (values once for "
                                        "the 4 columns, 64 bytes per element and column) "
                                        "over the engine's device time"},
            "workspace_gb": st["workspace_bytes"] / 1e9, **single,
            "single_values": {"value": reps * points / e32, "unit": "points/s",
                              "dtype": "c64 values, f64 vectors",
                              "ms_per_batch": 1e3 * e32 / reps,
                              "achieved_gbps": by32 / (ms32 * 1e-3) / 1e9,
                              "max_abs_diff_vs_double_batch": diff},
            "fp32": {"value": reps * points / ep, "unit": "points/s",
                     "dtype": "c64 values, vectors and products; hi+lo c64 accumulator; "
                              "f64 norms and trace check",
                     "ms_per_batch": 1e3 * ep / reps, "device_ms_per_batch": msp / reps,
                     "products": sp["products"], "cycles": sp["cycles"],
                     "kernel": "batch_work_kernel<4, true>", "achieved": achp,
                     "unit_bw": "GB/s", "frac": achp / HBM_PEAK_GBPS,
                     "bytes_basis": "layout bytes with single-precision values and 48 bytes "
                                    "per element and column",
                     "max_abs_diff_vs_double_batch": diffp, "trace_dev_max": sp["trace_dev"],
                     "bitwise_equal_to_single_walks_sampled": eqp}}


def single_instance_service(torch, qsw, reqs) -> list:
    """Service time of each request through the plain single-instance FP64
    path on the same GPU: build the operator, qsw_propagate the grid, gather
    the populations, synchronise."""
    dev = torch.device("cuda", 0)
    times = []
    for r in reqs:
        g = r["graph"]
        rho0 = torch.zeros((g.N, g.N), dtype=torch.complex128, device=dev)
        rho0[0, 0] = 1.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, r["omega"])
        out = op.propagate(rho0, 0.0, r["dt"], r["n_steps"])
        op.populations(out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        op.close()
        del out
    return times


def fifo_latencies(arrivals, service) -> np.ndarray:
    """Latencies of one server taking requests in arrival order with the
    given service times (the single-instance path has no overlap)."""
    free = 0.0
    lat = []
    for a, sv in zip(arrivals, service):
        start = max(a, free)
        free = start + sv
        lat.append(free - a)
    return np.array(lat)


def served_reference() -> dict:
    """{request index: the oracle's populations} of the sampled walks of the
    serving stream, from the committed fixture tests/golden/served_pops.npz
    (written from the oracle by tests/golden/make_served.py), or {} if it is
    absent."""
    path = os.path.join(ROOT, "tests", "golden", "served_pops.npz")
    try:
        z = np.load(path, allow_pickle=False)
    except OSError:
        return {}
    header = json.loads(bytes(z["header"]).decode())
    return {w["index"]: z[f"pops_{w['index']}"] for w in header["walks"]}


def served_leg(torch, qsw, workloads, qps_list, seconds: float, min_count: int,
               warmup_seconds: float = 3.0) -> dict:
    """Continuous batching: walks (N log-uniform in [16, 2048], ER mean degree
    6 with 10 % one-way edges, omega ~ U(0,1), 10..200 steps over t in
    [0, 10], rho0 = |0><0|, populations out) arrive as a Poisson process at
    each rate in qps_list for about `seconds` (at least `min_count` walks).
    Latency runs from a walk's arrival time to the moment its populations are
    ready (operator build, queueing and propagation included).  `backlog` is
    the number of walks not yet finished when the last one arrived.  The
    same request stream through the single-instance FP64 path (qsw_propagate
    per walk, measured service times, one walk at a time in arrival order)
    gives the baseline.  Each rate starts with `warmup_seconds` of other walks
    of the same mix through the same server (unmeasured), so that the
    measured stream meets a running server rather than its first
    allocations."""
    GB = 1 << 30
    count_max = max(min_count, int(max(qps_list) * seconds))
    reqs = workloads.served_requests(count_max)
    ref_pops = served_reference()  # sampled walks of the stream: the oracle's populations
    # baseline: measured service times of the single-instance path
    n_base = min(count_max, 48)
    progress(f"served: single-instance baseline on {n_base} walks")
    service = single_instance_service(torch, qsw, reqs[:n_base])
    base_rate = n_base / sum(service)
    def drive(srv, rq, arrivals, keep=()):
        """Submit rq at their arrival times, step until all are done:
        (latencies in finishing order, backlog at the last arrival, wall,
        {index: populations} of the walks whose index is in keep)."""
        count = len(arrivals)
        t_arr = {}
        idx = {}
        kept = {}
        lat = []
        i = 0
        backlog = None
        t0 = time.perf_counter()
        while len(lat) < count:
            now = time.perf_counter() - t0
            while i < count and arrivals[i] <= now:
                r = rq[i]
                rid = srv.submit(r["graph"], r["omega"], 0.0, r["dt"], r["n_steps"])
                t_arr[rid] = arrivals[i]
                idx[rid] = i
                i += 1
                if i == count:
                    backlog = count - len(lat)
            running, pending = srv.step(8)
            t_ready = time.perf_counter() - t0
            for rid, _, pops, _ in srv.poll():
                lat.append(t_ready - t_arr.pop(rid))
                if idx[rid] in keep:
                    kept[idx[rid]] = pops.cpu().numpy()
            if running == 0 and pending == 0 and i < count and len(lat) < count:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
        return lat, backlog, time.perf_counter() - t0, kept

    points = []
    for qps in qps_list:
        count = max(min_count, int(qps * seconds))
        srv = qsw.Server(96 * GB, 48 * GB, 4096)
        # warm-up: other walks of the same mix at the same rate (their graphs
        # differ from the measured ones, so no measured operator is cached)
        n_warm = max(8, int(qps * warmup_seconds))
        progress(f"served: {n_warm} warm-up walks at {qps} QPS")
        drive(srv, workloads.served_requests(n_warm, seed=workloads.BASE_SEED + 32),
              workloads.poisson_arrivals(n_warm, qps, seed=workloads.BASE_SEED + 33))
        st0 = srv.stats()
        progress(f"served: {count} walks at {qps} QPS")
        arrivals = workloads.poisson_arrivals(count, qps)
        lat, backlog, wall, kept = drive(srv, reqs, arrivals, set(ref_pops))
        err = max((float(np.abs(kept[i] - p).max()) for i, p in ref_pops.items() if i in kept),
                  default=None)
        st = srv.stats()
        srv.close()
        lat_ms = 1e3 * np.array(lat)
        half = len(lat_ms) // 2
        svc = np.array([service[k % n_base] for k in range(count)])
        base = 1e3 * fifo_latencies(arrivals, svc)
        points.append({"qps": qps, "walks": count, "walks_per_s": count / wall,
                       "p50_ms": float(np.percentile(lat_ms, 50)),
                       "p99_ms": float(np.percentile(lat_ms, 99)),
                       "mean_ms": float(lat_ms.mean()),
                       "p50_first_half_ms": float(np.percentile(lat_ms[:half], 50)),
                       "p50_second_half_ms": float(np.percentile(lat_ms[half:], 50)),
                       "backlog_at_last_arrival": backlog,
                       "max_abs_err_vs_oracle_sampled": err,
                       "cycles": st["cycles"] - st0["cycles"],
                       "build_ms": st["build_ms"] - st0["build_ms"], "warmup_walks": n_warm,
                       "single_instance": {
                           "walks_per_s": count / max(arrivals[-1] + base[-1] / 1e3, 1e-9),
                           "p50_ms": float(np.percentile(base, 50)),
                           "p99_ms": float(np.percentile(base, 99))}})
    return {"metric": "walks/s", "workload": "N~logU[16,2048] ER deg 6 (10% one-way), "
            "omega~U(0,1), 10..200 steps over t=0..10, rho0=|0><0|, populations out",
            "seconds_per_rate": seconds, "warmup_seconds_per_rate": warmup_seconds,
            "points": points,
            "accuracy": "max_abs_err_vs_oracle_sampled: the populations of the stream's "
                        "sampled walks (N <= 32) against the oracle's, committed in "
                        "tests/golden/served_pops.npz; every served walk is bitwise the "
                        "single-instance FP64 path (tested)",
            "single_instance_path": {
                "walks_per_s": base_rate, "sampled_walks": n_base,
                "note": "qsw_propagate per walk (build + propagate + populations, FP64), "
                        "one at a time; latencies from its measured service times in "
                        "arrival order"}}


PAPER_XC40_S = {"line": 1973.0, "lattice": 2010.0, "er": 2842.0, "complete": 27821.0}


def paper_leg(torch, qsw, workloads, kinds) -> dict:
    """The paper's four Section 5 benchmark shapes (about 1.28e8 superoperator
    entries each; omega = 0.5, which the paper does not state; rho0 = I/N):
    build, then one step to t = 100 (FP64, launch pacing 2).  The paper's
    single-process Cray XC40 wall times to t = 100 are quoted as context."""
    dev = torch.device("cuda", 0)
    res = {}
    for kind in kinds:
        progress(f"paper-shaped: {kind}")
        wl = workloads.paper_shaped(kind)
        g = wl.graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = qsw.Superop.from_graph(g.N, g.row_ptr, g.col_idx, g.w, wl.omega)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        op.set_pacing(2)
        rho0 = torch.from_numpy(wl.rho0).to(dev)
        t0 = time.perf_counter()
        out = op.propagate(rho0, 0.0, wl.dt, wl.n_steps)
        st = op.last_stats()
        prop_s = time.perf_counter() - t0
        info = op.info()
        tr = float(torch.diagonal(out[-1]).real.sum().item())
        per_us = 1e3 * st["ms"] / max(st["products"], 1)
        res[kind] = {"N": g.N, "n": info["n"], "nnz": info["nnz"], "arcs": g.n_arcs,
                     "norm1": info["norm1"], "m": st["m"], "s": st["s"],
                     "products": st["products"], "build_s": build_s,
                     "propagate_s": prop_s, "total_s": build_s + prop_s,
                     "avg_product_us": per_us,
                     "layout_gbps": st["bytes"] / max(st["products"], 1) / (per_us * 1e3),
                     "csr_equivalent_gbps": csr_bytes(info["n"], info["nnz"]) / (per_us * 1e3),
                     "trace_at_t100": tr,
                     "paper_xc40_one_process_s": PAPER_XC40_S[kind],
                     "note": "paper: Cray XC40, 2x Xeon E5-2690 v3, one MPI process, "
                             "omega not stated (context only)"}
        del out
        op.close()
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--cpu-one-thread-steps", type=int, default=1,
                    help="oracle intervals timed on one thread (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pace", type=int, default=2,
                    help="launch pacing lookahead of the single-walk passes (0: off)")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the complex64-values leg")
    ap.add_argument("--no-fp32", action="store_true", help="skip the single-precision leg")
    ap.add_argument("--no-csr", action="store_true", help="skip the CSR stream-engine leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the N=16 / N=256 legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-walks leg")
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batched-walks leg (for profiling) and print it")
    ap.add_argument("--no-batch-compare", action="store_true",
                    help="skip timing the batched walks one density matrix at a time")
    ap.add_argument("--no-serve", action="store_true", help="skip the continuous-batching leg")
    ap.add_argument("--serve-qps", default="2,4,8,12", help="arrival rates of the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="arrival time span of each serving rate")
    ap.add_argument("--serve-count", type=int, default=24, help="least walks per serving rate")
    ap.add_argument("--serve-warmup", type=float, default=3.0,
                    help="seconds of unmeasured warm-up walks before each serving rate")
    ap.add_argument("--paper", default="",
                    help="comma list of the paper's benchmark shapes to run to t=100 "
                         "(line,lattice,er,complete); none by default")
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

    def make_pass(mode):
        def one_pass(dst):
            op = build()
            op.set_pacing(args.pace)
            if mode != "double":
                op.set_precision(mode)
            op.propagate(rho0, wl.t0, wl.dt, q, out=dst, workspace=ws)
            st = op.last_stats()        # waits for the pass on the library stream
            info = op.info()
            op.close()
            return st, info
        return one_pass

    progress("headline: FP64 passes")
    stats, elapsed = timed_passes(args, make_pass("double"), out)

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
    traffic = measured_traffic()
    per_us = 1e3 * prop_ms / max(products, 1)

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
                   "distinct_entries": info0["distinct_entries"],
                   "launch_pacing": args.pace,
                   "build_ms": round(build_ms, 3),
                   "propagate_ms": round(prop_ms / args.steps, 3),
                   "products_per_step": products // args.steps,
                   "term_launches_per_step": launched // args.steps,
                   "terms_per_point": products / (args.steps * q),
                   "steps_per_s_excluding_build": q / (prop_ms / args.steps / 1e3)},
        "roofline": {"bound": "hbm",
                     "kernel": (f"term_kernel<{info0['engine']}> (sparse product + Taylor "
                                "epilogue, wave layout, rho-row staged in LDS, "
                                f"{'phase-split' if split else 'complex'} values)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "bytes_basis": ("layout bytes: every word each product reads or writes, "
                                     "served by HBM or by a cache (equal blocks share one "
                                     "copy); the complex CSR's bytes give csr_equivalent_gbps"),
                     "bytes_per_product": per_product,
                     "csr_bytes_per_product": csr_bytes(n, nnz),
                     "csr_equivalent_gbps": csr_bytes(n, nnz) / (per_us * 1e3),
                     "measured_hbm_gbps": None if traffic is None else traffic / (per_us * 1e3),
                     "measured_hbm_frac": (None if traffic is None else
                                           traffic / (per_us * 1e3) / HBM_PEAK_GBPS),
                     "avg_launch_us": 1e3 * prop_ms / max(launched, 1),
                     "avg_product_us": per_us},
    }
    if not args.no_csr:
        progress("CSR stream engine")
        result["csr_engine"] = csr_leg(args, make_pass, out, torch, q, n, nnz)
    if not args.no_fp32:
        progress("single-precision products")
        result["fp32"] = precision_leg(args, make_pass, out, torch, q, "fp32")
    if not args.no_single:
        progress("single-precision values")
        result["single_values"] = precision_leg(args, make_pass, out, torch, q, "single")
    if not args.no_configs:
        progress("N=16 and N=256 workloads")
        result["configs"] = configs_leg(torch, qsw, workloads, max(3, args.steps))
    if not args.no_batch:
        progress("batched walks")
        result["batched"] = batch_leg(torch, qsw, workloads, min(args.steps, 3),
                                      not args.no_batch_compare)
    if not args.no_serve:
        progress("continuous batching")
        result["served"] = served_leg(torch, qsw, workloads,
                                      [float(x) for x in args.serve_qps.split(",")],
                                      args.serve_seconds, args.serve_count,
                                      args.serve_warmup)
    if args.paper:
        result["paper_shaped"] = paper_leg(torch, qsw, workloads, args.paper.split(","))
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps,
                                              args.cpu_one_thread_steps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
