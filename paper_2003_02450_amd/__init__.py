"""L-QSW propagation on one MI355X: thin Python binding of libqsw.

Every step of the walk runs in the HIP kernels of ``libqsw.so`` (built from
``csrc/`` by ``python -m paper_2003_02450_amd.build``); this module only
marshals arguments.  PyTorch provides the device memory (complex128 tensors)
and the stream.

    op = Superop.from_graph(N, row_ptr, col_idx, w, omega=0.5)
    rho = op.propagate(rho0, t0=0.0, dt=1.0, n_steps=50)   # [51, N, N]

mirrors the paper's ``LQSW(omega, H, M_L)`` + ``series`` (Section 4);
``step(rho0, t)`` is ``step``; ``populations(rho)`` is
``gather_populations``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import QswError  # noqa: F401

__all__ = ["Superop", "Engine", "Server", "batch_propagate", "QswError", "theta",
           "select_params", "library_path"]

library_path = _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _prec_code(mode) -> int:
    if mode is True or mode == "single":
        return _lib.QSW_PREC_SINGLE
    if mode is False or mode is None or mode == "double":
        return _lib.QSW_PREC_DOUBLE
    if mode == "fp32":
        return _lib.QSW_PREC_FP32
    raise ValueError(f"precision {mode!r}")


def theta(m: int, single: bool = False) -> float:
    """theta_m of the Taylor backward-error bound (host-only library call)."""
    return float(_lib.load().qsw_theta(int(m), _lib.QSW_PREC_SINGLE if single else
                                       _lib.QSW_PREC_DOUBLE))


def select_params(norm1: float, d=None, t: float = 1.0, n0: int = 1, single: bool = False,
                  known_norms: bool = False):
    """(m, s) for exp(t L) from ||L||_1 and d[p] = ||L^p||_1^(1/p), p = 2..9
    (host-only library call; ``d`` indexable by p, or None).  ``single``: a
    precision as for Superop.set_precision (True / "single" / "fp32").
    ``known_norms``: the alpha_p rule whenever d is given (as propagate
    chooses with a handle's norms), without the switch for small ||tL||_1."""
    L = _lib.load()
    darr = None
    if d is not None:
        darr = np.zeros(10, np.float64)
        for p in range(2, 10):
            darr[p] = float(d[p])
    m, s = ctypes.c_int32(), ctypes.c_int32()
    st = L.qsw_select_params(float(norm1), None if darr is None else _ptr(darr), float(t),
                             int(n0), _prec_code(single) |
                             (_lib.QSW_PARAMS_KNOWN_NORMS if known_norms else 0),
                             ctypes.byref(m), ctypes.byref(s))
    _lib.check(st, "qsw_select_params")
    return m.value, s.value


class Superop:
    """Device-resident L-QSW superoperator (CSR) plus its 1-norm series."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device
        info = _lib.Info()
        _lib.check(_lib.load().qsw_superop_info(self._h, ctypes.byref(info)), "qsw_superop_info")
        self.N = info.N
        self.n = info.n
        self.nnz = info.nnz
        self.omega = info.omega
        self._info = info

    # ------------------------------------------------------------ builders
    @classmethod
    def from_graph(cls, N, row_ptr, col_idx, w, omega, gamma=1.0, h_mode="laplacian",
                   r_mode="transition", dephasing=False, device=None):
        """Graph CSR (row = target, column = source, w > 0) -> superoperator."""
        torch = _torch()
        L = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        flags = 0
        if h_mode == "adjacency":
            flags |= _lib.QSW_H_ADJACENCY
        elif h_mode != "laplacian":
            raise ValueError(h_mode)
        if r_mode == "colnorm":
            flags |= _lib.QSW_R_COLNORM
        elif r_mode != "transition":
            raise ValueError(r_mode)
        if dephasing:
            flags |= _lib.QSW_DEPHASING
        rp = np.ascontiguousarray(row_ptr, np.int64)
        ci = np.ascontiguousarray(col_idx, np.int32)
        ww = np.ascontiguousarray(w, np.float64)
        if rp.shape != (int(N) + 1,):
            raise ValueError("row_ptr must have N+1 entries")
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = L.qsw_superop_build(int(N), _ptr(rp), _ptr(ci), _ptr(ww), float(omega),
                                     float(gamma), flags, _stream(dev), ctypes.byref(h))
        _lib.check(st, "qsw_superop_build")
        return cls(h, dev)

    @classmethod
    def from_channels(cls, graph, omega, sources=(), sinks=(), gamma=1.0, h_mode="laplacian",
                      r_mode="transition", dephasing=False, device=None):
        """Walk on the augmented digraph (Section 2.5.1): sources = [(vertex,
        Gamma)], sinks = [(vertex, Theta)]; source k is vertex N + k, sink k
        vertex N + len(sources) + k; the channels act outside omega."""
        torch = _torch()
        L = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        rp = np.ascontiguousarray(graph.row_ptr, np.int64)
        ci = np.ascontiguousarray(graph.col_idx, np.int32)
        ww = np.ascontiguousarray(graph.w, np.float64)
        sv = np.ascontiguousarray([v for v, _ in sources], np.int32)
        sr = np.ascontiguousarray([r for _, r in sources], np.float64)
        kv = np.ascontiguousarray([v for v, _ in sinks], np.int32)
        kr = np.ascontiguousarray([r for _, r in sinks], np.float64)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = L.qsw_superop_build_channels(
                int(graph.N), _ptr(rp), _ptr(ci), _ptr(ww), float(omega), float(gamma),
                _flags(h_mode, r_mode, dephasing), len(sources), _ptr(sv), _ptr(sr), len(sinks),
                _ptr(kv), _ptr(kr), _stream(dev), ctypes.byref(h))
        _lib.check(st, "qsw_superop_build_channels")
        return cls(h, dev)

    @classmethod
    def from_general(cls, H, Ls, omega, H_rot=None, device=None):
        """Explicit Lindblad operators (Section 2.5.2): H and H_rot Hermitian,
        Ls a list of complex matrices (scipy sparse or dense); the G-QSW of
        eq. L_global is Ls = [G]."""
        torch = _torch()
        import scipy.sparse as sp
        L = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)

        def csr(M):
            C = sp.csr_matrix(M, dtype=np.complex128)
            C.sort_indices()
            return (np.ascontiguousarray(C.indptr, np.int64), np.ascontiguousarray(C.indices, np.int32),
                    np.ascontiguousarray(C.data, np.complex128).view(np.float64))
        hp, hc, hv = csr(H)
        N = hp.size - 1
        parts = [csr(M) for M in Ls]
        keep = parts
        lp = (ctypes.c_void_p * max(len(parts), 1))(*[_ptr(p[0]).value for p in parts])
        lc = (ctypes.c_void_p * max(len(parts), 1))(*[_ptr(p[1]).value for p in parts])
        lv = (ctypes.c_void_p * max(len(parts), 1))(*[_ptr(p[2]).value for p in parts])
        rp = rc = rv = None
        if H_rot is not None:
            rp, rc, rv = csr(H_rot)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = L.qsw_superop_build_general(
                N, _ptr(hp), _ptr(hc), _ptr(hv), len(parts), lp, lc, lv,
                _ptr(rp) if rp is not None else None, _ptr(rc) if rc is not None else None,
                _ptr(rv) if rv is not None else None, float(omega), _stream(dev), ctypes.byref(h))
        del keep
        _lib.check(st, "qsw_superop_build_general")
        return cls(h, dev)

    @classmethod
    def from_demoralised(cls, graph, omega, gamma=1.0, device=None):
        """The non-moralising G-QSW of a digraph (Section 2.5.2) on its
        expanded vertex set; `copies` (d_v per vertex) maps states and
        populations (demoralised_state / demoralised_populations)."""
        torch = _torch()
        L = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        rp = np.ascontiguousarray(graph.row_ptr, np.int64)
        ci = np.ascontiguousarray(graph.col_idx, np.int32)
        ww = np.ascontiguousarray(graph.w, np.float64)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = L.qsw_superop_build_demoralised(int(graph.N), _ptr(rp), _ptr(ci), _ptr(ww),
                                                 float(omega), float(gamma), _stream(dev),
                                                 ctypes.byref(h))
        _lib.check(st, "qsw_superop_build_demoralised")
        op = cls(h, dev)
        op.copies = demoralised_copies(graph)
        return op

    def set_omega(self, omega):
        """Rebuild for another omega (the paper's set_omega)."""
        torch = _torch()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_superop_set_omega(self._h, float(omega), _stream(self.device))
        _lib.check(st, "qsw_superop_set_omega")
        info = _lib.Info()
        _lib.check(_lib.load().qsw_superop_info(self._h, ctypes.byref(info)), "qsw_superop_info")
        self.omega = info.omega
        self.nnz = info.nnz
        self._info = info

    @classmethod
    def from_workload_graph(cls, graph, omega, **kw):
        return cls.from_graph(graph.N, graph.row_ptr, graph.col_idx, graph.w, omega, **kw)

    @classmethod
    def from_operators(cls, H, ML, omega, M_free=None, device=None):
        """The paper's LQSW(omega, H, M_L): Hermitian H and condensed Lindblad
        matrix M_L (each entry one L_k), given as scipy sparse or dense;
        M_free adds channels outside omega (eq. qsw_ss)."""
        torch = _torch()
        import scipy.sparse as sp
        L = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        Hc = sp.csr_matrix(H, dtype=np.complex128)
        Hc.sort_indices()
        Mc = sp.csr_matrix(ML, dtype=np.float64)
        Mc.sort_indices()
        N = Hc.shape[0]
        hp = np.ascontiguousarray(Hc.indptr, np.int64)
        hc = np.ascontiguousarray(Hc.indices, np.int32)
        hv = np.ascontiguousarray(Hc.data, np.complex128).view(np.float64)
        lp = np.ascontiguousarray(Mc.indptr, np.int64)
        lc = np.ascontiguousarray(Mc.indices, np.int32)
        lv = np.ascontiguousarray(Mc.data, np.float64)
        fp = fc = fv = None
        if M_free is not None:
            Fc = sp.csr_matrix(M_free, dtype=np.float64)
            Fc.sort_indices()
            fp = np.ascontiguousarray(Fc.indptr, np.int64)
            fc = np.ascontiguousarray(Fc.indices, np.int32)
            fv = np.ascontiguousarray(Fc.data, np.float64)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = L.qsw_superop_build_open(
                int(N), _ptr(hp), _ptr(hc), _ptr(hv), _ptr(lp), _ptr(lc), _ptr(lv),
                _ptr(fp) if fp is not None else None, _ptr(fc) if fc is not None else None,
                _ptr(fv) if fv is not None else None, float(omega), 0, _stream(dev),
                ctypes.byref(h))
        _lib.check(st, "qsw_superop_build_open")
        return cls(h, dev)

    # ------------------------------------------------------------- queries
    def info(self) -> dict:
        i = self._info
        return {"N": i.N, "n": i.n, "nnz": i.nnz, "omega": i.omega, "norm1": i.norm1,
                "d": {p: i.d[p] for p in range(2, 10)},
                "d_index": {p: i.d_index[p] for p in range(2, 10)},
                "d_probe": {p: i.d_probe[p] for p in range(2, 10)},
                "norm_products": i.norm_products, "build_ms": i.build_ms,
                "split": bool(i.split), "stream_entries": i.stream_entries,
                "shared_entries": i.shared_entries, "distinct_entries": i.distinct_entries,
                "engine": i.engine}

    def csr(self):
        """Host copies (row_ptr int64, col int32, val complex128)."""
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(self.nnz, np.int32)
        val = np.empty(self.nnz, np.complex128)
        st = _lib.load().qsw_superop_copy_csr(self._h, _ptr(rp), _ptr(col),
                                              _ptr(val.view(np.float64)))
        _lib.check(st, "qsw_superop_copy_csr")
        return rp, col, val

    def set_pacing(self, lookahead: int):
        """lookahead > 0: later propagate calls keep at most that many Taylor
        term launches in flight and enqueue no further terms of a scaling
        step once it has passed the stopping test (the call then returns
        when its last launches are enqueued); 0 turns pacing off."""
        torch = _torch()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_superop_set_pacing(self._h, int(lookahead))
        _lib.check(st, "qsw_superop_set_pacing")

    def set_precision(self, mode):
        """Precision of later propagate calls: False / "double" (complex128);
        True / "single": single-precision superoperator values (each real and
        imaginary part rounded to nearest) with the 2^-24 tolerance, vectors
        and sums complex128; "fp32": single-precision values, vectors and
        products with two-float (hi + lo) accumulation of the Taylor terms,
        norms and parameters in double, and a trace check per output point."""
        torch = _torch()
        prec = _prec_code(mode)
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_superop_set_precision(self._h, prec)
        _lib.check(st, "qsw_superop_set_precision")

    def autotune(self) -> dict:
        """Time the product kernel's launch configurations and keep the
        fastest (results are bitwise unchanged whichever is chosen)."""
        torch = _torch()
        t = _lib.Tuning()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_superop_autotune(self._h, _stream(self.device), ctypes.byref(t))
        _lib.check(st, "qsw_superop_autotune")
        return {"staged": int(t.staged), "grid": t.grid, "us_per_product": t.us_per_product,
                "from_cache": bool(t.from_cache)}

    def workspace_bytes(self, t0, dt, n_steps) -> int:
        return int(_lib.load().qsw_propagate_workspace_bytes(self._h, float(t0), float(dt),
                                                             int(n_steps)))

    # ---------------------------------------------------------- evolution
    def _as_device_state(self, rho0):
        torch = _torch()
        if not torch.is_tensor(rho0):
            rho0 = torch.from_numpy(np.ascontiguousarray(rho0, np.complex128))
        rho0 = rho0.to(device=self.device, dtype=torch.complex128).contiguous()
        if tuple(rho0.shape) not in ((self.N, self.N), (self.n,)):
            raise ValueError(f"rho0 must be {self.N} x {self.N}")
        return rho0

    def propagate(self, rho0, t0=0.0, dt=1.0, n_steps=1, out=None, workspace=None):
        """rho(t0 + k dt), k = 0..n_steps, as a [n_steps+1, N, N] complex128
        tensor on the device (enqueued on the current stream)."""
        torch = _torch()
        L = _lib.load()
        rho0 = self._as_device_state(rho0)
        if out is None:
            out = torch.empty((n_steps + 1, self.N, self.N), dtype=torch.complex128,
                              device=self.device)
        if out.dtype != torch.complex128 or not out.is_contiguous() or \
                out.numel() < (n_steps + 1) * self.n:
            raise ValueError("out must be a contiguous complex128 tensor of "
                             "(n_steps+1) N^2 elements")
        ws = self.workspace_bytes(t0, dt, n_steps)
        if ws == 0:
            raise QswError(1, "qsw_propagate_workspace_bytes")
        if workspace is None or workspace.numel() < ws + 256:
            workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        base = workspace.data_ptr()
        aligned = (base + 255) & ~255
        with torch.cuda.device(self.device):
            st = L.qsw_propagate(self._h, ctypes.c_void_p(rho0.data_ptr()), float(t0), float(dt),
                                 int(n_steps), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(aligned), ws, _stream(self.device))
        _lib.check(st, "qsw_propagate")
        self._keep = (rho0, workspace)  # alive until the stream has used them
        return out

    def step(self, rho0, t):
        """rho(t) = exp(t L) rho0 (the paper's `step`)."""
        return self.propagate(rho0, 0.0, float(t), 1)[1]

    def series(self, rho0, t1, tq, steps):
        """rho(t) at t = t1 + k (tq - t1) / steps, k = 0..steps (the paper's
        `series`): a [steps + 1, N, N] device tensor."""
        steps = int(steps)
        if steps < 1:
            raise ValueError("steps must be at least 1")
        return self.propagate(rho0, float(t1), (float(tq) - float(t1)) / steps, steps)

    def last_stats(self) -> dict:
        s = _lib.Stats()
        st = _lib.load().qsw_last_stats(self._h, ctypes.byref(s))
        if st not in (0, 5):
            _lib.check(st, "qsw_last_stats")
        return {"branch": s.branch, "m": s.m, "s": s.s, "m0": s.m0, "s0": s.s0,
                "launched": s.launched, "products": s.products, "nonfinite": bool(s.nonfinite),
                "ms": s.ms, "bytes": s.bytes, "prec": _lib.PREC_NAMES.get(s.prec, s.prec),
                "trace_dev": s.trace_dev}

    def apply(self, x, out=None):
        """y = L x for a length-n complex128 device vector."""
        torch = _torch()
        x = x.to(device=self.device, dtype=torch.complex128).contiguous().reshape(-1)
        if x.numel() != self.n:
            raise ValueError("x must have N^2 elements")
        y = torch.empty_like(x) if out is None else out
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_apply(self._h, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), _stream(self.device))
        _lib.check(st, "qsw_apply")
        return y

    def populations(self, rho):
        """Diagonals Re rho_k[a, a] of a [count, N, N] device series."""
        torch = _torch()
        rho = rho.contiguous()
        count = rho.numel() // self.n
        pops = torch.empty((count, self.N), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_populations(self._h, ctypes.c_void_p(rho.data_ptr()), count,
                                             ctypes.c_void_p(pops.data_ptr()),
                                             _stream(self.device))
        _lib.check(st, "qsw_populations")
        return pops

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().qsw_superop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ batched walks

def _walk_struct(op, rho0, t0, dt, n_steps, out, pops):
    torch = _torch()
    rho0 = rho0.to(device=op.device, dtype=torch.complex128).contiguous()
    if rho0.dim() == 2:
        rho0 = rho0.unsqueeze(0)
    n0 = rho0.shape[0]
    if tuple(rho0.shape[1:]) != (op.N, op.N):
        raise ValueError("rho0 must be [n0, N, N]")
    for t, shape, dtype in ((out, (n_steps + 1, n0, op.N, op.N), torch.complex128),
                            (pops, (n_steps + 1, n0, op.N), torch.float64)):
        if t is not None and (tuple(t.shape) != shape or t.dtype != dtype or
                              not t.is_contiguous() or t.device != rho0.device):
            raise ValueError(f"output must be a contiguous {dtype} tensor of shape {shape}")
    w = _lib.Walk(op._h, n0, rho0.data_ptr(), float(t0), float(dt), int(n_steps),
                  out.data_ptr() if out is not None else None,
                  pops.data_ptr() if pops is not None else None)
    return w, rho0


class Engine:
    """Many walks advancing together on one device (qsw_engine_*).

    The arena is one device tensor; a walk is admitted (``submit`` returns a
    ticket) only while its vectors fit, and its space returns when it ends.
    """

    def __init__(self, max_walks: int, rhs: int, arena_bytes: int, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)
        self.rhs = int(rhs)
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = (self._arena.data_ptr() + 255) & ~255
        self._e = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_engine_create(int(max_walks), self.rhs, ctypes.c_void_p(base),
                                               int(arena_bytes), _stream(self.device),
                                               ctypes.byref(self._e))
        _lib.check(st, "qsw_engine_create")
        self._held = {}

    @staticmethod
    def walk_bytes(op, n0, t0, dt, n_steps, rhs) -> int:
        w = _lib.Walk(op._h, int(n0), 1, float(t0), float(dt), int(n_steps), None, None)
        return int(_lib.load().qsw_walk_bytes(ctypes.byref(w), int(rhs)))

    def submit(self, op, rho0, t0, dt, n_steps, out=None, pops=None):
        """Ticket of the admitted walk, or None when it does not fit now."""
        torch = _torch()
        w, rho0 = _walk_struct(op, rho0, t0, dt, n_steps, out, pops)
        t = ctypes.c_int64()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_engine_submit(self._e, ctypes.byref(w), ctypes.byref(t))
        if st == 3:  # QSW_ERR_OOM: not admitted
            return None
        _lib.check(st, "qsw_engine_submit")
        self._held[t.value] = (op, rho0, out, pops)
        return t.value

    def run(self, max_cycles: int = 2 ** 31 - 1) -> int:
        torch = _torch()
        live = ctypes.c_int32()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_engine_run(self._e, int(max_cycles), ctypes.byref(live))
        if st != 5:
            _lib.check(st, "qsw_engine_run")
        return live.value

    def poll(self):
        buf = (ctypes.c_int64 * 4096)()
        cnt = ctypes.c_int32()
        done = []
        while True:
            _lib.check(_lib.load().qsw_engine_poll(self._e, buf, 4096, ctypes.byref(cnt)),
                       "qsw_engine_poll")
            done.extend(buf[i] for i in range(cnt.value))
            if cnt.value < 4096:
                break
        for t in done:
            self._held.pop(t, None)
        return done

    def stats(self) -> dict:
        s = _lib.EngineStats()
        _lib.check(_lib.load().qsw_engine_stats(self._e, ctypes.byref(s)), "qsw_engine_stats")
        return _engine_stats_dict(s)

    def close(self):
        if getattr(self, "_e", None):
            _lib.load().qsw_engine_destroy(self._e)
            self._e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _engine_stats_dict(s) -> dict:
    return {"cycles": s.cycles, "products": s.products, "live": s.live,
            "nonfinite": bool(s.nonfinite), "ms": s.ms, "bytes": s.bytes, "graphs": s.graphs,
            "graph_launches": s.graph_launches, "rounds": s.rounds, "staged": bool(s.staged),
            "trace_dev": s.trace_dev}


def batch_propagate(walks, rhs=None, workspace=None):
    """Propagate walks together: each item is (op, rho0[n0, N, N], t0, dt,
    n_steps, out, pops) with out / pops device tensors or None.  Returns the
    engine statistics; results land in the given tensors."""
    torch = _torch()
    if not walks:
        return {}
    structs, keep = [], []
    for (op, rho0, t0, dt, n_steps, out, pops) in walks:
        w, r = _walk_struct(op, rho0, t0, dt, n_steps, out, pops)
        structs.append(w)
        keep.append(r)
    if rhs is None:
        m = max(w.n0 for w in structs)
        rhs = 1 if m == 1 else (2 if m == 2 else 4)
    arr = (_lib.Walk * len(structs))(*structs)
    L = _lib.load()
    need = int(L.qsw_batch_workspace_bytes(arr, len(structs), int(rhs)))
    if need == 0:
        raise QswError(1, "qsw_batch_workspace_bytes")
    dev = walks[0][0].device
    if workspace is None or workspace.numel() < need + 256:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    base = (workspace.data_ptr() + 255) & ~255
    st_out = _lib.EngineStats()
    with torch.cuda.device(dev):
        st = L.qsw_batch_propagate(arr, len(structs), int(rhs), ctypes.c_void_p(base), need,
                                   _stream(dev), ctypes.byref(st_out))
    if st != 5:
        _lib.check(st, "qsw_batch_propagate")
    return {**_engine_stats_dict(st_out), "workspace_bytes": need}


# ------------------------------------------------------- demoralisation

def demoralised_copies(graph) -> np.ndarray:
    """d_v = max(1, number of arcs into v): copies of each vertex (host)."""
    rp = np.ascontiguousarray(graph.row_ptr, np.int64)
    ci = np.ascontiguousarray(graph.col_idx, np.int32)
    d = np.empty(int(graph.N), np.int32)
    M = _lib.load().qsw_demoralised_order(int(graph.N), _ptr(rp), _ptr(ci), _ptr(d))
    if M < 0:
        raise QswError(2, "qsw_demoralised_order")
    return d


def demoralised_state(rho, copies) -> np.ndarray:
    """rho (N x N) -> the expanded set's density matrix (host)."""
    rho = np.ascontiguousarray(rho, np.complex128)
    copies = np.ascontiguousarray(copies, np.int32)
    M = int(copies.sum())
    out = np.empty((M, M), np.complex128)
    _lib.check(_lib.load().qsw_demoralised_state(copies.size, _ptr(copies),
                                                 _ptr(rho.view(np.float64)),
                                                 _ptr(out.view(np.float64))),
               "qsw_demoralised_state")
    return out


def demoralised_populations(pops_d, copies) -> np.ndarray:
    """[count, M] populations of the expanded set -> [count, N] (host)."""
    p = np.ascontiguousarray(np.atleast_2d(pops_d), np.float64)
    copies = np.ascontiguousarray(copies, np.int32)
    out = np.empty((p.shape[0], copies.size), np.float64)
    _lib.check(_lib.load().qsw_demoralised_populations(copies.size, _ptr(copies), _ptr(p),
                                                       p.shape[0], _ptr(out)),
               "qsw_demoralised_populations")
    return out


# ---------------------------------------------------- continuous batching

def _flags(h_mode, r_mode, dephasing):
    f = 0
    if h_mode == "adjacency":
        f |= _lib.QSW_H_ADJACENCY
    elif h_mode != "laplacian":
        raise ValueError(h_mode)
    if r_mode == "colnorm":
        f |= _lib.QSW_R_COLNORM
    elif r_mode != "transition":
        raise ValueError(r_mode)
    if dephasing:
        f |= _lib.QSW_DEPHASING
    return f


class Server:
    """Walks arriving one at a time, each on its own graph, sharing one batch
    engine (qsw_server_*).  Operators are cached on the device by graph;
    outputs are device tensors the server hands back when a walk is done."""

    def __init__(self, arena_bytes: int, cache_bytes: int, max_walks: int = 1024, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)
        self._s = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_server_create(int(arena_bytes), int(cache_bytes), int(max_walks),
                                               _stream(self.device), ctypes.byref(self._s))
        _lib.check(st, "qsw_server_create")
        self._held = {}

    def submit(self, graph, omega, t0, dt, n_steps, rho0=None, gamma=1.0, h_mode="laplacian",
               r_mode="transition", dephasing=False, want_rho=False):
        """Queue a walk on `graph` (workloads.Graph-like: N, row_ptr, col_idx,
        w); rho0 defaults to |0><0|.  Returns the request id."""
        torch = _torch()
        N = int(graph.N)
        if rho0 is None:
            rho0 = torch.zeros((N, N), dtype=torch.complex128, device=self.device)
            rho0[0, 0] = 1.0
        rho0 = rho0.to(device=self.device, dtype=torch.complex128).contiguous()
        pops = torch.empty((n_steps + 1, N), dtype=torch.float64, device=self.device)
        out = (torch.empty((n_steps + 1, N, N), dtype=torch.complex128, device=self.device)
               if want_rho else None)
        rp = np.ascontiguousarray(graph.row_ptr, np.int64)
        ci = np.ascontiguousarray(graph.col_idx, np.int32)
        ww = np.ascontiguousarray(graph.w, np.float64)
        rid = ctypes.c_int64()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_server_submit(
                self._s, N, _ptr(rp), _ptr(ci), _ptr(ww), float(omega), float(gamma),
                _flags(h_mode, r_mode, dephasing), ctypes.c_void_p(rho0.data_ptr()), float(t0),
                float(dt), int(n_steps),
                ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                ctypes.c_void_p(pops.data_ptr()), ctypes.byref(rid))
        _lib.check(st, "qsw_server_submit")
        self._held[rid.value] = (rho0, pops, out)
        return rid.value

    def step(self, max_cycles: int = 16):
        """Run engine cycles; returns (running, pending)."""
        torch = _torch()
        running, pending = ctypes.c_int32(), ctypes.c_int32()
        with torch.cuda.device(self.device):
            st = _lib.load().qsw_server_step(self._s, int(max_cycles), ctypes.byref(running),
                                             ctypes.byref(pending))
        if st != 5:
            _lib.check(st, "qsw_server_step")
        return running.value, pending.value

    def poll(self):
        """[(request id, server latency ms, pops tensor, rho tensor or None)]
        for walks finished since the last poll."""
        ids = (ctypes.c_int64 * 1024)()
        lat = (ctypes.c_double * 1024)()
        cnt = ctypes.c_int32()
        done = []
        while True:
            _lib.check(_lib.load().qsw_server_poll(self._s, ids, lat, 1024, ctypes.byref(cnt)),
                       "qsw_server_poll")
            for i in range(cnt.value):
                rho0, pops, out = self._held.pop(ids[i])
                done.append((ids[i], lat[i], pops, out))
            if cnt.value < 1024:
                break
        return done

    def stats(self) -> dict:
        s = _lib.ServerStats()
        _lib.check(_lib.load().qsw_server_stats(self._s, ctypes.byref(s)), "qsw_server_stats")
        return {k: getattr(s, k) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None):
            _lib.load().qsw_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
