"""Python binding of libprhip.so (the C ABI in include/prhip.h).

Argument marshalling only: torch provides device memory and the stream, and
every step of the computation runs in the library's HIP kernels. There is no
CPU fallback; if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_PKG, "libprhip.so")

PR_OK, PR_NOT_CONVERGED = 0, 1
PR_EINVAL, PR_EGRAPH, PR_EBATCH, PR_ENOMEM, PR_EHIP = -1, -2, -3, -4, -5
MODES = {"dfp": 0, "df": 1, "nd": 2, "dt": 3}

ALPHA, TOL, FRONTIER_TOL, PRUNE_TOL, MAX_ITERATIONS = 0.85, 1e-10, 1e-6, 1e-6, 500
NOALLOC_MAX_N = 1 << 20  # PR_NOALLOC_MAX_N


class PrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"prhip error {code}: {msg}")
        self.code = code


class PrCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("in_offsets", ctypes.c_void_p), ("in_sources", ctypes.c_void_p),
                ("out_offsets", ctypes.c_void_p), ("out_targets", ctypes.c_void_p)]


class PrCsrOut(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("in_offsets", ctypes.c_void_p), ("in_sources", ctypes.c_void_p),
                ("out_offsets", ctypes.c_void_p), ("out_targets", ctypes.c_void_p)]


class PrEdges(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("count", ctypes.c_int32)]


class PrTuning(ctypes.Structure):
    _fields_ = [("lane_max_degree", ctypes.c_int32), ("wave_max_degree", ctypes.c_int32),
                ("expand_lane_max_degree", ctypes.c_int32), ("iters_per_sync", ctypes.c_int32),
                ("hub_chunk_edges", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("relabel", ctypes.c_int32), ("xcd_split_degree", ctypes.c_int32),
                ("expand_pull_per_mille", ctypes.c_int32), ("frontier_list", ctypes.c_int32),
                ("chain_numbering", ctypes.c_int32), ("ppr_chunk_edges", ctypes.c_int32)]


TUNING_FIELDS = ("lane_max_degree", "wave_max_degree", "expand_lane_max_degree",
                 "iters_per_sync", "hub_chunk_edges", "grid_blocks", "relabel",
                 "xcd_split_degree", "expand_pull_per_mille", "frontier_list", "chain_numbering",
                 "ppr_chunk_edges")


class PrStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("final_delta", ctypes.c_double), ("affected_initial", ctypes.c_int64),
                ("rank_kernel_ms", ctypes.c_double), ("rank_kernel_launches", ctypes.c_int32),
                ("numbering", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("affected_max", ctypes.c_int64), ("edges_processed", ctypes.c_int64),
                ("reserved", ctypes.c_double * 2)]


EXPORTED = ["pr_static", "pr_static_noalloc", "pr_dfp", "pr_dfp_ex", "pr_ppr", "pr_static_batched", "pr_weighted",
            "pr_adjoint", "pr_apply_batch",
            "pr_validate_csr", "pr_set_tuning",
            "pr_get_tuning", "pr_last_stats", "pr_set_profiling", "pr_set_stream",
            "pr_last_error", "pr_release"]

_lib = None


def load_library(path: str = SO_PATH):
    """Load libprhip.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None and path == SO_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    d = ctypes.c_double
    i = ctypes.c_int
    lib.pr_static.argtypes = [P(PrCsr), d, d, i, vp]
    lib.pr_static_noalloc.argtypes = [P(PrCsr), d, d, i, vp]
    lib.pr_dfp.argtypes = [P(PrCsr), P(PrCsr), P(PrEdges), P(PrEdges), vp, d, d, d, d, vp]
    lib.pr_dfp_ex.argtypes = [P(PrCsr), P(PrCsr), P(PrEdges), P(PrEdges), vp, d, d, d, d, i, i,
                              vp]
    lib.pr_ppr.argtypes = [P(PrCsr), vp, i, d, d, i, vp, P(ctypes.c_int32)]
    lib.pr_static_batched.argtypes = [P(PrCsr), i, P(vp), d, d, i, P(vp), P(ctypes.c_int32)]
    lib.pr_weighted.argtypes = [P(PrCsr), vp, vp, d, d, i, vp]
    lib.pr_adjoint.argtypes = [P(PrCsr), vp, vp, vp, d, d, i, vp, vp, vp]
    lib.pr_validate_csr.argtypes = [P(PrCsr)]
    lib.pr_set_tuning.argtypes = [P(PrTuning)]
    lib.pr_get_tuning.argtypes = [P(PrTuning)]
    lib.pr_last_stats.argtypes = [P(PrStats)]
    lib.pr_set_profiling.argtypes = [i]
    lib.pr_set_stream.argtypes = [vp]
    lib.pr_set_stream.restype = None
    lib.pr_last_error.argtypes = []
    lib.pr_last_error.restype = ctypes.c_char_p
    lib.pr_release.argtypes = []
    lib.pr_release.restype = None
    lib.pr_apply_batch.argtypes = [P(PrCsr), P(PrEdges), P(PrEdges), P(PrCsrOut)]
    for f in ("pr_static", "pr_static_noalloc", "pr_dfp", "pr_dfp_ex", "pr_ppr", "pr_static_batched", "pr_weighted",
              "pr_adjoint", "pr_apply_batch",
              "pr_validate_csr", "pr_set_tuning",
              "pr_get_tuning", "pr_last_stats", "pr_set_profiling"):
        getattr(lib, f).restype = ctypes.c_int
    if path == SO_PATH:
        _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("prhip needs a HIP GPU (torch.cuda.is_available() is False)")
    return torch


def _check(rc: int, lib) -> int:
    if rc < 0:
        raise PrError(rc, lib.pr_last_error().decode())
    if rc == PR_NOT_CONVERGED:
        warnings.warn("prhip: iteration cap reached before the tolerance", RuntimeWarning,
                      stacklevel=3)
    return rc


def _bind_stream(lib, torch):
    lib.pr_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _tensor(x, name, dtype, device, numel=None, shape=None):
    """x as the C ABI receives it: a contiguous tensor of `dtype` on `device`
    with the given size. Anything else raises here (TypeError for the kind,
    ValueError for place, layout or size), before a pointer reaches a kernel."""
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(x).__name__}")
    if x.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {x.dtype}")
    if x.device != device:
        raise ValueError(f"{name}: expected a tensor on {device}, got one on {x.device}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and x.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {x.numel()}")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(x.shape)}")
    return x


def _on_current_device(device, torch):
    """The library allocates its workspace and launches on the current device
    and stream, so the tensors must live there."""
    if device.type != "cuda":
        raise ValueError(f"graph tensors must be on a GPU, got {device}")
    cur = torch.cuda.current_device()
    if device.index is not None and device.index != cur:
        raise ValueError(f"graph is on {device} but the current device is cuda:{cur}; "
                         f"call under torch.cuda.device({device.index})")


class DeviceGraph:
    """Both CSR views of a graph as int32 device tensors (torch storage)."""

    def __init__(self, n, m, in_offsets, in_sources, out_offsets, out_targets):
        self.n, self.m = int(n), int(m)
        self.in_offsets, self.in_sources = in_offsets, in_sources
        self.out_offsets, self.out_targets = out_offsets, out_targets

    @staticmethod
    def from_host(g, device="cuda") -> "DeviceGraph":
        torch = _torch()

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)

        return DeviceGraph(g.n, g.m, t(g.in_offsets), t(g.in_sources), t(g.out_offsets),
                           t(g.out_targets))

    @property
    def device(self):
        return self.in_offsets.device

    def csr(self) -> PrCsr:
        """The pr_csr view, after checking that every present array is int32,
        contiguous, on the graph's device and of its CSR size."""
        import torch
        if self.n < 0 or self.m < 0:
            raise ValueError(f"graph sizes must be non-negative, got n={self.n} m={self.m}")
        dev, i32 = self.device, torch.int32
        _tensor(self.in_offsets, "in_offsets", i32, dev, numel=self.n + 1)
        _tensor(self.in_sources, "in_sources", i32, dev, numel=self.m)
        if self.out_offsets is not None:
            _tensor(self.out_offsets, "out_offsets", i32, dev, numel=self.n + 1)
        if self.out_targets is not None:
            _tensor(self.out_targets, "out_targets", i32, dev, numel=self.m)

        def p(x):
            return None if x is None else x.data_ptr()

        return PrCsr(self.n, self.m, p(self.in_offsets), p(self.in_sources), p(self.out_offsets),
                     p(self.out_targets))


class DeviceBatch:
    """A batch update (deletions src/dst, insertions src/dst) on the device."""

    def __init__(self, del_src, del_dst, ins_src, ins_dst):
        self.del_src, self.del_dst, self.ins_src, self.ins_dst = del_src, del_dst, ins_src, ins_dst

    @staticmethod
    def from_host(b, device="cuda") -> "DeviceBatch":
        torch = _torch()

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)

        return DeviceBatch(t(b.del_src), t(b.del_dst), t(b.ins_src), t(b.ins_dst))

    def edges(self, device=None):
        """The two pr_edges views (deletions, insertions), after checking that
        the arrays are int32, contiguous, on `device` (default: where del_src
        is) and that each dst matches its src in length."""
        import torch
        dev = device if device is not None else self.del_src.device

        def e(s, d, name):
            _tensor(s, name + "_src", torch.int32, dev)
            n = int(s.numel())
            if d is not None:
                _tensor(d, name + "_dst", torch.int32, dev, numel=n)
            return PrEdges(s.data_ptr() if n else None, d.data_ptr() if (d is not None and n) else None, n)

        return e(self.del_src, self.del_dst, "del"), e(self.ins_src, self.ins_dst, "ins")


@dataclass
class Result:
    ranks: object  # torch float64 tensor on the device
    status: int
    iterations: int
    converged: bool
    final_delta: float
    stats: dict


def last_stats() -> dict:
    lib = load_library()
    s = PrStats()
    lib.pr_last_stats(ctypes.byref(s))
    return dict(iterations=s.iterations, converged=bool(s.converged), final_delta=s.final_delta,
                affected_initial=s.affected_initial, rank_kernel_ms=s.rank_kernel_ms,
                rank_kernel_launches=s.rank_kernel_launches, total_ms=s.total_ms,
                affected_max=s.affected_max, edges_processed=s.edges_processed,
                numbering=s.numbering)


def _result(rc, out):
    st = last_stats()
    return Result(out, rc, st["iterations"], st["converged"], st["final_delta"], st)


def static(g: DeviceGraph, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, out=None) -> Result:
    """Static PageRank (Alg. 1, Eq. 1) through pr_static."""
    torch = _torch()
    lib = load_library()
    _on_current_device(g.device, torch)
    csr = g.csr()
    if out is None:
        out = torch.empty(g.n, dtype=torch.float64, device=g.device)
    _tensor(out, "out", torch.float64, g.device, numel=g.n)
    _bind_stream(lib, torch)
    rc = _check(lib.pr_static(ctypes.byref(csr), alpha, tol, max_iter, out.data_ptr()), lib)
    return _result(rc, out)


def static_noalloc(g: DeviceGraph, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS,
                   out=None) -> Result:
    """Static PageRank through pr_static_noalloc (no device allocation inside
    the call; n <= NOALLOC_MAX_N). `out` is required by callers that must not
    allocate either; without it one output tensor is allocated here."""
    torch = _torch()
    lib = load_library()
    _on_current_device(g.device, torch)
    csr = g.csr()
    if out is None:
        out = torch.empty(g.n, dtype=torch.float64, device=g.device)
    _tensor(out, "out", torch.float64, g.device, numel=g.n)
    _bind_stream(lib, torch)
    rc = _check(lib.pr_static_noalloc(ctypes.byref(csr), alpha, tol, max_iter, out.data_ptr()),
                lib)
    return _result(rc, out)


def dfp(g_new: DeviceGraph, batch: DeviceBatch, ranks_prev, alpha=ALPHA, tol=TOL,
        frontier_tol=FRONTIER_TOL, prune_tol=PRUNE_TOL, max_iter=MAX_ITERATIONS, mode="dfp",
        out=None, g_old: DeviceGraph | None = None) -> Result:
    """DF-P (default), DF, ND or DT update through pr_dfp / pr_dfp_ex."""
    torch = _torch()
    lib = load_library()
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}, got {mode!r}")
    dev = g_new.device
    _on_current_device(dev, torch)
    csr_new = g_new.csr()
    csr_old = g_old.csr() if g_old is not None else None
    if g_old is not None and (g_old.device != dev or g_old.n != g_new.n):
        raise ValueError("g_old must have g_new's vertex count and device")
    de, ie = batch.edges(dev)
    _tensor(ranks_prev, "ranks_prev", torch.float64, dev, numel=g_new.n)
    if out is None:
        out = torch.empty(g_new.n, dtype=torch.float64, device=dev)
    _tensor(out, "out", torch.float64, dev, numel=g_new.n)
    _bind_stream(lib, torch)
    if mode == "dfp" and max_iter == MAX_ITERATIONS:
        rc = lib.pr_dfp(ctypes.byref(csr_old) if csr_old else None, ctypes.byref(csr_new),
                        ctypes.byref(de), ctypes.byref(ie), ranks_prev.data_ptr(), alpha, tol,
                        frontier_tol, prune_tol, out.data_ptr())
    else:
        rc = lib.pr_dfp_ex(ctypes.byref(csr_old) if csr_old else None, ctypes.byref(csr_new),
                           ctypes.byref(de), ctypes.byref(ie), ranks_prev.data_ptr(), alpha, tol,
                           frontier_tol, prune_tol, max_iter, MODES[mode], out.data_ptr())
    _check(rc, lib)
    return _result(rc, out)


def apply_batch(g_old: DeviceGraph, batch: DeviceBatch, out_view: bool = True) -> DeviceGraph:
    """G^t = G^{t-1} - deletions + insertions on the device (pr_apply_batch);
    the batch must be normalised (set differences) and carry insertion
    targets. Returns a new DeviceGraph."""
    torch = _torch()
    lib = load_library()
    dev = g_old.device
    _on_current_device(dev, torch)
    csr_old = g_old.csr()
    de, ie = batch.edges(dev)
    nd, ni = de.count, ie.count
    m = g_old.m - nd + ni
    e = lambda k: torch.empty(k, dtype=torch.int32, device=dev)
    io, isrc = e(g_old.n + 1), e(max(m, 1))
    oo, otg = (e(g_old.n + 1), e(max(m, 1))) if out_view else (None, None)
    p = lambda x: None if x is None else x.data_ptr()
    out = PrCsrOut(g_old.n, m, p(io), p(isrc), p(oo), p(otg))
    _bind_stream(lib, torch)
    rc = lib.pr_apply_batch(ctypes.byref(csr_old), ctypes.byref(de), ctypes.byref(ie),
                            ctypes.byref(out))
    _check(rc, lib)
    return DeviceGraph(g_old.n, m, io, isrc[:m], oo, otg[:m] if otg is not None else None)


def ppr(g: DeviceGraph, teleport, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, out=None):
    """Personalised PageRank through pr_ppr. teleport: [n][k] float64 device
    tensor (vertex-major). Returns (Result with ranks [n][k], iterations per
    vector as a numpy array)."""
    torch = _torch()
    lib = load_library()
    _on_current_device(g.device, torch)
    csr = g.csr()
    _tensor(teleport, "teleport", torch.float64, g.device)
    if teleport.dim() == 1:
        teleport = teleport.view(-1, 1)
    if teleport.dim() != 2 or teleport.shape[0] != g.n or teleport.shape[1] < 1:
        raise ValueError(f"teleport: expected shape ({g.n}, k) with k >= 1, got "
                         f"{tuple(teleport.shape)}")
    n, k = teleport.shape
    if out is None:
        out = torch.empty((n, k), dtype=torch.float64, device=g.device)
    _tensor(out, "out", torch.float64, g.device, shape=(n, k))
    its = np.zeros(k, np.int32)
    _bind_stream(lib, torch)
    rc = _check(lib.pr_ppr(ctypes.byref(csr), teleport.data_ptr(), k, alpha, tol, max_iter,
                           out.data_ptr(), its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                lib)
    return _result(rc, out), its


def _ptr(x):
    return None if x is None else x.data_ptr()


def static_batched(graphs, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, outs=None,
                   teleports=None):
    """Static PageRank on many graphs in one batched call (pr_static_batched).
    teleports: None (every graph uniform) or a list with, per graph, None
    (uniform) or an [n_g] float64 device tensor s_g (personalised PageRank
    on that graph). A graph may appear several times, once per vector.
    Returns (Result with ranks = list of [n_g] tensors, iterations per graph)."""
    torch = _torch()
    lib = load_library()
    G = len(graphs)
    if G < 1:
        raise ValueError("static_batched needs at least one graph")
    dev = graphs[0].device
    _on_current_device(dev, torch)
    if any(g.device != dev for g in graphs):
        raise ValueError("all graphs of a batched call must be on one device")
    csrs = (PrCsr * G)(*[g.csr() for g in graphs])
    if outs is None:
        outs = [torch.empty(g.n, dtype=torch.float64, device=dev) for g in graphs]
    if len(outs) != G:
        raise ValueError(f"outs: expected {G} tensors, got {len(outs)}")
    for i, (g, o) in enumerate(zip(graphs, outs)):
        _tensor(o, f"outs[{i}]", torch.float64, dev, numel=g.n)
    ptrs = (ctypes.c_void_p * G)(*[o.data_ptr() for o in outs])
    tptrs = None
    if teleports is not None:
        if len(teleports) != G:
            raise ValueError(f"teleports: expected {G} entries, got {len(teleports)}")
        for i, (g, t) in enumerate(zip(graphs, teleports)):
            if t is not None:
                _tensor(t, f"teleports[{i}]", torch.float64, dev, numel=g.n)
        tptrs = (ctypes.c_void_p * G)(*[_ptr(t) for t in teleports])
    its = np.zeros(G, np.int32)
    _bind_stream(lib, torch)
    rc = _check(lib.pr_static_batched(csrs, G, tptrs, alpha, tol, max_iter, ptrs,
                                      its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), lib)
    return _result(rc, outs), its


def weighted(g: DeviceGraph, in_weights, teleport=None, alpha=ALPHA, tol=TOL,
             max_iter=MAX_ITERATIONS, out=None) -> Result:
    """Weighted forward r = alpha*A r + (1-alpha) s through pr_weighted.
    in_weights: [m] float64 in in-CSR order; teleport: [n] or None (1/n)."""
    torch = _torch()
    lib = load_library()
    _on_current_device(g.device, torch)
    csr = g.csr()
    _tensor(in_weights, "in_weights", torch.float64, g.device, numel=g.m)
    if teleport is not None:
        _tensor(teleport, "teleport", torch.float64, g.device, numel=g.n)
    if out is None:
        out = torch.empty(g.n, dtype=torch.float64, device=g.device)
    _tensor(out, "out", torch.float64, g.device, numel=g.n)
    _bind_stream(lib, torch)
    rc = _check(lib.pr_weighted(ctypes.byref(csr), in_weights.data_ptr(), _ptr(teleport), alpha,
                                tol, max_iter, out.data_ptr()), lib)
    return _result(rc, out)


def adjoint(g: DeviceGraph, in_weights, ranks, grad_ranks, alpha=ALPHA, tol=TOL,
            max_iter=MAX_ITERATIONS, want_weights=True, want_teleport=True, want_lambda=False):
    """Adjoint of pr_weighted through pr_adjoint. Returns (grad_weights [m] in
    in-CSR order or None, grad_teleport [n] or None, lambda [n] or None)."""
    torch = _torch()
    lib = load_library()
    dev = g.device
    _on_current_device(dev, torch)
    csr = g.csr()
    if g.out_offsets is None or g.out_targets is None:
        raise ValueError("adjoint needs the graph's out-CSR view")
    _tensor(in_weights, "in_weights", torch.float64, dev, numel=g.m)
    _tensor(ranks, "ranks", torch.float64, dev, numel=g.n)
    _tensor(grad_ranks, "grad_ranks", torch.float64, dev, numel=g.n)
    gw = torch.empty(g.m, dtype=torch.float64, device=dev) if want_weights else None
    gs = torch.empty(g.n, dtype=torch.float64, device=dev) if want_teleport else None
    lam = torch.empty(g.n, dtype=torch.float64, device=dev) if want_lambda else None
    _bind_stream(lib, torch)
    _check(lib.pr_adjoint(ctypes.byref(csr), in_weights.data_ptr(), ranks.data_ptr(),
                          grad_ranks.data_ptr(), alpha, tol, max_iter, _ptr(gw), _ptr(gs),
                          _ptr(lam)), lib)
    return gw, gs, lam


def validate(g: DeviceGraph) -> None:
    """Raises PrError(PR_EGRAPH) if the graph breaks the input contract."""
    torch = _torch()
    lib = load_library()
    _on_current_device(g.device, torch)
    csr = g.csr()
    _bind_stream(lib, torch)
    _check(lib.pr_validate_csr(ctypes.byref(csr)), lib)


def get_tuning() -> dict:
    lib = load_library()
    t = PrTuning()
    lib.pr_get_tuning(ctypes.byref(t))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def set_tuning(**kw) -> None:
    """Update fields of the process-wide tuning; set_tuning() with no
    arguments restores the defaults."""
    lib = load_library()
    if not kw:
        _check(lib.pr_set_tuning(None), lib)
        return
    cur = get_tuning()
    unknown = set(kw) - set(TUNING_FIELDS)
    if unknown:
        raise KeyError(f"unknown tuning fields {sorted(unknown)}")
    cur.update(kw)
    t = PrTuning(*[cur[f] for f in TUNING_FIELDS])
    _check(lib.pr_set_tuning(ctypes.byref(t)), lib)


def set_profiling(enable: bool, counters: bool = True) -> None:
    """Per-launch event timing on or off; with `counters` (the default) also
    the affected-set counters of the dynamic variants (profiling level 2)."""
    lib = load_library()
    _check(lib.pr_set_profiling((2 if counters else 1) if enable else 0), lib)


def release() -> None:
    load_library().pr_release()
