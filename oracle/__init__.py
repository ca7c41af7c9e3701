"""CPU oracle for Static and DF-P PageRank -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its binding) never does, and this package imports nothing from it.

It is a ctypes wrapper over ``pr_oracle.c``: a plain sequential FP64
implementation of the paper's Alg. 1 (Static, Eq. 1), Alg. 2/3/5 (DF and DF-P,
Eq. 2), plus personalised PageRank, the weighted forward and its adjoint.
Inputs are edge lists (src, dst) of a canonical graph; the oracle builds its
own adjacency from them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pr_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)
_U8P = ctypes.POINTER(ctypes.c_uint8)

OK, NOT_CONVERGED = 0, 1

# Paper defaults (Sec. 5.1.2): alpha, frontier/prune tolerance, iteration
# tolerance (L-infinity) and the iteration cap.
ALPHA = 0.85
TAU_F = 1e-6
TAU_P = 1e-6
TOL = 1e-10
MAX_ITERATIONS = 500


def build_library(force: bool = True, extra_flags=(), so_path: str | None = None) -> str:
    """Compile pr_oracle.c (gcc -O2 -ffp-contract=off). `extra_flags` exists so
    that tests can build deliberately broken variants into another file."""
    so = so_path or _SO
    if force or not os.path.exists(so):
        tmp = so + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-shared", "-fPIC", "-Wall",
               *extra_flags, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, so)
    return so


def _bind(lib):
    c = ctypes
    lib.oracle_static.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, c.c_double, c.c_double,
                                  c.c_int32, _F64P, _F64P, _I32P, _F64P]
    lib.oracle_static_csr.argtypes = [c.c_int32, _I32P, _I32P, _I32P, c.c_double, c.c_double,
                                      c.c_int32, _F64P, _I32P, _F64P, _F64P]
    lib.oracle_dfp.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, c.c_int64, _I32P, _I32P,
                               c.c_int64, _I32P, _F64P, c.c_double, c.c_double, c.c_double,
                               c.c_double, c.c_int32, c.c_int32, _F64P, _I32P, _F64P, _I64P,
                               _U8P]
    lib.oracle_dt.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, c.c_int64, _I32P, _I32P,
                              c.c_int64, _I32P, _F64P, c.c_double, c.c_double, c.c_int32, _F64P,
                              _I32P, _F64P, _I64P]
    lib.oracle_ppr.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, c.c_int32, _F64P, c.c_double,
                               c.c_double, c.c_int32, _F64P, _I32P]
    lib.oracle_weighted.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, _F64P, _F64P,
                                    c.c_double, c.c_double, c.c_int32, _F64P, _F64P, _I32P, _F64P]
    lib.oracle_adjoint.argtypes = [c.c_int32, c.c_int64, _I32P, _I32P, _F64P, _F64P, _F64P,
                                   c.c_double, c.c_double, c.c_int32, _F64P, _F64P, _F64P, _I32P]
    lib.oracle_pull_rows.argtypes = [c.c_int32, _I32P, _I32P, _I32P, _F64P, _F64P, c.c_int32,
                                     _F64P, c.c_double, c.c_int64, _I32P, _I32P, _F64P]
    lib.oracle_dfp_csr.argtypes = [c.c_int32, _I32P, _I32P, _I32P, _I32P, c.c_int64, _I32P, _I32P,
                                   c.c_int64, _I32P, _F64P, c.c_double, c.c_double, c.c_double,
                                   c.c_double, c.c_int32, c.c_int32, _F64P, _I32P, _F64P, _I64P]
    for f in (lib.oracle_static, lib.oracle_static_csr, lib.oracle_dfp, lib.oracle_dt, lib.oracle_ppr,
              lib.oracle_weighted, lib.oracle_adjoint, lib.oracle_pull_rows, lib.oracle_dfp_csr):
        f.restype = c.c_int
    return lib


def load(so_path: str | None = None):
    """Load the oracle library (building it if absent). A non-default path
    loads a separately built variant."""
    global _lib
    if so_path is not None:
        return _bind(ctypes.CDLL(so_path))
    if _lib is None:
        if not os.path.exists(_SO):
            build_library(force=True)
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def _check(rc, name):
    if rc < 0:
        raise ValueError(f"{name} failed with status {rc}")
    return rc


@dataclass
class Result:
    ranks: np.ndarray
    iters: int
    delta: float
    status: int
    stats: dict | None = None
    trace: np.ndarray | None = None


def static(n, src, dst, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, init=None,
           lib=None) -> Result:
    """Alg. 1 with Eq. 1; `init` gives the Naive-dynamic variant."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    r = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    pin = None
    if init is not None:
        init, pin = _f64(init)
    rc = lib.oracle_static(n, src.size, ps, pd, alpha, tol, max_iter, pin,
                           r.ctypes.data_as(_F64P), ctypes.byref(it), ctypes.byref(d))
    _check(rc, "oracle_static")
    return Result(r, it.value, d.value, rc)


def static_csr(n, in_offsets, in_sources, out_offsets, alpha=ALPHA, tol=TOL,
               max_iter=MAX_ITERATIONS, lib=None):
    """Alg. 1 over a given in-CSR (rows ascending). Returns (Result, seconds
    spent in the iteration loop)."""
    lib = lib or load()
    io, pio = _i32(in_offsets)
    isrc, pis = _i32(in_sources)
    oo, poo = _i32(out_offsets)
    r = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    sec = ctypes.c_double(0.0)
    rc = lib.oracle_static_csr(n, pio, pis, poo, alpha, tol, max_iter, r.ctypes.data_as(_F64P),
                               ctypes.byref(it), ctypes.byref(d), ctypes.byref(sec))
    _check(rc, "oracle_static_csr")
    return Result(r, it.value, d.value, rc), sec.value


def pull_rows(n, in_offsets, in_sources, out_offsets, ranks, rows, cols=None, weights=None,
              teleport=None, alpha=ALPHA, lib=None):
    """One update of the pull iteration for listed rows (and vectors `cols`
    of a vertex-major ranks[n][k]) only, over a given in-CSR: Eq. 1 by
    default, the weighted forward with per-in-edge `weights`, personalised
    PageRank with a teleport[n][k]. A sample of one step of an iteration on a
    graph too large for the full oracle here."""
    lib = lib or load()
    io, pio = _i32(in_offsets)
    isrc, pis = _i32(in_sources)
    oo, poo = (None, None) if out_offsets is None else _i32(out_offsets)
    r = np.ascontiguousarray(ranks, dtype=np.float64)
    ld = 1 if r.ndim == 1 else r.shape[1]
    rows, prow = _i32(rows)
    cl, pcl = (None, None) if cols is None else _i32(cols)
    w, pw = (None, None) if weights is None else _f64(weights)
    t, pt = (None, None) if teleport is None else _f64(teleport)
    out = np.empty(rows.size, np.float64)
    rc = lib.oracle_pull_rows(n, pio, pis, poo, pw, r.ctypes.data_as(_F64P), ld, pt, alpha,
                              rows.size, prow, pcl, out.ctypes.data_as(_F64P))
    _check(rc, "oracle_pull_rows")
    return out


def static_rows(n, in_offsets, in_sources, out_offsets, ranks, rows, alpha=ALPHA, lib=None):
    """One Eq. 1 update from `ranks` for the listed rows only."""
    return pull_rows(n, in_offsets, in_sources, out_offsets, ranks, rows, alpha=alpha, lib=lib)


def dfp(n, src, dst, batch, ranks_prev, alpha=ALPHA, tol=TOL, tau_f=TAU_F, tau_p=TAU_P,
        max_iter=MAX_ITERATIONS, prune=True, trace=False, lib=None) -> Result:
    """Alg. 2 (DF-P when prune, DF otherwise) on G^t = (src, dst).
    `batch` has del_src, del_dst, ins_src (insertion targets are not read)."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    ds, pds = _i32(batch.del_src)
    dd, pdd = _i32(batch.del_dst)
    is_, pis = _i32(batch.ins_src)
    rp, prp = _f64(ranks_prev)
    r = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    st = np.zeros(4, np.int64)
    tr = np.zeros((max_iter + 1, n), np.uint8) if trace else None
    rc = lib.oracle_dfp(n, src.size, ps, pd, ds.size, pds, pdd, is_.size, pis, prp, alpha, tol,
                        tau_f, tau_p, max_iter, 1 if prune else 0, r.ctypes.data_as(_F64P),
                        ctypes.byref(it), ctypes.byref(d), st.ctypes.data_as(_I64P),
                        tr.ctypes.data_as(_U8P) if trace else None)
    _check(rc, "oracle_dfp")
    stats = dict(affected_initial=int(st[0]), affected_max=int(st[1]),
                 edges_processed=int(st[2]), affected_ever=int(st[3]))
    return Result(r, it.value, d.value, rc, stats, tr[: it.value + 1] if trace else None)


def dfp_csr(g, batch, ranks_prev, alpha=ALPHA, tol=TOL, tau_f=TAU_F, tau_p=TAU_P,
            max_iter=MAX_ITERATIONS, prune=True, lib=None) -> Result:
    """The same run as dfp() over G^t given in both CSR views (an object with
    n, in_offsets, in_sources, out_offsets, out_targets), for graphs whose
    adjacency construction from an edge list is too slow here."""
    lib = lib or load()
    io, pio = _i32(g.in_offsets)
    isrc, pis_ = _i32(g.in_sources)
    oo, poo = _i32(g.out_offsets)
    ot, pot = _i32(g.out_targets)
    ds, pds = _i32(batch.del_src)
    dd, pdd = _i32(batch.del_dst)
    is_, pis = _i32(batch.ins_src)
    rp, prp = _f64(ranks_prev)
    r = np.empty(g.n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    st = np.zeros(4, np.int64)
    rc = lib.oracle_dfp_csr(g.n, pio, pis_, poo, pot, ds.size, pds, pdd, is_.size, pis, prp, alpha,
                            tol, tau_f, tau_p, max_iter, 1 if prune else 0, r.ctypes.data_as(_F64P),
                            ctypes.byref(it), ctypes.byref(d), st.ctypes.data_as(_I64P))
    _check(rc, "oracle_dfp_csr")
    stats = dict(affected_initial=int(st[0]), affected_max=int(st[1]),
                 edges_processed=int(st[2]), affected_ever=int(st[3]))
    return Result(r, it.value, d.value, rc, stats)


def dt(n, src, dst, batch, ranks_prev, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS,
       lib=None) -> Result:
    """Dynamic Traversal (Alg. 7) on G^t = (src, dst): the vertices reachable
    from the batch are affected, Eq. 1 runs over them. stats['affected']."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    ds, pds = _i32(batch.del_src)
    dd, pdd = _i32(batch.del_dst)
    is_, pis = _i32(batch.ins_src)
    rp, prp = _f64(ranks_prev)
    r = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    na = ctypes.c_int64(0)
    rc = lib.oracle_dt(n, src.size, ps, pd, ds.size, pds, pdd, is_.size, pis, prp, alpha, tol,
                       max_iter, r.ctypes.data_as(_F64P), ctypes.byref(it), ctypes.byref(d),
                       ctypes.byref(na))
    _check(rc, "oracle_dt")
    return Result(r, it.value, d.value, rc, dict(affected=int(na.value)), None)


def ppr(n, src, dst, teleport, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, lib=None):
    """Personalised PageRank, teleport [n][k] vertex-major. Returns (ranks[n][k], iters[k])."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    s = np.ascontiguousarray(teleport, dtype=np.float64)
    if s.ndim == 1:
        s = s[:, None]
    k = s.shape[1]
    r = np.empty((n, k), np.float64)
    its = np.zeros(k, np.int32)
    rc = lib.oracle_ppr(n, src.size, ps, pd, k, s.ctypes.data_as(_F64P), alpha, tol, max_iter,
                        r.ctypes.data_as(_F64P), its.ctypes.data_as(_I32P))
    _check(rc, "oracle_ppr")
    return r, its


def weighted(n, src, dst, w, s, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, init=None,
             lib=None) -> Result:
    """Weighted forward r = alpha*A r + (1-alpha) s with A[v][u] = w(u->v)."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    w, pw = _f64(w)
    s, pss = _f64(s)
    r = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    d = ctypes.c_double(0.0)
    pin = None
    if init is not None:
        init, pin = _f64(init)
    rc = lib.oracle_weighted(n, src.size, ps, pd, pw, pss, alpha, tol, max_iter, pin,
                             r.ctypes.data_as(_F64P), ctypes.byref(it), ctypes.byref(d))
    _check(rc, "oracle_weighted")
    return Result(r, it.value, d.value, rc)


def adjoint(n, src, dst, w, r, g, alpha=ALPHA, tol=TOL, max_iter=MAX_ITERATIONS, lib=None):
    """Returns (grad_w[m] in edge-list order, grad_s[n], lambda[n], iters)."""
    lib = lib or load()
    src, ps = _i32(src)
    dst, pd = _i32(dst)
    w, pw = _f64(w)
    r, pr = _f64(r)
    g, pg = _f64(g)
    gw = np.empty(src.size, np.float64)
    gs = np.empty(n, np.float64)
    lam = np.empty(n, np.float64)
    it = ctypes.c_int32(0)
    rc = lib.oracle_adjoint(n, src.size, ps, pd, pw, pr, pg, alpha, tol, max_iter,
                            gw.ctypes.data_as(_F64P), gs.ctypes.data_as(_F64P),
                            lam.ctypes.data_as(_F64P), ctypes.byref(it))
    _check(rc, "oracle_adjoint")
    return gw, gs, lam, it.value
