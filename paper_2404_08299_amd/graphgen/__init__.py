"""Seeded synthetic inputs: graphs and batch updates (host side, numpy).

This module holds no PageRank arithmetic. It builds the canonical graphs of
the paper's input contract (a self-loop on every vertex, no duplicate edges,
int32 vertex IDs; Sec. 3.1 and Sec. 5.1.3) in both CSR views, and batch updates
of the form of Sec. 3.3 / Sec. 5.1.4 (deletions of existing non-self-loop
edges, insertions of absent edges, fixed vertex set). Both the HIP library's
tests and benchmarks and the CPU oracle's tests take their inputs from here.

The heavy lifting is in ``graphgen.cpp`` (OpenMP, counter-based SplitMix64
streams, so results do not depend on the thread count).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None

_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def build_library(force: bool = True) -> str:
    """Compile graphgen.cpp into libgraphgen.so next to it."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-Wall",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_library(force=True)
        lib = ctypes.CDLL(_SO)
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                _I32P, _I32P]
        lib.gg_rmat.restype = None
        lib.gg_build.argtypes = [ctypes.c_int32, ctypes.c_int64, _I32P, _I32P, _I32P, _I32P,
                                 _I32P, _I32P]
        lib.gg_build.restype = ctypes.c_int64
        lib.gg_csr_to_edges.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, _I32P]
        lib.gg_csr_to_edges.restype = None
        lib.gg_random_batch.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_uint64, _I32P, _I32P, _I32P,
                                        _I32P]
        lib.gg_random_batch.restype = ctypes.c_int
        lib.gg_apply_view.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int64, _I32P, _I32P,
                                      ctypes.c_int64, _I32P, _I32P, _I32P, _I32P]
        lib.gg_apply_view.restype = ctypes.c_int64
        lib.gg_pa_temporal.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _I32P,
                                       _I32P]
        lib.gg_pa_temporal.restype = ctypes.c_int64
        lib.gg_edge_weights.argtypes = [ctypes.c_int64, _I32P, _I32P, ctypes.c_uint64,
                                        ctypes.c_double, ctypes.c_double, _F64P]
        lib.gg_edge_weights.restype = None
        lib.gg_distinct_vertices.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint64, _I32P]
        lib.gg_distinct_vertices.restype = None
        lib.gg_uniform.argtypes = [ctypes.c_int64, ctypes.c_uint64, _F64P]
        lib.gg_new_pairs.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int64, _I32P, _I32P,
                                     _I32P, _I32P]
        lib.gg_new_pairs.restype = ctypes.c_int64
        lib.gg_uniform.restype = None
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I32P)


def _pf(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_F64P)


@dataclass
class Graph:
    """A canonical directed graph in both CSR views (int32)."""
    n: int
    m: int
    out_offsets: np.ndarray  # [n+1]
    out_targets: np.ndarray  # [m], each row ascending
    in_offsets: np.ndarray   # [n+1]
    in_sources: np.ndarray   # [m], each row ascending

    def out_degree(self) -> np.ndarray:
        return np.diff(self.out_offsets).astype(np.int32)

    def in_degree(self) -> np.ndarray:
        return np.diff(self.in_offsets).astype(np.int32)

    def edges(self):
        """Edge list (src, dst) in out-CSR order (sorted by src, then dst)."""
        src = np.empty(self.m, np.int32)
        dst = np.empty(self.m, np.int32)
        _load().gg_csr_to_edges(self.n, _p32(self.out_offsets), _p32(self.out_targets),
                                _p32(src), _p32(dst))
        return src, dst


@dataclass
class Batch:
    """A batch update: deletions (src, dst) and insertions (src, dst)."""
    del_src: np.ndarray
    del_dst: np.ndarray
    ins_src: np.ndarray
    ins_dst: np.ndarray

    @property
    def size(self) -> int:
        return int(self.del_src.size + self.ins_src.size)

    @staticmethod
    def empty() -> "Batch":
        z = np.zeros(0, np.int32)
        return Batch(z, z.copy(), z.copy(), z.copy())


def rmat_edges(scale: int, n_edges: int, seed: int, a=0.57, b=0.19, c=0.19,
               scramble: bool = True, n: int | None = None):
    """Raw R-MAT edges; endpoints >= n are returned as -1 (rejected)."""
    n = (1 << scale) if n is None else int(n)
    src = np.empty(n_edges, np.int32)
    dst = np.empty(n_edges, np.int32)
    _load().gg_rmat(scale, n_edges, n, a, b, c, seed, int(bool(scramble)), _p32(src), _p32(dst))
    return src, dst


def from_edges(n: int, src, dst) -> Graph:
    """Canonical graph from an edge list: negative endpoints dropped,
    duplicates removed, one self-loop added per vertex."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.size and (src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    e = src.size
    cap = e + n
    oo = np.empty(n + 1, np.int32)
    ot = np.empty(cap, np.int32)
    io = np.empty(n + 1, np.int32)
    isrc = np.empty(cap, np.int32)
    m = _load().gg_build(n, e, _p32(src), _p32(dst), _p32(oo), _p32(ot), _p32(io), _p32(isrc))
    if m < 0:
        raise ValueError("gg_build failed")
    return Graph(n, int(m), oo, ot[:m].copy() if m < cap else ot, io,
                 isrc[:m].copy() if m < cap else isrc)


def rmat_graph(scale: int, edge_factor: float, seed: int = 1, a=0.57, b=0.19, c=0.19,
               scramble: bool = True, n: int | None = None) -> Graph:
    """R-MAT graph, Graph500 style: edge_factor * 2^scale generated edges,
    deduplicated, self-loops added (a self-loop drawn by R-MAT merges into it)."""
    nv = (1 << scale) if n is None else int(n)
    n_edges = int(round(edge_factor * (1 << scale)))
    src, dst = rmat_edges(scale, n_edges, seed, a, b, c, scramble, nv)
    g = from_edges(nv, src, dst)
    del src, dst
    return g


def random_batch(g: Graph, size: int, seed: int, insert_frac: float = 0.8) -> Batch:
    """Random batch of `size` edge updates: round(insert_frac*size) insertions
    of uniform absent pairs (u != v), the rest deletions drawn uniformly
    without replacement from existing non-self-loop edges."""
    n_ins = int(round(insert_frac * size))
    n_del = int(size) - n_ins
    ds = np.empty(n_del, np.int32)
    dd = np.empty(n_del, np.int32)
    is_ = np.empty(n_ins, np.int32)
    id_ = np.empty(n_ins, np.int32)
    rc = _load().gg_random_batch(g.n, _p32(g.out_offsets), _p32(g.out_targets), n_del, n_ins,
                                 seed, _p32(ds), _p32(dd), _p32(is_), _p32(id_))
    if rc != 0:
        raise ValueError("graph too small for the requested batch")
    return Batch(ds, dd, is_, id_)


def batch_size_for(g: Graph, fraction: float) -> int:
    """Batch size for a fraction of |E| (|E| counts self-loops)."""
    return max(1, int(round(fraction * g.m)))


def apply_batch(g: Graph, b: Batch) -> Graph:
    """G^t = G^{t-1} minus deletions plus insertions, both CSR views."""
    lib = _load()
    cap = g.m + b.ins_src.size
    oo = np.empty(g.n + 1, np.int32)
    ot = np.empty(cap, np.int32)
    m1 = lib.gg_apply_view(g.n, _p32(g.out_offsets), _p32(g.out_targets),
                           b.del_src.size, _p32(b.del_src), _p32(b.del_dst),
                           b.ins_src.size, _p32(b.ins_src), _p32(b.ins_dst), _p32(oo), _p32(ot))
    io = np.empty(g.n + 1, np.int32)
    isrc = np.empty(cap, np.int32)
    m2 = lib.gg_apply_view(g.n, _p32(g.in_offsets), _p32(g.in_sources),
                           b.del_src.size, _p32(b.del_dst), _p32(b.del_src),
                           b.ins_src.size, _p32(b.ins_dst), _p32(b.ins_src), _p32(io), _p32(isrc))
    if m1 < 0 or m2 < 0 or m1 != m2:
        raise ValueError("batch is not a normalised update of this graph")
    return Graph(g.n, int(m1), oo, ot[:m1], io, isrc[:m1])


def pa_temporal_events(n: int, n_events: int, seed: int, gamma: float = 2.1,
                       k_min: int = 3, k_max: int | None = None):
    """Preferential-attachment temporal edge stream (src, dst) in time order."""
    k_max = n if k_max is None else k_max
    src = np.empty(n_events, np.int32)
    dst = np.empty(n_events, np.int32)
    k = _load().gg_pa_temporal(n, n_events, gamma, k_min, k_max, seed, _p32(src), _p32(dst))
    if k != n_events:
        raise ValueError("gg_pa_temporal failed")
    return src, dst


def temporal_batch(g: Graph, ev_src, ev_dst, n_del: int, seed: int) -> Batch:
    """One batch of a temporal stream against the current graph g, as set
    differences: the events' unique non-self-loop pairs absent from g are the
    insertions; n_del existing non-self-loop edges of g, drawn uniformly without
    replacement, are the deletions."""
    ev_src = np.ascontiguousarray(ev_src, dtype=np.int32)
    ev_dst = np.ascontiguousarray(ev_dst, dtype=np.int32)
    is_ = np.empty(ev_src.size, np.int32)
    id_ = np.empty(ev_src.size, np.int32)
    k = _load().gg_new_pairs(g.n, _p32(g.out_offsets), _p32(g.out_targets), ev_src.size,
                             _p32(ev_src), _p32(ev_dst), _p32(is_), _p32(id_))
    ds = np.empty(n_del, np.int32)
    dd = np.empty(n_del, np.int32)
    z = np.empty(0, np.int32)
    rc = _load().gg_random_batch(g.n, _p32(g.out_offsets), _p32(g.out_targets), n_del, 0, seed,
                                 _p32(ds), _p32(dd), _p32(z), _p32(z))
    if rc != 0:
        raise ValueError("graph too small for the requested deletions")
    return Batch(ds, dd, is_[:k].copy(), id_[:k].copy())


def temporal_stream(n: int, n_events: int, seed: int, load_frac: float = 0.9,
                    batches: int = 100, del_frac: float = 0.1):
    """Preferential-attachment temporal graph: the first load_frac of the
    events form G^0; the rest are cut into `batches` consecutive insertion
    batches, each with round(del_frac * its event count) deletions of random
    existing edges. Returns (G^0, generator of (batch, G^t)); each batch is
    normalised against the graph it updates (batch seed = seed * 1000 + t)."""
    src, dst = pa_temporal_events(n, n_events, seed)
    n0 = int(round(load_frac * n_events))
    g0 = from_edges(n, src[:n0], dst[:n0])
    cuts = np.linspace(n0, n_events, batches + 1).round().astype(np.int64)

    def steps():
        g = g0
        for t in range(batches):
            a, b = cuts[t], cuts[t + 1]
            bt = temporal_batch(g, src[a:b], dst[a:b], int(round(del_frac * (b - a))),
                                seed=seed * 1000 + t)
            g = apply_batch(g, bt)
            yield bt, g

    return g0, steps()


def edge_weights(src, dst, seed: int, lo: float = 0.1, hi: float = 1.0) -> np.ndarray:
    """Per-edge weights in (lo, hi], a pure function of (seed, src, dst)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    w = np.empty(src.size, np.float64)
    _load().gg_edge_weights(src.size, _p32(src), _p32(dst), seed, lo, hi, _pf(w))
    return w


def distinct_vertices(n: int, sets: int, k: int, seed: int) -> np.ndarray:
    """`sets` rows of k distinct uniform vertex IDs."""
    out = np.empty((sets, k), np.int32)
    _load().gg_distinct_vertices(n, sets, k, seed, _p32(out.reshape(-1)))
    return out


def uniform(count: int, seed: int) -> np.ndarray:
    """`count` uniform doubles in [0, 1)."""
    out = np.empty(count, np.float64)
    _load().gg_uniform(count, seed, _pf(out))
    return out


def relabel(g: Graph, perm) -> Graph:
    """The same graph with vertex v renamed perm[v] (perm a permutation)."""
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    s, d = g.edges()
    out = from_edges(g.n, perm[s], perm[d])
    return out


def degree_order(g: Graph, by: str = "out") -> np.ndarray:
    """perm[v] = position of v when vertices are sorted by descending degree
    (ties by ID)."""
    deg = g.out_degree() if by == "out" else g.in_degree()
    order = np.argsort(-deg.astype(np.int64), kind="stable")
    perm = np.empty(g.n, np.int32)
    perm[order] = np.arange(g.n, dtype=np.int32)
    return perm


def graph_from_arrays(n, out_offsets, out_targets, in_offsets, in_sources) -> Graph:
    return Graph(int(n), int(out_offsets[-1]), np.ascontiguousarray(out_offsets, np.int32),
                 np.ascontiguousarray(out_targets, np.int32),
                 np.ascontiguousarray(in_offsets, np.int32),
                 np.ascontiguousarray(in_sources, np.int32))
