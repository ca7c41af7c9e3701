"""Autotuner for the launch parameters of libprhip (pr_tuning).

Alg. 4 leaves the degree threshold that splits vertices between the
thread-per-vertex and block-per-vertex kernels unspecified; here the
thresholds (lane / wavefront / die-split / split-chunk sizes, the expand
threshold), the gather-side relabelling switch and the host/device
pipelining depth are picked by measurement on the graph at hand.

Search: coordinate descent over one field at a time (two passes), each
candidate scored by short runs of the real entry point with the iteration cap
lowered and the tolerance at 0. A run of k iterations costs roughly
fixed + k * per_iteration, so two caps (k1 < k2) give both terms and the score
is fixed + expected_iterations * per_iteration. The tuning only changes the
order of floating-point summation in wavefront/workgroup reductions, never the
method, so a tuned call returns the same ranks up to rounding (tested).

Best tunings are cached in a JSON file keyed by the entry point and a size
class of the graph (log2 of n and of the average degree, rounded), so later
calls on similar graphs reuse them.
"""
from __future__ import annotations

import json
import math
import os
import time
import warnings

from . import prhip

DEFAULT_SPACE = {
    "lane_max_degree": [4, 8, 32, 64, 128, 256],
    "wave_max_degree": [1024, 4096, 16384],
    "xcd_split_degree": [0, 65, 129, 257, 1024],
    "hub_chunk_edges": [1024, 4096, 8192],
    "relabel": [0, 1],
    "iters_per_sync": [1, 2, 4],
}
DFP_SPACE = dict(DEFAULT_SPACE, expand_lane_max_degree=[8, 32, 128],
                 expand_pull_per_mille=[0, 5, 20, 100], frontier_list=[0, 1])
# pr_ppr reads the row-split size, the die split on/off, the relabel switch
# and the pipelining depth (its long rows are split at ppr_chunk_edges)
PPR_SPACE = {
    "ppr_chunk_edges": [64, 128, 256, 512, 1024],
    "xcd_split_degree": [0, 129],
    "relabel": [0, 1],
    "iters_per_sync": [1, 2, 4],
}

CACHE_PATH = os.environ.get("PRHIP_TUNING_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "prhip_tuning.json"))


def size_class(n: int, m: int) -> str:
    return f"n2^{round(math.log2(max(n, 1)))}_d2^{round(math.log2(max(m / max(n, 1), 1.0)))}"


def _valid(t: dict) -> bool:
    return (t["lane_max_degree"] <= t["wave_max_degree"]
            and t.get("expand_lane_max_degree", 0) <= t["wave_max_degree"])


def _timed(fn) -> float:
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def score(run, tuning: dict, k1: int, k2: int, expected_iters: int, repeats: int = 2) -> float:
    """Estimated seconds of a full call: run(max_iter) is timed at two caps."""
    prhip.set_tuning(**tuning)
    _timed(lambda: run(k1))  # warm-up (workspace, code paths)
    t1 = min(_timed(lambda: run(k1)) for _ in range(repeats))
    t2 = min(_timed(lambda: run(k2)) for _ in range(repeats))
    per_iter = max(0.0, (t2 - t1) / (k2 - k1))
    fixed = max(0.0, t1 - k1 * per_iter)
    return fixed + expected_iters * per_iter


def coordinate_descent(run, space: dict, base: dict | None = None, k1: int = 2, k2: int = 6,
                       expected_iters: int = 64, passes: int = 2, log=None) -> tuple[dict, float]:
    """Minimise score() one field at a time; returns (best tuning, score)."""
    prhip.set_tuning()
    best = dict(prhip.get_tuning())
    if base:
        best.update(base)
    best_s = score(run, best, k1, k2, expected_iters)
    seen = {tuple(sorted(best.items())): best_s}
    for _ in range(passes):
        improved = False
        for field, values in space.items():
            for v in values:
                cand = dict(best, **{field: v})
                if not _valid(cand):
                    continue
                key = tuple(sorted(cand.items()))
                if key in seen:
                    s = seen[key]
                else:
                    s = score(run, cand, k1, k2, expected_iters)
                    seen[key] = s
                    if log:
                        log(f"autotune {field}={v}: {s * 1e3:.2f} ms")
                if s < best_s * 0.995:
                    best, best_s, improved = cand, s, True
        if not improved:
            break
    prhip.set_tuning(**best)
    return best, best_s


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _cached(kind: str, n: int, m: int, tune, cache_path: str | None, refresh: bool):
    path = cache_path or CACHE_PATH
    key = f"{kind}:{size_class(n, m)}"
    cache = _load_cache(path)
    if key in cache and not refresh:
        prhip.set_tuning(**cache[key]["tuning"])
        return cache[key]["tuning"]
    best, s = tune()
    cache = _load_cache(path)
    cache[key] = {"tuning": best, "score_ms": s * 1e3}
    _store_cache(path, cache)
    return best


def tune_static(g: "prhip.DeviceGraph", expected_iters: int = 64, cache_path: str | None = None,
                refresh: bool = False, log=None) -> dict:
    """Tune pr_static on graph g; sets and returns the best tuning."""
    import torch
    out = torch.empty(g.n, dtype=torch.float64, device=g.in_offsets.device)

    def run(k):
        prhip.static(g, tol=0.0, max_iter=k, out=out)

    return _cached("static", g.n, g.m,
                   lambda: coordinate_descent(run, DEFAULT_SPACE, expected_iters=expected_iters,
                                              log=log), cache_path, refresh)


def tune_batched(graphs, expected_iters: int = 64, cache_path: str | None = None,
                 refresh: bool = False, log=None) -> dict:
    """Tune pr_static_batched on a list of graphs."""
    import torch
    outs = [torch.empty(g.n, dtype=torch.float64, device=g.in_offsets.device) for g in graphs]
    n = sum(g.n for g in graphs)
    m = sum(g.m for g in graphs)

    def run(k):
        prhip.static_batched(graphs, tol=0.0, max_iter=k, outs=outs)

    return _cached(f"batched{len(graphs)}", n, m,
                   lambda: coordinate_descent(run, DEFAULT_SPACE, k1=2, k2=6,
                                              expected_iters=expected_iters, log=log),
                   cache_path, refresh)


def tune_ppr(g: "prhip.DeviceGraph", teleport, expected_iters: int = 64,
             cache_path: str | None = None, refresh: bool = False, log=None) -> dict:
    """Tune pr_ppr on graph g with the [n][k] teleport matrix (the cache key
    includes k)."""
    import torch
    k = int(teleport.shape[1])
    out = torch.empty(g.n, k, dtype=torch.float64, device=g.in_offsets.device)

    def run(it):
        prhip.ppr(g, teleport, tol=0.0, max_iter=it, out=out)

    return _cached(f"ppr{k}", g.n, g.m,
                   lambda: coordinate_descent(run, PPR_SPACE, k1=2, k2=6,
                                              expected_iters=expected_iters, log=log),
                   cache_path, refresh)


def tune_dfp(g_new, batch, ranks_prev, expected_iters: int = 16, cache_path: str | None = None,
             refresh: bool = False, log=None) -> dict:
    """Tune pr_dfp for one batch update."""
    import torch
    out = torch.empty(g_new.n, dtype=torch.float64, device=g_new.in_offsets.device)

    def run(k):
        prhip.dfp(g_new, batch, ranks_prev, max_iter=k, out=out)

    return _cached("dfp", g_new.n, g_new.m,
                   lambda: coordinate_descent(run, DFP_SPACE, k1=2, k2=5,
                                              expected_iters=expected_iters, log=log),
                   cache_path, refresh)
