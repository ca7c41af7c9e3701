#!/usr/bin/env python3
"""Benchmark of the PageRank hot path on one MI355X.

Headline workload (synthetic, seeded): R-MAT scale 24 (a, b, c, d = 0.57,
0.19, 0.19, 0.05), edge factor 16, seed 1, Graph500-style scrambled IDs,
duplicates removed, one self-loop per vertex, int32 CSR, FP64 ranks,
alpha 0.85, tol 1e-10 (L-infinity), at most 500 iterations. Random batch
updates of 1e-7 .. 1e-3 |E| (one per decade, batch seed = decade index + 1),
80 % insertions of absent pairs, 20 % deletions of existing non-self-loop
edges; R^{t-1} is the Static result on G^{t-1}.

One step runs every part of the path once:
  static   pr_static on G^t                         (scale 24)
  dfp      pr_dfp(G^t, batch, R^{t-1})               (scale 24; decades cycle over steps)
  ppr      pr_ppr, 64 teleport vectors of 16 seeds   (R-MAT scale 20, edge factor 16)
  batched  pr_static_batched on 256 R-MAT graphs, n log-uniform in [2^10, 2^20],
           edge factor uniform in [4, 32], seeds 1000 + i
  adjoint  pr_weighted + pr_adjoint, weights U(0.1, 1] row-normalised, loss = sum of
           squared ranks of 1024 random targets      (R-MAT scale 20, edge factor 16)
After the timed steps (a chain, so not part of a step), unless --temporal-batches 0:
  temporal preferential-attachment stream, 2M vertices, 40M events: 90 % loaded, the
           rest in 100 batches (10 % deletions); DF-P chained batch to batch, beside
           pr_static on every G^t, errors against a tight Static every 10th batch.
Also untimed (unless --no-compare): ND, DT and DF beside DF-P on the same batches;
  pr_apply_batch per batch; an ablation of the rank kernel; and a sweep of
  --sweep-batches random batches per decade (seeds 1..5 by default), each G^t built
  on the device, DF-P against Static summarised by geometric means per decade.
Inputs are resident in HBM before the timed region. `value` is the Static
GTEPS per iteration (m * iterations / call time). Prints one JSON line on
stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time
import warnings

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS & HBM GB/s per iteration; ms per batch update, DF-P vs Static"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rank_static_rmat24.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2404_08299_amd", "csrc", f)
                  for f in ("kernels.h", "wave.h")]
PPR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ppr_rmat20_k64.txt")
PPR_SOURCES = [os.path.join(ROOT, "paper_2404_08299_amd", "csrc", f)
               for f in ("ppr.h", "kernels.h", "wave.h")]
ALL_LEGS = ("static", "dfp", "ppr", "batched", "adjoint")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(sources=None):
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n, m):
    """Compulsory bytes of one Static rank update: 4(n+1) in_offsets + 4m
    in_sources + 8n ranks gathered once + 4n out-degrees + 8n new ranks
    written + 4n vertex permutation, i.e. 4m + 28n."""
    return 4 * m + 28 * n


def read_traffic(path=None, sources=None):
    """Measured HBM bytes per launch from a committed rocprofv3 PMC summary
    (default: the Static rank kernel's), if it was taken on the current
    kernel source (else None)."""
    path = path or TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sha256") != kernel_hash(sources):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def ppr_algorithmic_bytes(n, m, k):
    """Compulsory bytes of one personalised-PageRank launch over k active
    vectors: 4m in_sources + 8kn contributions gathered once + 8kn new ranks
    written (the teleport rows are sparse and the offsets negligible)."""
    return 4 * m + 16 * k * n


def cpu_info():
    """Host CPU model, logical CPUs and the CPUs this process may run on."""
    model, mhz = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if model is None and line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
            if mhz is None and line.startswith("cpu MHz"):
                mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return {"cpu_model": model, "cpu_mhz": mhz, "nproc": os.cpu_count(), "affinity_cpus": aff}


def size_sweep(gg, prhip, torch, np, scales=(18, 20, 22, 23, 24), calls=3):
    """Static on R-MAT (edge factor 16, seed 1) at several sizes with the
    lane-class bound (32, 128) and the die split (off, on) crossed: which
    defaults hold at which size. One JSON object per case on stdout."""
    for sc in scales:
        g = gg.rmat_graph(sc, 16, seed=1)
        dg = prhip.DeviceGraph.from_host(g)
        del g
        out = torch.empty(dg.n, dtype=torch.float64, device="cuda")
        for lane in (32, 128):
            for xs in (0, 129):
                prhip.set_tuning(lane_max_degree=lane, xcd_split_degree=xs)
                prhip.static(dg, out=out)
                ts = [timed(lambda: prhip.static(dg, out=out))[1] for _ in range(calls)]
                it = prhip.last_stats()["iterations"]
                med = float(np.median(ts))
                print(json.dumps({"scale": sc, "n": dg.n, "m": dg.m, "lane_max_degree": lane,
                                  "xcd_split_degree": xs, "ms_per_call": round(med, 3),
                                  "iterations": it,
                                  "us_per_iteration": round(med * 1e3 / it, 1)}), flush=True)
        prhip.set_tuning()
        del dg, out
        torch.cuda.empty_cache()


def copy_probe(gib=1.0, reps=5):
    """A plain device copy of known size (torch's copy kernel), for
    calibrating the PMC byte counters and as a measured copy ceiling."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    gbs = 2 * n * 8 / dt / 1e9
    log(f"copy probe: {n * 8} bytes read + written per copy, {dt * 1e3:.3f} ms, {gbs:.0f} GB/s")
    return gbs


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) * 1e3


def temporal_leg(args, gg, prhip, torch, np):
    """DF-P chained over the batches of a preferential-attachment temporal
    stream, beside Static on every G^t (each call timed alone, inputs resident
    in HBM). Errors against a Static run at tol 0 every 10th batch."""
    t = time.time()
    g0, steps = gg.temporal_stream(args.temporal_n, args.temporal_events, seed=1,
                                   batches=args.temporal_batches)
    dgs, dbs, sizes = [], [], []
    for b, g in steps:
        dgs.append(prhip.DeviceGraph.from_host(g))
        dbs.append(prhip.DeviceBatch.from_host(b))
        sizes.append((int(b.ins_src.size), int(b.del_src.size)))
    log(f"temporal: n={g0.n} m0={g0.m} m_end={dgs[-1].m}, {len(dgs)} batches "
        f"({time.time() - t:.1f} s)")
    prev = prhip.static(prhip.DeviceGraph.from_host(g0)).ranks
    g0_ranks = prev.clone()
    prev_df = prev.clone()
    abl_cases = []
    outs = [torch.empty(g0.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    outs_df = [torch.empty(g0.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    st_out = torch.empty(g0.n, dtype=torch.float64, device="cuda")
    ref = torch.empty(g0.n, dtype=torch.float64, device="cuda")
    dfp_ms, df_ms, st_ms, dfp_it, df_it, st_it, errs = [], [], [], [], [], [], []
    refs = {}
    for k, (dg, db) in enumerate(zip(dgs, dbs)):
        # DF-P and DF (no pruning, the paper's accuracy fallback) each chained
        # over the stream, and Static on G^t
        out, out_df = outs[k & 1], outs_df[k & 1]
        if k < args.ablation_batches:
            abl_cases.append((dg, db, prev.clone()))
        _, ms_d = timed(lambda: prhip.dfp(dg, db, prev, out=out))
        dfp_it.append(prhip.last_stats()["iterations"])
        _, ms_f = timed(lambda: prhip.dfp(dg, db, prev_df, mode="df", out=out_df))
        df_it.append(prhip.last_stats()["iterations"])
        _, ms_s = timed(lambda: prhip.static(dg, out=st_out))
        st_it.append(prhip.last_stats()["iterations"])
        dfp_ms.append(ms_d)
        df_ms.append(ms_f)
        st_ms.append(ms_s)
        prev, prev_df = out, out_df
        if k % 10 == 9 or k == len(dgs) - 1:
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                prhip.static(dg, tol=0.0, max_iter=500, out=ref)
            refs[k] = ref.clone()
            d = (out - ref).abs()
            d_df = (out_df - ref).abs()
            errs.append({"batch": k + 1, "dfp_linf": float(d.max()), "dfp_l1": float(d.sum()),
                         "df_linf": float(d_df.max()), "df_l1": float(d_df.sum()),
                         "static_linf": float((st_out - ref).abs().max()),
                         "max_rank": float(ref.max())})
    gm = lambda a: float(np.exp(np.mean(np.log(a))))
    res = {"workload": f"pa_temporal_n{args.temporal_n}_ev{args.temporal_events}"
                       f"_b{args.temporal_batches}",
           "n": g0.n, "m0": g0.m, "m_end": dgs[-1].m,
           "mean_insertions": round(float(np.mean([a for a, _ in sizes])), 1),
           "deletions_per_batch": sizes[0][1],
           "dfp_ms_geomean": round(gm(dfp_ms), 3), "static_ms_geomean": round(gm(st_ms), 3),
           "dfp_speedup_geomean": round(gm(np.array(st_ms) / np.array(dfp_ms)), 2),
           "dfp_iters_mean": round(float(np.mean(dfp_it)), 2),
           "df_ms_geomean": round(gm(df_ms), 3),
           "df_speedup_geomean": round(gm(np.array(st_ms) / np.array(df_ms)), 2),
           "df_iters_mean": round(float(np.mean(df_it)), 2),
           "max_dfp_linf": max(e["dfp_linf"] for e in errs),
           "max_df_linf": max(e["df_linf"] for e in errs), "errors": errs}
    log(f"temporal: DF-P {res['dfp_ms_geomean']} ms, DF {res['df_ms_geomean']} ms vs Static "
        f"{res['static_ms_geomean']} ms per batch (geomean), max L-inf DF-P "
        f"{res['max_dfp_linf']:.2e}, DF {res['max_df_linf']:.2e}")
    # DF-P chained again with tighter frontier and prune tolerances (the
    # paper's are 1e-6 each): what the speedup costs in accuracy on this
    # stream, errors against the same reference runs
    sweep = []
    for tl in (1e-7, 1e-8):
        p, t_ms, e_max = g0_ranks.clone(), [], 0.0
        for k, (dg, db) in enumerate(zip(dgs, dbs)):
            out = outs[k & 1]
            t_ms.append(timed(lambda: prhip.dfp(dg, db, p, frontier_tol=tl, prune_tol=tl,
                                                out=out))[1])
            p = out
            if k in refs:
                e_max = max(e_max, float((out - refs[k]).abs().max()))
        sweep.append({"frontier_tol": tl, "prune_tol": tl, "dfp_ms_geomean": round(gm(t_ms), 3),
                      "dfp_speedup_geomean": round(gm(np.array(st_ms) / np.array(t_ms)), 2),
                      "max_dfp_linf": e_max})
    res["tolerance_sweep"] = sweep
    log("temporal tolerance sweep: " + ", ".join(
        f"{e['prune_tol']:g}: {e['dfp_ms_geomean']} ms ({e['dfp_speedup_geomean']}x), "
        f"L-inf {e['max_dfp_linf']:.2e}" for e in sweep))
    if not args.no_tune:
        # the same chain with the autotuner's choices for this graph size
        # (untimed tuning: DF-P on the first batch, Static on G^0), DF taking
        # DF-P's; the defaults were chosen at scale 24
        from paper_2404_08299_amd import autotune
        t = time.time()
        prev0 = prhip.static(prhip.DeviceGraph.from_host(g0)).ranks
        with tempfile.TemporaryDirectory() as td:
            cache = os.path.join(td, "tuning.json")
            tn_st = autotune.tune_static(dgs[0], expected_iters=int(np.median(st_it)),
                                         cache_path=cache)
            tn_dy = autotune.tune_dfp(dgs[0], dbs[0], prev0,
                                      expected_iters=int(np.median(dfp_it)), cache_path=cache)
        prhip.set_tuning()
        defaults = prhip.get_tuning()
        log(f"temporal autotune ({time.time() - t:.1f} s): Static {tn_st}, DF-P {tn_dy}")
        prev, prev_df = prev0, prev0.clone()
        t_dfp, t_df, t_st = [], [], []
        for k, (dg, db) in enumerate(zip(dgs, dbs)):
            out, out_df = outs[k & 1], outs_df[k & 1]
            prhip.set_tuning(**tn_dy)
            t_dfp.append(timed(lambda: prhip.dfp(dg, db, prev, out=out))[1])
            t_df.append(timed(lambda: prhip.dfp(dg, db, prev_df, mode="df", out=out_df))[1])
            prhip.set_tuning(**tn_st)
            t_st.append(timed(lambda: prhip.static(dg, out=st_out))[1])
            prev, prev_df = out, out_df
        prhip.set_tuning()
        res["tuned"] = {
            "dfp_tuning": {k: v for k, v in tn_dy.items() if v != defaults[k]},
            "static_tuning": {k: v for k, v in tn_st.items() if v != defaults[k]},
            "dfp_ms_geomean": round(gm(t_dfp), 3), "df_ms_geomean": round(gm(t_df), 3),
            "static_ms_geomean": round(gm(t_st), 3),
            "dfp_speedup_geomean": round(gm(np.array(t_st) / np.array(t_dfp)), 2),
            "df_speedup_geomean": round(gm(np.array(t_st) / np.array(t_df)), 2)}
        log(f"temporal tuned: {res['tuned']}")
    if abl_cases and not args.no_compare:
        # Sec. 4.4's partitioning study on the first batches of the stream,
        # each from the DF-P chain's R^{t-1}
        abl = partition_ablation(prhip, torch, abl_cases)
        res["partition_ablation"] = {
            "batches": len(abl_cases),
            **{k: {"ms_geomean": round(gm(v["ms"]), 3), "iters_mean":
                   round(float(np.mean(v["iters"])), 2), "linf_vs_default": v["linf_vs_default"]}
               for k, v in abl.items()}}
        log(f"temporal partition ablation: "
            + ", ".join(f"{k} {v['ms_geomean']} ms" for k, v in res["partition_ablation"].items()
                        if isinstance(v, dict)))
    return res


# The partitioning study of Sec. 4.4 for DF and DF-P: no partitioning (one
# lane per vertex in the rank update and in expandAffected), partitioning of
# G' only (the rank update's in-degree classes; marking one lane per vertex),
# and partitioning of both G' and G (the default: in-degree classes for the
# rank update, out-degree classes for the marking).
PARTITION_STRATEGIES = {
    "none": dict(lane_max_degree=1 << 30, wave_max_degree=1 << 30,
                 expand_lane_max_degree=1 << 30, xcd_split_degree=0),
    "in_only": dict(wave_max_degree=1 << 30, expand_lane_max_degree=1 << 30),
    "in_and_out": {},
}


def partition_ablation(prhip, torch, cases):
    """DF-P and DF under each partitioning strategy on `cases`, a list of
    (G^t, batch, R^{t-1}): one untimed and one timed call each. Returns per
    strategy and mode the times (ms), the iteration counts and the largest
    L-infinity distance to the default strategy's ranks (the strategies
    change only the order of floating-point summation)."""
    n = cases[0][0].n
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ref = {}
    res = {}
    for name in ("in_and_out", "in_only", "none"):
        prhip.set_tuning()
        prhip.set_tuning(**PARTITION_STRATEGIES[name])
        for mode in ("dfp", "df"):
            ms, its, dev = [], [], 0.0
            for i, (dg, db, prev) in enumerate(cases):
                prhip.dfp(dg, db, prev, mode=mode, out=out)
                _, t = timed(lambda: prhip.dfp(dg, db, prev, mode=mode, out=out))
                ms.append(round(t, 3))
                its.append(prhip.last_stats()["iterations"])
                if name == "in_and_out":
                    ref[(mode, i)] = out.clone()
                else:
                    dev = max(dev, float((out - ref[(mode, i)]).abs().max()))
            res[f"{mode}_{name}"] = {"ms": ms, "iters": its, "linf_vs_default": dev}
    prhip.set_tuning()
    return res


def small_leg(gg, prhip, torch, np, calls=30, tune=True):
    """The small configuration: R-MAT scale 14, edge factor 8, seed 1, Static
    at tol 1e-10. About 1 MB of data per iteration, resident in L2: a latency
    figure (microseconds per iteration), not a bandwidth one. Each iteration
    launches three kernels (rank update, long-row finalize, L-infinity final)
    and copies the 64-byte control block to the host."""
    g = gg.rmat_graph(14, 8, seed=1)
    dg = prhip.DeviceGraph.from_host(g)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")

    def measure():
        for _ in range(3):
            prhip.static(dg, out=out)
        times = []
        for _ in range(calls):
            _, ms = timed(lambda: prhip.static(dg, out=out))
            times.append(ms)
        iters = prhip.last_stats()["iterations"]
        prhip.set_profiling(True, counters=False)
        prhip.static(dg, out=out)
        st = prhip.last_stats()
        prhip.set_profiling(False)
        med = float(np.median(times))
        return {"iters": iters, "calls": calls,
                "call_us_median": round(med * 1e3, 1), "call_us_min": round(min(times) * 1e3, 1),
                "us_per_iteration": round(med * 1e3 / iters, 2),
                "gteps_per_iteration": round(g.m * iters / (med / 1e3) / 1e9, 3),
                "rank_kernel_us": round(st["rank_kernel_ms"] / st["rank_kernel_launches"] * 1e3, 2),
                "device_us_per_call": round(st["total_ms"] * 1e3, 1)}

    res = {"workload": "rmat14_ef8_static", "n": g.n, "m": g.m}
    res.update(measure())
    res.update(launches_per_iteration=3, host_copies_per_iteration=1)
    if tune:
        # the autotuner on this graph (untimed): the defaults were chosen at
        # scale 24, where the LDS-staged lane class pays; on a graph this
        # small its few tiles leave most of the chip idle
        from paper_2404_08299_amd import autotune
        with tempfile.TemporaryDirectory() as td:
            best = autotune.tune_static(dg, expected_iters=res["iters"],
                                        cache_path=os.path.join(td, "tuning.json"))
        tuned = measure()
        prhip.set_tuning()
        tuned["tuning"] = {k: v for k, v in best.items() if v != prhip.get_tuning()[k]}
        res["tuned"] = tuned
    log(f"small graph: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=float, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--fractions", default="1e-7,1e-6,1e-5,1e-4,1e-3")
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="comma-separated subset of " + ",".join(ALL_LEGS))
    ap.add_argument("--aux-scale", type=int, default=20, help="scale of the PPR/adjoint graph")
    ap.add_argument("--ppr-k", type=int, default=64)
    ap.add_argument("--batch-graphs", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="run the batched leg at the default tuning instead of autotuning it")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the untimed comparison runs (single calls vs batched)")
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--sweep-batches", type=int, default=5,
                    help="batches per decade (seeds 1..N) in the untimed DF-P vs Static sweep; "
                         "0 skips it")
    ap.add_argument("--temporal-batches", type=int, default=100)
    ap.add_argument("--ablation-batches", type=int, default=10,
                    help="temporal batches in the partitioning study (Sec. 4.4)")
    ap.add_argument("--temporal-n", type=int, default=2_000_000)
    ap.add_argument("--temporal-events", type=int, default=40_000_000)
    ap.add_argument("--order", default="scrambled", choices=["scrambled", "natural", "degree"],
                    help="vertex numbering of the input: Graph500 scrambled IDs, R-MAT's own "
                         "IDs, or relabelled by descending out-degree")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the calibration copy kernel")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only run Static over R-MAT scales 18-24, lane bound and die split "
                         "crossed")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the path runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2404_08299_amd import graphgen as gg
    from paper_2404_08299_amd import prhip

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    prhip.load_library()
    if args.copy_probe:
        copy_probe()
        return
    if args.size_sweep:
        size_sweep(gg, prhip, torch, np)
        return
    legs = [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in ALL_LEGS:
            raise SystemExit(f"unknown leg {x}")
    if "dfp" in legs and "static" not in legs:
        legs.insert(0, "static")

    # ------------------------------------------------------------ inputs
    fracs = [float(x) for x in args.fractions.split(",")]
    t = time.time()
    g0 = gg.rmat_graph(args.scale, args.edge_factor, seed=args.seed,
                       scramble=(args.order == "scrambled"))
    if args.order == "degree":
        g0 = gg.relabel(g0, gg.degree_order(g0, "out"))
    n = g0.n
    log(f"R-MAT scale {args.scale}: n={n} m={g0.m} ({time.time() - t:.1f} s)")
    dg0 = prhip.DeviceGraph.from_host(g0)
    dgs, dbs, sizes, ms = [], [], [], []
    for j, f in enumerate(fracs):
        t = time.time()
        b = gg.random_batch(g0, gg.batch_size_for(g0, f), seed=j + 1)
        g1 = gg.apply_batch(g0, b)
        dgs.append(prhip.DeviceGraph.from_host(g1))
        dbs.append(prhip.DeviceBatch.from_host(b))
        sizes.append(b.size)
        ms.append(g1.m)
        del g1
        log(f"batch {f:g}|E|: {b.size} updates ({b.ins_src.size} ins, {b.del_src.size} del), "
            f"m={ms[-1]} ({time.time() - t:.1f} s)")

    aux = {}
    if "ppr" in legs or "adjoint" in legs:
        t = time.time()
        ga = gg.rmat_graph(args.aux_scale, 16, seed=1)
        aux["g"] = ga
        aux["dg"] = prhip.DeviceGraph.from_host(ga)
        if "ppr" in legs:
            sets = gg.distinct_vertices(ga.n, args.ppr_k, 16, seed=2)
            T = np.zeros((ga.n, args.ppr_k))
            for j in range(args.ppr_k):
                T[sets[j], j] = 1.0 / 16
            aux["tele"] = torch.from_numpy(T).cuda()
            aux["ppr_out"] = torch.empty((ga.n, args.ppr_k), dtype=torch.float64, device="cuda")
        if "adjoint" in legs:
            dst = np.repeat(np.arange(ga.n, dtype=np.int32), ga.in_degree())
            src = ga.in_sources
            w = gg.edge_weights(src, dst, seed=1)
            W = np.bincount(src, weights=w, minlength=ga.n)
            aux["P"] = torch.from_numpy(w / W[src]).cuda()
            aux["s"] = torch.full((ga.n,), 1.0 / ga.n, dtype=torch.float64, device="cuda")
            tg = np.random.default_rng(2).choice(ga.n, 1024, replace=False)
            aux["targets"] = torch.from_numpy(tg).cuda()
            aux["fw_out"] = torch.empty(ga.n, dtype=torch.float64, device="cuda")
        log(f"R-MAT scale {args.aux_scale}: n={ga.n} m={ga.m} ({time.time() - t:.1f} s)")
    if "batched" in legs:
        t = time.time()
        rng = np.random.default_rng(7)
        bgs = []
        for i in range(args.batch_graphs):
            nb = int(2 ** rng.uniform(10, 20))
            ef = float(rng.uniform(4, 32))
            sc = int(np.ceil(np.log2(nb)))
            bgs.append(prhip.DeviceGraph.from_host(
                gg.rmat_graph(sc, ef * nb / (1 << sc), seed=1000 + i, n=nb)))
        aux["bgs"] = bgs
        aux["bouts"] = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in bgs]
        log(f"{len(bgs)} batched graphs: N={sum(g.n for g in bgs)} M={sum(g.m for g in bgs)} "
            f"({time.time() - t:.1f} s)")
        aux["btune"] = {}
        if not args.no_tune:
            # degree-bucket thresholds of the batched call picked by the autotuner
            # (coordinate descent, each candidate timed at two iteration caps)
            import tempfile
            from paper_2404_08299_amd import autotune
            t = time.time()
            with tempfile.TemporaryDirectory() as td:
                aux["btune"] = autotune.tune_batched(bgs, expected_iters=80, refresh=True,
                                                     cache_path=os.path.join(td, "tuning.json"))
            prhip.set_tuning()
            log(f"batched autotune: {aux['btune']} ({time.time() - t:.1f} s)")
    torch.cuda.synchronize()

    # R^{t-1}: Static on G^{t-1} (untimed)
    prev = prhip.static(dg0).ranks
    log(f"R^(t-1): {prhip.last_stats()['iterations']} iterations")
    static_out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in fracs]
    dfp_out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in fracs]
    rec = {j: {"static_ms": [], "dfp_ms": [], "static_iters": [], "dfp_iters": [],
               "rank_ms": [], "rank_launches": []} for j in range(len(fracs))}
    other = {"ppr_ms": [], "ppr_iters": [], "ppr_vec_iters": [], "ppr_rank_ms": [],
             "ppr_launches": [], "batched_ms": [], "batched_iters": [],
             "fw_ms": [], "fw_iters": [], "adj_ms": [], "adj_iters": []}

    def step(s, record):
        j = s % len(fracs)
        # recorded steps: HIP events around every call and every rank-kernel
        # launch (the live roofline figures), for every leg alike; no
        # affected-set counting passes
        prhip.set_profiling(record, counters=False)
        if "static" in legs:
            t0 = time.perf_counter()
            prhip.static(dgs[j], out=static_out[j])
            t1 = time.perf_counter()
            st = prhip.last_stats()
            if record:
                r = rec[j]
                r["static_ms"].append((t1 - t0) * 1e3)
                r["static_iters"].append(st["iterations"])
                r["rank_ms"].append(st["rank_kernel_ms"])
                r["rank_launches"].append(st["rank_kernel_launches"])
        if "dfp" in legs:
            t1 = time.perf_counter()
            prhip.dfp(dgs[j], dbs[j], prev, out=dfp_out[j])
            t2 = time.perf_counter()
            if record:
                rec[j]["dfp_ms"].append((t2 - t1) * 1e3)
                rec[j]["dfp_iters"].append(prhip.last_stats()["iterations"])
        if "ppr" in legs:
            t0 = time.perf_counter()
            _, its = prhip.ppr(aux["dg"], aux["tele"], out=aux["ppr_out"])
            t1 = time.perf_counter()
            if record:
                st = prhip.last_stats()
                other["ppr_ms"].append((t1 - t0) * 1e3)
                other["ppr_iters"].append(int(its.max()))
                other["ppr_vec_iters"].append(int(its.sum()))
                other["ppr_rank_ms"].append(st["rank_kernel_ms"])
                other["ppr_launches"].append(st["rank_kernel_launches"])
        if "batched" in legs:
            prhip.set_tuning(**aux["btune"])
            t0 = time.perf_counter()
            _, its = prhip.static_batched(aux["bgs"], outs=aux["bouts"])
            t1 = time.perf_counter()
            prhip.set_tuning()
            if record:
                other["batched_ms"].append((t1 - t0) * 1e3)
                other["batched_iters"].append(int(its.max()))
        if "adjoint" in legs:
            t0 = time.perf_counter()
            fr = prhip.weighted(aux["dg"], aux["P"], aux["s"], out=aux["fw_out"])
            t1 = time.perf_counter()
            grad = torch.zeros_like(fr.ranks)
            grad[aux["targets"]] = 2 * fr.ranks[aux["targets"]]
            t2 = time.perf_counter()
            prhip.adjoint(aux["dg"], aux["P"], fr.ranks, grad)
            t3 = time.perf_counter()
            if record:
                other["fw_ms"].append((t1 - t0) * 1e3)
                other["fw_iters"].append(fr.iterations)
                other["adj_ms"].append((t3 - t2) * 1e3)
                other["adj_iters"].append(prhip.last_stats()["iterations"])
        prhip.set_profiling(False)

    for s in range(args.warmup):
        step(s, False)
    log(f"warmup {args.warmup} steps done")
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    for s in range(args.steps):
        step(args.warmup + s, True)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    ms_per_step = (T1 - T0) / args.steps * 1e3
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    out = {"metric": METRIC, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "value": None}
    out["config"] = {"workload": f"rmat{args.scale}_ef{int(args.edge_factor)}_static_and_dfp",
                     "vertex_order": args.order, "n": n, "m": g0.m, "scale": args.scale,
                     "edge_factor": args.edge_factor, "seed": args.seed,
                     "batch_fractions": fracs, "alpha": 0.85, "tol": 1e-10,
                     "frontier_tol": 1e-6, "prune_tol": 1e-6, "max_iter": 500, "legs": legs,
                     "tuning": prhip.get_tuning()}

    if "static" in legs:
        edges_iter = bytes_iter = t_static = rank_ms = rank_bytes = 0.0
        launches = 0
        per_batch = []
        for j, f in enumerate(fracs):
            r = rec[j]
            if not r["static_ms"]:
                continue
            for k in range(len(r["static_ms"])):
                edges_iter += ms[j] * r["static_iters"][k]
                bytes_iter += algorithmic_bytes(n, ms[j]) * r["static_iters"][k]
                t_static += r["static_ms"][k] / 1e3
                rank_ms += r["rank_ms"][k]
                rank_bytes += algorithmic_bytes(n, ms[j]) * r["rank_launches"][k]
                launches += r["rank_launches"][k]
            item = {"fraction": f, "batch_size": sizes[j],
                    "static_ms": round(float(np.mean(r["static_ms"])), 3),
                    "static_iters": r["static_iters"][0]}
            if r["dfp_ms"]:
                dm = float(np.mean(r["dfp_ms"]))
                item.update(dfp_ms=round(dm, 3), dfp_iters=r["dfp_iters"][0],
                            dfp_speedup=round(item["static_ms"] / dm, 2))
            per_batch.append(item)
        gteps = edges_iter / t_static / 1e9
        gbs = bytes_iter / t_static / 1e9
        avg_rank_ms = rank_ms / max(1, launches)
        achieved = rank_bytes / (rank_ms / 1e3) / 1e9 if rank_ms > 0 else None
        log(f"Static {gteps:.2f} GTEPS, {gbs:.0f} GB/s algorithmic (whole call); rank kernel "
            f"{avg_rank_ms * 1e3:.1f} us avg over {launches} launches, {achieved:.0f} GB/s")
        out["value"] = round(gteps, 3)
        out["static_gbs_per_iteration"] = round(gbs, 1)
        out["batches"] = per_batch
        out["rank_gteps"] = round(g0.m / (avg_rank_ms / 1e3) / 1e9, 2)
        out["paper_style_medges_per_s"] = round(
            float(np.mean([ms[j] / (np.mean(rec[j]["static_ms"]) / 1e3) / 1e6
                           for j in range(len(fracs)) if rec[j]["static_ms"]])), 1)
        out["roofline"] = {"bound": "hbm", "kernel": "k_rank_static",
                           "achieved": round(achieved, 1) if achieved else None,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                           "traffic": read_traffic(),
                           "traffic_kind": "L2-to-fabric bytes per launch (rocprofv3 FETCH_SIZE + "
                                           "WRITE_SIZE, copy-calibrated; Infinity Cache hits "
                                           "included, not DRAM-only)",
                           "avg_launch_us": round(avg_rank_ms * 1e3, 2),
                           "algorithmic_bytes_per_launch": algorithmic_bytes(n, g0.m)}

    if "ppr" in legs:
        ga = aux["g"]
        pm = float(np.mean(other["ppr_ms"]))
        out["ppr"] = {"workload": f"rmat{args.aux_scale}_ef16_k{args.ppr_k}", "n": ga.n,
                      "m": ga.m, "k": args.ppr_k, "ms": round(pm, 3),
                      "iters": other["ppr_iters"][0],
                      "vector_gteps": round(ga.m * args.ppr_k * other["ppr_iters"][0] / pm / 1e6, 2)}
        # roofline of k_ppr_rank: a launch over k active vectors moves
        # 4m + 16kn algorithmic bytes; a vector that met the tolerance is
        # frozen (its lanes neither read nor write), so over a call the bytes
        # are launches * 4m + 16n * (sum of the vectors' iteration counts)
        p_launch = sum(other["ppr_launches"])
        p_ms = sum(other["ppr_rank_ms"])
        p_bytes = sum(L * 4 * ga.m + 16 * ga.n * vi
                      for L, vi in zip(other["ppr_launches"], other["ppr_vec_iters"]))
        if p_ms > 0 and p_launch > 0:
            p_ach = p_bytes / (p_ms / 1e3) / 1e9
            p_traffic = read_traffic(PPR_TRAFFIC_FILE, PPR_SOURCES)
            p_alg_full = ppr_algorithmic_bytes(ga.n, ga.m, args.ppr_k)
            out["ppr"]["roofline"] = {
                "bound": "hbm", "kernel": "k_ppr_rank", "achieved": round(p_ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(p_ach / HBM_PEAK_GBS, 4),
                "traffic": p_traffic,
                "traffic_over_algorithmic": round(p_traffic / p_alg_full, 2) if p_traffic else None,
                "avg_launch_us": round(p_ms / p_launch * 1e3, 2),
                "algorithmic_bytes_per_launch_all_active": p_alg_full,
                "algorithmic_bytes_per_launch_mean": round(p_bytes / p_launch)}
    if "batched" in legs:
        bm = float(np.mean(other["batched_ms"]))
        out["batched"] = {"graphs": len(aux["bgs"]), "n": sum(g.n for g in aux["bgs"]),
                          "m": sum(g.m for g in aux["bgs"]), "ms": round(bm, 3),
                          "max_iters": other["batched_iters"][0],
                          "tuning": aux["btune"] or "default"}
    if "adjoint" in legs:
        out["adjoint"] = {"workload": f"weighted_rmat{args.aux_scale}_ef16_1024_targets",
                          "forward_ms": round(float(np.mean(other["fw_ms"])), 3),
                          "forward_iters": other["fw_iters"][0],
                          "adjoint_ms": round(float(np.mean(other["adj_ms"])), 3),
                          "adjoint_iters": other["adj_iters"][0]}

    # ------------------------------------------------------------ untimed comparisons
    if not args.no_compare:
        if "batched" in legs:
            # the plain per-graph forward: pr_static on each graph, default tuning
            _, t_single = timed(lambda: [prhip.static(g) for g in aux["bgs"]])
            # at the batched call's tuning, single calls give the same bits
            prhip.set_tuning(**aux["btune"])
            ref, _ = prhip.static_batched(aux["bgs"], outs=aux["bouts"])
            same = all(torch.equal(prhip.static(g).ranks, r)
                       for g, r in zip(aux["bgs"][:8], ref.ranks[:8]))
            prhip.set_tuning()
            out["batched"].update(sum_of_single_calls_ms=round(t_single, 3),
                                  speedup=round(t_single / out["batched"]["ms"], 2),
                                  bitwise_equal_to_single_calls=same)
        if "ppr" in legs:
            _, t_single = timed(lambda: [prhip.static(aux["dg"]) for _ in range(args.ppr_k)])
            out["ppr"].update(k_static_solves_ms=round(t_single, 3),
                              speedup_vs_k_static=round(t_single / out["ppr"]["ms"], 2))
        log(f"comparisons: batched {out.get('batched')}, ppr {out.get('ppr')}")

    if not args.no_compare and "dfp" in legs:
        # the paper's method comparison on the same batches (one timed call
        # each after a warm-up call): Naive-dynamic, Dynamic Traversal,
        # Dynamic Frontier without pruning
        tmp = torch.empty(n, dtype=torch.float64, device="cuda")
        modes = []
        for j, f in enumerate(fracs):
            item = {"fraction": f}
            for mode in ("nd", "dt", "df"):
                prhip.dfp(dgs[j], dbs[j], prev, mode=mode, out=tmp)
                _, t_mode = timed(lambda: prhip.dfp(dgs[j], dbs[j], prev, mode=mode, out=tmp))
                item[f"{mode}_ms"] = round(t_mode, 3)
                item[f"{mode}_iters"] = prhip.last_stats()["iterations"]
            # DF-P with the ID-tile sweeps instead of the compacted affected list
            prhip.set_tuning(frontier_list=0)
            prhip.dfp(dgs[j], dbs[j], prev, out=tmp)
            _, t_sw = timed(lambda: prhip.dfp(dgs[j], dbs[j], prev, out=tmp))
            prhip.set_tuning()
            item["dfp_sweep_ms"] = round(t_sw, 3)
            # the batch applied on the device (pr_apply_batch: both views of G^t from G^{t-1})
            prhip.apply_batch(dg0, dbs[j])
            _, t_apply = timed(lambda: prhip.apply_batch(dg0, dbs[j]))
            item["apply_batch_ms"] = round(t_apply, 3)
            dm = float(np.mean(rec[j]["dfp_ms"])) if rec[j]["dfp_ms"] else None
            if dm:
                for mode in ("nd", "dt", "df"):
                    item[f"dfp_speedup_vs_{mode}"] = round(item[f"{mode}_ms"] / dm, 2)
            modes.append(item)
        out["dynamic_methods"] = modes
        log(f"methods: {modes}")

    if not args.no_compare and "dfp" in legs:
        # Sec. 4.4's partitioning study for DF and DF-P, one batch per decade
        # (the timed steps' batches, from R^{t-1} = Static on G^{t-1})
        abl = partition_ablation(prhip, torch, [(dgs[j], dbs[j], prev) for j in range(len(fracs))])
        out["partition_ablation"] = {
            "strategies": PARTITION_STRATEGIES,
            "decades": [{"fraction": f, **{k: {"ms": v["ms"][j], "iters": v["iters"][j]}
                                           for k, v in abl.items()}}
                        for j, f in enumerate(fracs)],
            "linf_vs_default": {k: v["linf_vs_default"] for k, v in abl.items()}}
        log("partition ablation (ms per call, DF-P: none / G' / G' and G): "
            + ", ".join(f"{f:g}: {abl['dfp_none']['ms'][j]} / {abl['dfp_in_only']['ms'][j]} / "
                        f"{abl['dfp_in_and_out']['ms'][j]}" for j, f in enumerate(fracs)))

    if not args.no_compare and "dfp" in legs and args.sweep_batches > 0:
        # DF-P against Static over several random batches per decade (batch
        # seeds 1 .. sweep_batches): each G^t is built on the device from
        # G^{t-1} (pr_apply_batch), both methods run once untimed and once
        # timed, and each decade is summarised by geometric means
        t = time.time()
        tmp_s = torch.empty(n, dtype=torch.float64, device="cuda")
        tmp_d = torch.empty(n, dtype=torch.float64, device="cuda")

        def gmean(x):
            return float(np.exp(np.mean(np.log(x))))

        sweep = []
        for f in fracs:
            sm, dm, sp, its, err = [], [], [], [], 0.0
            a0, amax, edges, work = [], [], [], []
            for seed in range(1, args.sweep_batches + 1):
                db = prhip.DeviceBatch.from_host(
                    gg.random_batch(g0, gg.batch_size_for(g0, f), seed=seed))
                dgt = prhip.apply_batch(dg0, db)
                prhip.static(dgt, out=tmp_s)
                prhip.dfp(dgt, db, prev, out=tmp_d)
                _, ts = timed(lambda: prhip.static(dgt, out=tmp_s))
                static_iters = prhip.last_stats()["iterations"]
                _, td = timed(lambda: prhip.dfp(dgt, db, prev, out=tmp_d))
                its.append(prhip.last_stats()["iterations"])
                err = max(err, float((tmp_d - tmp_s).abs().max()))
                sm.append(ts)
                dm.append(td)
                sp.append(ts / td)
                # the affected-set counters, from one more (untimed) call
                prhip.set_profiling(True)
                prhip.dfp(dgt, db, prev, out=tmp_d)
                st = prhip.last_stats()
                prhip.set_profiling(False)
                a0.append(st["affected_initial"])
                amax.append(st["affected_max"])
                edges.append(st["edges_processed"])
                work.append(st["edges_processed"] / (dgt.m * static_iters))
                del dgt, db
            sweep.append({"fraction": f, "batches": args.sweep_batches,
                          "batch_seeds": f"1..{args.sweep_batches}",
                          "static_ms_geomean": round(gmean(sm), 3),
                          "dfp_ms_geomean": round(gmean(dm), 3),
                          "dfp_speedup_geomean": round(gmean(sp), 2),
                          "dfp_speedup_min": round(min(sp), 2),
                          "dfp_speedup_max": round(max(sp), 2),
                          "dfp_iters": its, "max_dfp_vs_static_linf": err,
                          "affected_initial": a0, "affected_max": amax,
                          "in_edges_processed": edges,
                          "work_vs_static_geomean": round(gmean(work), 5)})
        out["batch_sweep"] = sweep
        log(f"batch sweep ({time.time() - t:.1f} s): "
            + ", ".join(f"{x['fraction']:g}: {x['dfp_speedup_geomean']}x "
                        f"[{x['dfp_speedup_min']}, {x['dfp_speedup_max']}]" for x in sweep))

    if not args.no_compare and "static" in legs:
        # ablation of the rank kernel's design choices: rank-kernel time per
        # launch (6 Static iterations at tol 0 on G^{t-1}) under each setting
        settings = {
            "default": {},
            "no_partition_lane_per_vertex": dict(lane_max_degree=1 << 30, wave_max_degree=1 << 30),
            "paper_two_kernels_32": dict(lane_max_degree=32, wave_max_degree=1 << 30,
                                         xcd_split_degree=0),
            "no_die_split": dict(xcd_split_degree=0),
            "no_relabel": dict(relabel=0),
            "no_die_split_no_relabel": dict(xcd_split_degree=0, relabel=0),
        }
        tmp = torch.empty(n, dtype=torch.float64, device="cuda")
        abl = {}
        prhip.set_profiling(True)
        for name, kw in settings.items():
            prhip.set_tuning()
            prhip.set_tuning(**kw)
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                prhip.static(dg0, tol=0.0, max_iter=2, out=tmp)
                prhip.static(dg0, tol=0.0, max_iter=6, out=tmp)
            st = prhip.last_stats()
            abl[name] = round(st["rank_kernel_ms"] / st["rank_kernel_launches"] * 1e3, 1)
        prhip.set_profiling(False)
        prhip.set_tuning()
        out["ablation_rank_us"] = abl
        log(f"ablation (rank kernel us per launch): {abl}")

    if not args.no_accuracy and "dfp" in legs:
        acc = []
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        for j, f in enumerate(fracs):
            # reference Static run at a vanishing tolerance, capped at 500 iterations
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                prhip.static(dgs[j], tol=0.0, max_iter=500, out=ref)
            d_dfp = (dfp_out[j] - ref).abs()
            d_st = (static_out[j] - ref).abs()
            acc.append({"fraction": f,
                        "dfp_vs_static_linf": float((dfp_out[j] - static_out[j]).abs().max()),
                        "dfp_linf": float(d_dfp.max()), "dfp_l1": float(d_dfp.sum()),
                        "static_linf": float(d_st.max()), "static_l1": float(d_st.sum()),
                        "max_rank": float(ref.max())})
        out["accuracy"] = acc
        log(f"accuracy: max DF-P vs Static L-inf {max(a['dfp_vs_static_linf'] for a in acc):.3e}")

    if not args.no_compare and "static" in legs:
        out["small_graph"] = small_leg(gg, prhip, torch, np, tune=not args.no_tune)

    if args.temporal_batches > 0:
        out["temporal"] = temporal_leg(args, gg, prhip, torch, np)

    if "static" in legs:
        # measured ceiling of a plain streaming device copy on this machine
        out["roofline"]["copy_ceiling_gbs"] = round(copy_probe(), 1)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log(f"cpu baseline: oracle Static on the same graph, {args.cpu_iters} iterations")
        res, sec = oracle.static_csr(n, g0.in_offsets, g0.in_sources, g0.out_offsets, tol=0.0,
                                     max_iter=args.cpu_iters)
        cpu = {"value": round(g0.m * res.iters / sec / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", **cpu_info(),
               "sample": f"{res.iters} Static iterations (Alg. 1) of the sequential FP64 oracle on "
                         f"the scale-{args.scale} graph G^(t-1), iteration loop only "
                         f"({sec:.1f} s)"}
        log(f"cpu baseline {cpu}")
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
