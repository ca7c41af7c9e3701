#!/usr/bin/env python3
"""Benchmark: Static vs DF-P PageRank on one MI355X.

Workload (synthetic, seeded): R-MAT scale 24 (a, b, c, d = 0.57, 0.19, 0.19,
0.05), edge factor 16, seed 1, duplicates removed, one self-loop per vertex,
int32 CSR, FP64 ranks, alpha 0.85, tol 1e-10 (L-infinity), at most 500
iterations. Random batch updates of 1e-7 .. 1e-3 |E| (one per decade, batch
seed = decade index + 1), 80 % insertions of absent pairs, 20 % deletions of
existing non-self-loop edges. R^{t-1} is the Static result on G^{t-1}.

One step = pr_static on G^t plus pr_dfp(G^t, batch, R^{t-1}) for the batch
of that step; consecutive steps cycle through the decades. Inputs are resident
in HBM before the timed region. Prints one JSON line on stdout; progress goes
to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS & HBM GB/s per iteration; ms per batch update, DF-P vs Static"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rank_static_rmat24.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2404_08299_amd", "csrc", f)
                  for f in ("kernels.h", "wave.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n, m):
    """Compulsory bytes of one Static rank update: 4(n+1) in_offsets + 4m
    in_sources + 8n ranks gathered once + 4n out-degrees + 8n new ranks
    written + 4n vertex permutation, i.e. 4m + 28n."""
    return 4 * m + 28 * n


def read_traffic():
    """Measured HBM bytes per rank-kernel launch from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sha256") != kernel_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=float, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--fractions", default="1e-7,1e-6,1e-5,1e-4,1e-3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--order", default="scrambled", choices=["scrambled", "natural", "degree"],
                    help="vertex numbering of the input: Graph500 scrambled IDs, R-MAT's own "
                         "IDs, or relabelled by descending out-degree")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the calibration copy kernel")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              f"(the method is single-GPU; sharding is described in DESIGN.md)", file=sys.stderr)
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
    torch.cuda.synchronize()

    # R^{t-1}: Static on G^{t-1} (untimed)
    prev = prhip.static(dg0).ranks
    log(f"R^(t-1): {prhip.last_stats()['iterations']} iterations")
    static_out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in fracs]
    dfp_out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in fracs]
    rec = {j: {"static_ms": [], "dfp_ms": [], "static_iters": [], "dfp_iters": [],
               "rank_ms": [], "rank_launches": []} for j in range(len(fracs))}

    def step(s, record):
        j = s % len(fracs)
        t0 = time.perf_counter()
        prhip.static(dgs[j], out=static_out[j])
        t1 = time.perf_counter()
        st = prhip.last_stats()
        prhip.dfp(dgs[j], dbs[j], prev, out=dfp_out[j])
        t2 = time.perf_counter()
        sd = prhip.last_stats()
        if record:
            r = rec[j]
            r["static_ms"].append((t1 - t0) * 1e3)
            r["dfp_ms"].append((t2 - t1) * 1e3)
            r["static_iters"].append(st["iterations"])
            r["dfp_iters"].append(sd["iterations"])
            r["rank_ms"].append(st["rank_kernel_ms"])
            r["rank_launches"].append(st["rank_kernel_launches"])

    for s in range(args.warmup):
        step(s, False)
    log(f"warmup {args.warmup} steps done")
    prhip.set_profiling(True)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    for s in range(args.steps):
        step(args.warmup + s, True)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    prhip.set_profiling(False)
    ms_per_step = (T1 - T0) / args.steps * 1e3
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    edges_iter = 0.0
    bytes_iter = 0.0
    t_static = 0.0
    rank_ms = 0.0
    rank_bytes = 0.0
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
        sm = float(np.mean(r["static_ms"]))
        dm = float(np.mean(r["dfp_ms"]))
        per_batch.append({"fraction": f, "batch_size": sizes[j], "static_ms": round(sm, 3),
                          "dfp_ms": round(dm, 3), "dfp_speedup": round(sm / dm, 2),
                          "static_iters": r["static_iters"][0], "dfp_iters": r["dfp_iters"][0]})
    gteps = edges_iter / t_static / 1e9
    gbs = bytes_iter / t_static / 1e9
    launches = sum(sum(rec[j]["rank_launches"]) for j in rec)
    avg_rank_ms = rank_ms / max(1, launches)
    achieved = rank_bytes / (rank_ms / 1e3) / 1e9 if rank_ms > 0 else None
    traffic = read_traffic()
    log(f"Static {gteps:.2f} GTEPS, {gbs:.0f} GB/s algorithmic (whole call); rank kernel "
        f"{avg_rank_ms * 1e3:.1f} us avg over {launches} launches, {achieved:.0f} GB/s")

    accuracy = None
    if not args.no_accuracy:
        accuracy = []
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        for j, f in enumerate(fracs):
            # reference Static run at a vanishing tolerance, capped at 500 iterations
            with np.errstate(all="ignore"):
                import warnings
                with warnings.catch_warnings():
                    warnings.simplefilter("ignore")
                    prhip.static(dgs[j], tol=0.0, max_iter=500, out=ref)
            d_dfp = (dfp_out[j] - ref).abs()
            d_st = (static_out[j] - ref).abs()
            accuracy.append({
                "fraction": f,
                "dfp_vs_static_linf": float((dfp_out[j] - static_out[j]).abs().max()),
                "dfp_linf": float(d_dfp.max()), "dfp_l1": float(d_dfp.sum()),
                "static_linf": float(d_st.max()), "static_l1": float(d_st.sum()),
                "max_rank": float(ref.max())})
            log(f"accuracy {f:g}: {accuracy[-1]}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log(f"cpu baseline: oracle Static on the same graph, {args.cpu_iters} iterations")
        res, sec = oracle.static_csr(n, g0.in_offsets, g0.in_sources, g0.out_offsets, tol=0.0,
                                     max_iter=args.cpu_iters)
        cpu = {"value": round(g0.m * res.iters / sec / 1e9, 5), "unit": "GTEPS", "cores": 1,
               "kind": "oracle",
               "sample": f"{res.iters} Static iterations (Alg. 1) of the sequential FP64 oracle on "
                         f"the scale-{args.scale} graph G^(t-1), iteration loop only "
                         f"({sec:.1f} s)"}
        log(f"cpu baseline {cpu}")

    out = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{int(args.edge_factor)}_static_and_dfp",
                   "vertex_order": args.order,
                   "n": n, "m": g0.m, "scale": args.scale, "edge_factor": args.edge_factor,
                   "seed": args.seed, "batch_fractions": fracs, "alpha": 0.85, "tol": 1e-10,
                   "frontier_tol": 1e-6, "prune_tol": 1e-6, "max_iter": 500,
                   "tuning": prhip.get_tuning()},
        "static_gbs_per_iteration": round(gbs, 1),
        "batches": per_batch,
        "roofline": {"bound": "hbm", "kernel": "k_rank_static",
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic,
                     "avg_launch_us": round(avg_rank_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": algorithmic_bytes(n, g0.m)},
        "accuracy": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
