"""Parity at full size for the other workloads the benchmark times, on the
same seeded inputs and with the default tuning and launch shape:

- personalised PageRank on R-MAT scale 20 (edge factor 16, seed 1), 64
  teleport vectors each uniform over 16 distinct seed vertices;
- the weighted forward and its adjoint on the same graph, weights
  U(0.1, 1] row-normalised, teleport 1/N, the loss the sum of squared ranks of
  1024 random targets;
- 256 R-MAT graphs of log-uniform size in [2^10, 2^20] in one batched call;
- the preferential-attachment temporal stream (2 M vertices, 40 M events).

Whole oracle runs at these sizes do not fit a test, so the iterations are
checked one step at a time on sampled (row, vector) pairs with the oracle's
row step (relative bound 2 (deg + 2) u, u = 2^-53, the rounding of a sum of
positive terms in any order), the fixed points by properties that hold at any
size, the adjoint by its defining equation on sampled rows and by central
differences along two directions, the batched call against single calls bit
for bit and against whole oracle runs on its eight smallest graphs, and the
temporal stream by whole oracle DF-P runs on its first batches.
"""
import math
import warnings

import numpy as np
import pytest

import oracle
from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_08299_amd import prhip  # noqa: E402

U = 2.0 ** -53
ALPHA = 0.85


@pytest.fixture(scope="module")
def g20():
    prhip.set_tuning()
    g = gg.rmat_graph(20, 16, seed=1)
    print(f"scale 20: n={g.n} m={g.m}", flush=True)
    yield g, prhip.DeviceGraph.from_host(g)
    prhip.set_tuning()


def sample_rows(g, rng, k=2048):
    d = g.in_degree()
    picks = [np.argsort(-d, kind="stable")[:128], [0, g.n - 1], rng.choice(g.n, k, replace=False)]
    for lo, hi in [(1, 1), (2, 32), (33, 128), (129, 4096), (4097, 1 << 30)]:
        cand = np.flatnonzero((d >= lo) & (d <= hi))
        if cand.size:
            picks.append(rng.choice(cand, min(128, cand.size), replace=False))
    return np.unique(np.concatenate(picks)).astype(np.int32)


def quiet(fn, *a, **kw):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        return fn(*a, **kw)


def check_step(label, g, prev, cur, rows, cols=None, **kw):
    o = oracle.pull_rows(g.n, g.in_offsets, g.in_sources, g.out_offsets, prev, rows, cols=cols, **kw)
    got = cur[rows] if cols is None else cur[rows, cols]
    rel = np.abs(got - o) / o
    bound = 2 * (g.in_degree()[rows].astype(np.float64) + 2) * U
    print(f"{label}: {rows.size} samples, max rel diff {rel.max():.2e}, max rel/bound "
          f"{(rel / bound).max():.3f}", flush=True)
    assert (rel <= bound).all()


def ppr_teleport(n, K=64):
    sets = gg.distinct_vertices(n, K, 16, seed=2)
    T = np.zeros((n, K))
    for j in range(K):
        T[sets[j], j] = 1.0 / 16
    return T


def test_ppr_full_size(g20):
    g, dg = g20
    T = ppr_teleport(g.n)
    Td = torch.from_numpy(T).cuda()
    rng = np.random.default_rng(3)
    rows = sample_rows(g, rng)
    cols = rng.integers(0, T.shape[1], rows.size).astype(np.int32)
    it = {}

    def after(k):
        if k not in it:
            res, its = quiet(prhip.ppr, dg, Td, tol=0.0, max_iter=k)
            assert (its == k).all()
            it[k] = res.ranks.cpu().numpy()
        return it[k]

    for k in (1, 2, 40):
        prev = np.full((g.n, T.shape[1]), 1.0 / g.n) if k == 1 else after(k - 1)
        check_step(f"PPR step {k - 1} -> {k}", g, prev, after(k), rows, cols, teleport=T)
    res, its = prhip.ppr(dg, Td)
    r = res.ranks.cpu().numpy()
    print(f"PPR: iterations per vector {its.min()} .. {its.max()}", flush=True)
    assert res.converged
    for j in range(T.shape[1]):
        assert abs(math.fsum(r[:, j]) - 1.0) <= 1e-9
    assert (r >= (1 - ALPHA) * T * (1 - 1e-12)).all()


@pytest.fixture(scope="module")
def weighted_case(g20):
    g, dg = g20
    dst = np.repeat(np.arange(g.n, dtype=np.int32), g.in_degree())
    src = g.in_sources
    w = gg.edge_weights(src, dst, seed=1)
    W = np.bincount(src, weights=w, minlength=g.n)
    P = w / W[src]
    s = np.full(g.n, 1.0 / g.n)
    targets = np.random.default_rng(2).choice(g.n, 1024, replace=False)
    return g, dg, src, dst, P, s, targets


def test_weighted_forward_full_size(weighted_case):
    g, dg, src, dst, P, s, _ = weighted_case
    Pd, sd = torch.from_numpy(P).cuda(), torch.from_numpy(s).cuda()
    rows = sample_rows(g, np.random.default_rng(4))
    prev = np.full(g.n, 1.0 / g.n)
    for k in (1, 2, 3):
        cur = quiet(prhip.weighted, dg, Pd, sd, tol=0.0, max_iter=k).ranks.cpu().numpy()
        check_step(f"weighted step {k - 1} -> {k}", g, prev, cur, rows, weights=P, teleport=s)
        prev = cur
    r = prhip.weighted(dg, Pd, sd).ranks.cpu().numpy()
    assert abs(math.fsum(r) - 1.0) <= 1e-9 and r.min() >= (1 - ALPHA) / g.n * (1 - 1e-12)


def test_adjoint_full_size(weighted_case):
    g, dg, src, dst, P, s, targets = weighted_case
    Pd, sd = torch.from_numpy(P).cuda(), torch.from_numpy(s).cuda()
    tol = 1e-15
    r = prhip.weighted(dg, Pd, sd, tol=tol, max_iter=3000).ranks
    rh = r.cpu().numpy()
    gvec = np.zeros(g.n)
    gvec[targets] = 2 * rh[targets]
    gw, gs, lam = prhip.adjoint(dg, Pd, r, torch.from_numpy(gvec).cuda(), tol=tol, max_iter=3000,
                                want_lambda=True)
    gw, gs, lam = gw.cpu().numpy(), gs.cpu().numpy(), lam.cpu().numpy()
    # the defining equation lambda = g + alpha P^T lambda on sampled rows (a
    # pull over out-edges with the weights in out-CSR order)
    order = np.lexsort((dst, src))
    P_out = P[order]
    rows = sample_rows(g, np.random.default_rng(5))
    a_pl = oracle.pull_rows(g.n, g.out_offsets, g.out_targets, None, lam, rows, weights=P_out,
                            teleport=np.zeros(g.n))
    res = np.abs(lam[rows] - gvec[rows] - a_pl)
    print(f"adjoint: max |lambda| {np.abs(lam).max():.3e}, max residual on {rows.size} rows "
          f"{res.max():.2e}", flush=True)
    # at the stop the last change is <= tol, so the residual is <= alpha * tol
    # plus the rounding of the sums
    assert res.max() <= 2 * tol + 1e-12 * np.abs(lam).max()
    # the gradients are the products the adjoint defines
    assert np.allclose(gs, (1 - ALPHA) * lam, rtol=4 * U, atol=0)
    e = np.random.default_rng(6).choice(g.m, 4096, replace=False)
    assert np.allclose(gw[e], ALPHA * rh[src[e]] * lam[dst[e]], rtol=8 * U, atol=0)

    # central differences along P and along s: the loss moves by <grad,
    # direction>, a sum over every edge or vertex. The forward solves run to
    # the floating-point fixed point (tol 0), so the differences are not
    # swamped by the solves' own stopping error.
    tg = torch.from_numpy(targets).cuda()

    def loss(Pv, sv):
        rr = quiet(prhip.weighted, dg, torch.from_numpy(Pv).cuda(), torch.from_numpy(sv).cuda(),
                   tol=0.0, max_iter=1500).ranks
        return float((rr[tg] ** 2).sum())

    h = 1e-5
    fd_p = (loss(P * (1 + h), s) - loss(P * (1 - h), s)) / (2 * h)
    fd_s = (loss(P, s * (1 + h)) - loss(P, s * (1 - h))) / (2 * h)
    an_p, an_s = math.fsum(gw * P), math.fsum(gs * s)
    print(f"directional derivatives: along P fd {fd_p:.9e} adjoint {an_p:.9e}; along s fd "
          f"{fd_s:.9e} adjoint {an_s:.9e}", flush=True)
    assert abs(fd_p - an_p) <= 1e-6 * abs(an_p)
    assert abs(fd_s - an_s) <= 1e-6 * abs(an_s)


def test_adjoint_full_size_per_edge_fd(weighted_case):
    """The workload's own gradient check: central differences (h = 1e-6) of
    the loss on 100 random edges, half of them in-edges of the 1024 target
    rows (where the gradient is largest) and half drawn from all edges. Each
    difference perturbs one entry of P on the device and runs both forward
    solves to the floating-point fixed point (tol 0), so the solves' own
    stopping error does not swamp a change of the loss of about 1e-18. The
    difference divides by the perturbation actually applied (P_e + h minus
    P_e - h in FP64). Bound: |g_adj - g_fd| <= 1e-4 |g_fd| + 1e-6 max|g_adj|."""
    g, dg, src, dst, P, s, targets = weighted_case
    Pd, sd = torch.from_numpy(P).cuda(), torch.from_numpy(s).cuda()
    tol = 1e-15
    r = prhip.weighted(dg, Pd, sd, tol=tol, max_iter=3000).ranks
    rh = r.cpu().numpy()
    gvec = np.zeros(g.n)
    gvec[targets] = 2 * rh[targets]
    gw, _, _ = prhip.adjoint(dg, Pd, r, torch.from_numpy(gvec).cuda(), tol=tol, max_iter=3000,
                             want_lambda=True)
    gw = gw.cpu().numpy()
    rng = np.random.default_rng(3)
    into_targets = np.flatnonzero(np.isin(dst, targets))
    edges = np.concatenate([rng.choice(into_targets, 50, replace=False),
                            rng.choice(g.m, 50, replace=False)])
    tg = torch.from_numpy(targets).cuda()
    h = 1e-6

    def loss(Pv):
        rr = quiet(prhip.weighted, dg, Pv, sd, tol=0.0, max_iter=1500).ranks
        return math.fsum((rr[tg] ** 2).cpu().numpy())

    errs, scale = [], float(np.abs(gw).max())
    Pw = Pd.clone()
    for e in edges.tolist():
        p0 = float(P[e])
        hi_, lo_ = p0 + h, p0 - h
        Pw[e] = hi_
        lp = loss(Pw)
        Pw[e] = lo_
        lm = loss(Pw)
        Pw[e] = p0
        fd = (lp - lm) / (hi_ - lo_)
        err = abs(gw[e] - fd)
        errs.append((err, fd, gw[e]))
        assert err <= 1e-4 * abs(fd) + 1e-6 * scale, (e, fd, gw[e])
    a = np.array(errs)
    rel = a[:, 0] / np.maximum(np.abs(a[:, 1]), 1e-300)
    print(f"per-edge FD on {len(edges)} edges (h = {h:g}): |g| {np.abs(a[:, 2]).min():.2e} .. "
          f"{np.abs(a[:, 2]).max():.2e}; relative error median {np.median(rel[:50]):.2e}, "
          f"max {rel[:50].max():.2e} (target in-edges), median {np.median(rel[50:]):.2e}, "
          f"max {rel[50:].max():.2e} (random edges); max abs error {a[:, 0].max():.2e}",
          flush=True)


def test_batched_full_size():
    prhip.set_tuning()
    rng = np.random.default_rng(7)
    hosts = []
    for i in range(256):
        nb = int(2 ** rng.uniform(10, 20))
        ef = float(rng.uniform(4, 32))
        sc = int(np.ceil(np.log2(nb)))
        hosts.append(gg.rmat_graph(sc, ef * nb / (1 << sc), seed=1000 + i, n=nb))
    dgs = [prhip.DeviceGraph.from_host(h) for h in hosts]
    print(f"256 graphs: N={sum(h.n for h in hosts)} M={sum(h.m for h in hosts)}", flush=True)
    res, its = prhip.static_batched(dgs)
    assert res.converged
    for d, r in zip(dgs, res.ranks):
        assert torch.equal(prhip.static(d).ranks, r)
    small = np.argsort([h.n for h in hosts])[:8]
    for i in small:
        h = hosts[i]
        o = oracle.static(h.n, *h.edges())
        err = float(np.abs(res.ranks[i].cpu().numpy() - o.ranks).max())
        print(f"graph {i}: n={h.n} m={h.m} iters gpu {its[i]} oracle {o.iters} Linf {err:.2e}",
              flush=True)
        assert err <= 1e-9 and abs(int(its[i]) - o.iters) <= 1


def test_temporal_full_size():
    prhip.set_tuning()
    g0, steps = gg.temporal_stream(2_000_000, 40_000_000, seed=1, batches=100)
    prev = prhip.static(prhip.DeviceGraph.from_host(g0)).ranks
    for t, (b, g) in enumerate(steps):
        if t == 3:
            break
        d = prhip.dfp(prhip.DeviceGraph.from_host(g), prhip.DeviceBatch.from_host(b), prev)
        o = oracle.dfp_csr(g, b, prev.cpu().numpy())
        err = float(np.abs(d.ranks.cpu().numpy() - o.ranks).max())
        print(f"temporal batch {t}: +{b.ins_src.size} -{b.del_src.size}, m={g.m}, iters gpu "
              f"{d.iterations} oracle {o.iters}, Linf {err:.2e}", flush=True)
        assert d.converged and err <= 1e-9 and abs(d.iterations - o.iters) <= 1
        prev = d.ranks
