"""Pins for the CPU oracle.

Each pin checks the oracle against something other than itself: a dense
linear solve (numpy LAPACK) of the PageRank fixed point, closed forms on
hand-analysed graphs, invariants of the fixed point, brute-force
reachability, or central finite differences of a dense forward solve. Every
pin is a function of the loaded oracle library so that the mutation test can
run the same pins against deliberately broken builds of the oracle and show
that some pin fails for each planted mistake.

Fixed point (Eq. 1, Sec. 3.1): r = alpha * A r + (1 - alpha)/N * 1 with
A[v][u] = 1/|out(u)| for each edge u -> v; every vertex has a self-loop
(Sec. 3.1, dead ends), so A is column-stochastic and sum(r) = 1.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2404_08299_amd import graphgen as gg

ALPHA = 0.85


# ---------------------------------------------------------------- dense refs
def dense_A(n, src, dst, w=None):
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if w is None:
        d = np.bincount(src, minlength=n).astype(np.float64)
        w = 1.0 / d[src]
    A = np.zeros((n, n))
    np.add.at(A, (dst, src), w)
    return A


def dense_solve(n, src, dst, alpha=ALPHA, s=None, w=None):
    """Exact fixed point of r = alpha*A r + (1-alpha) s by LU (numpy)."""
    A = dense_A(n, src, dst, w)
    s = np.full(n, 1.0 / n) if s is None else np.asarray(s, np.float64)
    return np.linalg.solve(np.eye(n) - alpha * A, (1 - alpha) * s)


# ------------------------------------------------------------- small graphs
def cycle(n):
    v = np.arange(n, dtype=np.int32)
    return gg.from_edges(n, v, (v + 1) % n)


def in_star(k):
    """Leaves 1..k point at center 0 (self-loops added by from_edges)."""
    leaves = np.arange(1, k + 1, dtype=np.int32)
    return gg.from_edges(k + 1, leaves, np.zeros(k, np.int32))


def out_star(k):
    """Center 0 points at leaves 1..k."""
    leaves = np.arange(1, k + 1, dtype=np.int32)
    return gg.from_edges(k + 1, np.zeros(k, np.int32), leaves)


def random_graph(n, e, seed):
    rng = np.random.default_rng(seed)
    return gg.from_edges(n, rng.integers(0, n, e, dtype=np.int32),
                         rng.integers(0, n, e, dtype=np.int32))


def small_graphs():
    yield "rmat6", gg.rmat_graph(6, 4, seed=3)
    yield "rmat9", gg.rmat_graph(9, 8, seed=1)
    yield "er300", random_graph(300, 1500, seed=5)
    yield "rmat9-unscrambled", gg.rmat_graph(9, 8, seed=2, scramble=False)


# -------------------------------------------------------------- static pins
def pin_static_dense(lib):
    for name, g in small_graphs():
        s, d = g.edges()
        res = oracle.static(g.n, s, d, tol=1e-14, max_iter=5000, lib=lib)
        assert res.status == oracle.OK, name
        ref = dense_solve(g.n, s, d)
        err = np.abs(res.ranks - ref).max()
        assert err <= 1e-12, (name, err)


def pin_static_cycle(lib):
    """Directed cycle with self-loops: uniform ranks are the fixed point and
    the uniform start is already there, so one iteration converges."""
    n = 7
    g = cycle(n)
    s, d = g.edges()
    res = oracle.static(n, s, d, tol=1e-15, lib=lib)
    assert res.iters == 1 and res.delta <= 1e-16, (res.iters, res.delta)
    assert np.abs(res.ranks - 1.0 / n).max() <= 1e-16


def pin_static_single_vertex(lib):
    g = gg.from_edges(1, [], [])
    s, d = g.edges()
    res = oracle.static(1, s, d, tol=0.0, lib=lib)
    assert res.status == oracle.OK and res.iters == 1
    assert abs(res.ranks[0] - 1.0) <= 1e-15


def pin_static_in_star(lib):
    """In-star: leaves have out-degree 2 and in-degree 1, the center
    out-degree 1. Fixed point r_leaf = 2(1-a)/(N(2-a)), r_center = 1 - k r_leaf.
    The iterates obey a two-variable recurrence (leaf x, center y):
      x' = C0 + a x/2,  y' = C0 + a (y + k x/2),
    so the iteration count and the returned iterate are pinned too."""
    k = 9
    n = k + 1
    a = ALPHA
    g = in_star(k)
    s, d = g.edges()
    res = oracle.static(n, s, d, tol=1e-15, max_iter=1000, lib=lib)
    rl = 2 * (1 - a) / (n * (2 - a))
    rc = 1 - k * rl
    assert abs(res.ranks[0] - rc) <= 1e-14 and np.abs(res.ranks[1:] - rl).max() <= 1e-14
    for tol in (1e-6, 1e-10):
        C0 = (1 - a) / n
        x = y = 1.0 / n
        it = 0
        while True:
            x2 = C0 + a * (x / 2)
            y2 = C0 + a * (y + k * (x / 2))
            it += 1
            delta = max(abs(x2 - x), abs(y2 - y))
            x, y = x2, y2
            if delta <= tol:
                break
        res = oracle.static(n, s, d, tol=tol, lib=lib)
        assert res.iters == it, (tol, res.iters, it)
        assert abs(res.ranks[0] - y) <= 1e-15 and np.abs(res.ranks[1:] - x).max() <= 1e-15


def pin_static_out_star(lib):
    """Out-star: r_c = (1-a)/(N(1 - a/(k+1))), r_leaf = (a r_c/(k+1) + (1-a)/N)/(1-a)."""
    k = 6
    n = k + 1
    a = ALPHA
    g = out_star(k)
    s, d = g.edges()
    res = oracle.static(n, s, d, tol=1e-15, max_iter=2000, lib=lib)
    rc = (1 - a) / (n * (1 - a / (k + 1)))
    rl = (a * rc / (k + 1) + (1 - a) / n) / (1 - a)
    assert abs(res.ranks[0] - rc) <= 1e-14 and np.abs(res.ranks[1:] - rl).max() <= 1e-14


def pin_static_local_closed_form(lib):
    """A vertex whose only in-edge is its self-loop has r = (1-a)/(N(1 - a/d))."""
    g = gg.rmat_graph(10, 8, seed=1)
    s, d = g.edges()
    res = oracle.static(g.n, s, d, tol=1e-14, max_iter=5000, lib=lib)
    indeg = g.in_degree()
    outdeg = g.out_degree()
    sel = indeg == 1
    assert sel.sum() > 50
    ref = (1 - ALPHA) / (g.n * (1 - ALPHA / outdeg[sel]))
    assert np.abs(res.ranks[sel] - ref).max() <= 1e-14


def pin_static_invariants(lib):
    """sum r = 1, r >= (1-a)/N, relabelling permutes r."""
    g = gg.rmat_graph(9, 8, seed=4)
    s, d = g.edges()
    res = oracle.static(g.n, s, d, tol=1e-14, max_iter=5000, lib=lib)
    assert abs(res.ranks.sum() - 1.0) <= 1e-12
    assert res.ranks.min() >= (1 - ALPHA) / g.n * (1 - 1e-12)
    perm = np.random.default_rng(7).permutation(g.n).astype(np.int32)
    res2 = oracle.static(g.n, perm[s], perm[d], tol=1e-14, max_iter=5000, lib=lib)
    assert np.abs(res2.ranks[perm] - res.ranks).max() <= 1e-13


def pin_static_contraction(lib):
    """||r_k - r*||_1 <= a^k ||r_0 - r*||_1 (A column-stochastic), and the
    first step from the uniform vector moves toward r*."""
    g = gg.rmat_graph(8, 8, seed=9)
    s, d = g.edges()
    ref = dense_solve(g.n, s, d)
    e0 = np.abs(np.full(g.n, 1.0 / g.n) - ref).sum()
    for k in range(1, 6):
        res = oracle.static(g.n, s, d, tol=0.0, max_iter=k, lib=lib)
        assert res.status == oracle.NOT_CONVERGED and res.iters == k
        ek = np.abs(res.ranks - ref).sum()
        assert ek <= ALPHA ** k * e0 * (1 + 1e-9), (k, ek, ALPHA ** k * e0)


def pin_static_rows_dense(lib):
    """One Eq. 1 step for listed rows (the sampled check of full-size runs)
    equals the dense product (1-a)/N + a * A x, row by row, for an arbitrary
    positive x (not a PageRank iterate), repeated and unordered rows."""
    g = gg.rmat_graph(9, 8, seed=11)
    s, d = g.edges()
    A = dense_A(g.n, s, d)
    x = np.random.default_rng(3).random(g.n) + 0.1
    ref = (1 - ALPHA) / g.n + ALPHA * (A @ x)
    rows = np.concatenate([np.arange(g.n), [g.n - 1, 0, 7, 7]]).astype(np.int32)[::-1]
    got = oracle.static_rows(g.n, g.in_offsets, g.in_sources, g.out_offsets, x, rows, lib=lib)
    assert np.abs(got - ref[rows]).max() <= 1e-14 * np.abs(ref).max()
    assert oracle.static_rows(g.n, g.in_offsets, g.in_sources, g.out_offsets, x,
                              np.zeros(0, np.int32), lib=lib).size == 0


def pin_pull_rows_weighted_and_ppr_dense(lib):
    """The same row step with per-in-edge weights, and with K teleport vectors
    (sampled (row, vector) pairs of a vertex-major [n][K] iterate): equal to
    the dense products (1-a) S[:, j] + a * A_w X[:, j] and (1-a) S[:, j] +
    a * A X[:, j], column by column."""
    g = gg.rmat_graph(8, 8, seed=12)
    rng = np.random.default_rng(5)
    dst = np.repeat(np.arange(g.n), g.in_degree())
    src = g.in_sources
    w = rng.random(g.m) + 0.05
    K = 3
    X = rng.random((g.n, K)) + 0.1
    S = rng.random((g.n, K))
    rows = rng.integers(0, g.n, 300).astype(np.int32)
    cols = rng.integers(0, K, 300).astype(np.int32)
    Aw = dense_A(g.n, src, dst, w)
    A = dense_A(g.n, src, dst)
    for weights, M in ((w, Aw), (None, A)):
        ref = (1 - ALPHA) * S + ALPHA * (M @ X)
        got = oracle.pull_rows(g.n, g.in_offsets, g.in_sources, g.out_offsets, X, rows, cols=cols,
                               weights=weights, teleport=S, lib=lib)
        assert np.abs(got - ref[rows, cols]).max() <= 1e-14 * np.abs(ref).max()
    # weighted, one vector, uniform teleport term
    got = oracle.pull_rows(g.n, g.in_offsets, g.in_sources, None, X[:, 1].copy(), rows,
                           weights=w, lib=lib)
    ref = (1 - ALPHA) / g.n + ALPHA * (Aw @ X[:, 1])
    assert np.abs(got - ref[rows]).max() <= 1e-14 * np.abs(ref).max()


def _in_star_recurrence(k, x, y, tol, a=ALPHA, max_iter=100000):
    """Eq. 1 iterates of the in-star from leaf value x and center value y:
    x' = C0 + a x/2, y' = C0 + a (y + k x/2). Returns [(x_i, y_i)] for
    i = 1 .. the first iteration whose L-infinity change is <= tol."""
    n = k + 1
    C0 = (1 - a) / n
    out = []
    for _ in range(max_iter):
        x2 = C0 + a * (x / 2)
        y2 = C0 + a * (y + k * (x / 2))
        delta = max(abs(x2 - x), abs(y2 - y))
        x, y = x2, y2
        out.append((x, y))
        if delta <= tol:
            break
    return out


def _check_star_iterate(ranks, xy, k):
    x, y = xy
    assert abs(ranks[0] - y) <= 1e-15 and np.abs(ranks[1:k + 1] - x).max() <= 1e-15, (
        ranks[:3], x, y)


def pin_nd_start_vector(lib):
    """Naive-dynamic (Sec. 3.4.1) is Alg. 1 started from the previous ranks.
    From a non-uniform start on the in-star, the first iterate and the
    iteration counts at two tolerances follow the Eq. 1 recurrence started
    from that vector (a run from 1/N gives other iterates and counts)."""
    k = 9
    n = k + 1
    g = in_star(k)
    s, d = g.edges()
    x0 = 0.02
    init = np.full(n, x0)
    init[0] = 1.0 - k * x0
    seq = _in_star_recurrence(k, x0, init[0], tol=0.0, max_iter=1)
    res = oracle.static(n, s, d, tol=0.0, max_iter=1, init=init, lib=lib)
    assert res.status == oracle.NOT_CONVERGED and res.iters == 1
    _check_star_iterate(res.ranks, seq[0], k)
    for tol in (1e-6, 1e-10):
        seq = _in_star_recurrence(k, x0, init[0], tol)
        res = oracle.static(n, s, d, tol=tol, init=init, lib=lib)
        assert res.status == oracle.OK and res.iters == len(seq), (tol, res.iters, len(seq))
        _check_star_iterate(res.ranks, seq[-1], k)
    assert res.iters != oracle.static(n, s, d, tol=1e-10, lib=lib).iters


# ---------------------------------------------------------------- DF-P pins
def _affected_all(n):
    """A marking-only batch whose insertion sources are every vertex:
    initialAffected then flags delta_N everywhere, so with self-loops every
    vertex becomes affected (only insertion sources are read)."""
    z = np.zeros(0, np.int32)
    return gg.Batch(z, z.copy(), np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32))


def pin_dfp_empty_batch(lib):
    """Nothing affected: the ranks are carried forward unchanged, the first
    L-infinity change is exactly 0, so the run stops after one iteration even
    with tol = 0."""
    g = gg.rmat_graph(8, 8, seed=2)
    s, d = g.edges()
    prev = oracle.static(g.n, s, d, lib=lib).ranks
    res = oracle.dfp(g.n, s, d, gg.Batch.empty(), prev, tol=0.0, lib=lib)
    assert res.status == oracle.OK and res.iters == 1 and res.delta == 0.0
    assert np.array_equal(res.ranks, prev)


def pin_dfp_eq2_fixed_point(lib):
    """With every vertex affected and pruning off, DF-P is a plain Eq. 2
    sweep; its fixed point is the Eq. 1 fixed point (dense solve)."""
    for name, g in small_graphs():
        s, d = g.edges()
        prev = np.random.default_rng(3).random(g.n) + 0.5
        prev /= prev.sum()
        res = oracle.dfp(g.n, s, d, _affected_all(g.n), prev, tol=1e-14, tau_f=-1.0,
                         tau_p=-1.0, max_iter=5000, lib=lib)
        assert res.status == oracle.OK, name
        err = np.abs(res.ranks - dense_solve(g.n, s, d)).max()
        assert err <= 1e-12, (name, err)


def _reach(adj_out, start, hops):
    cur = set(start)
    for _ in range(hops):
        cur = cur | {w for u in cur for w in adj_out[u]}
    return cur


def pin_dfp_frontier_reachability(lib):
    """tau_f = -1 (every updated vertex expands) and tau_p = -1 (no pruning):
    the affected set at iteration i is out^{i+1}(batch sources) together with
    out^{i}(deletion targets), brute-forced by breadth-first search."""
    n = 12
    es = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (6, 7), (7, 8), (8, 6), (9, 10), (5, 11)]
    g = gg.from_edges(n, [e[0] for e in es], [e[1] for e in es])
    s, d = g.edges()
    adj_out = {u: set(g.out_targets[g.out_offsets[u]:g.out_offsets[u + 1]].tolist()) for u in range(n)}
    batch = gg.Batch(np.array([6], np.int32), np.array([9], np.int32),
                     np.array([0], np.int32), np.array([3], np.int32))
    prev = np.full(n, 1.0 / n)
    iters = 4
    res = oracle.dfp(n, s, d, batch, prev, tol=0.0, tau_f=-1.0, tau_p=-1.0, max_iter=iters,
                     trace=True, lib=lib)
    assert res.iters == iters
    for i in range(iters):
        expect = _reach(adj_out, {6, 0}, i + 1) | _reach(adj_out, {9}, i)
        got = set(np.nonzero(res.trace[i])[0].tolist())
        assert got == expect, (i, sorted(got), sorted(expect))


def pin_dfp_initial_marking(lib):
    """After initialAffected + expandAffected: exactly out_t(u) for every
    batch source u, plus every deletion target (brute force over sets)."""
    g0 = gg.rmat_graph(8, 8, seed=5)
    b = gg.random_batch(g0, 40, seed=11)
    g = gg.apply_batch(g0, b)
    s, d = g.edges()
    prev = oracle.static(g0.n, *g0.edges(), lib=lib).ranks
    res = oracle.dfp(g.n, s, d, b, prev, trace=True, lib=lib)
    expect = set(b.del_dst.tolist())
    for u in set(b.del_src.tolist()) | set(b.ins_src.tolist()):
        expect |= set(g.out_targets[g.out_offsets[u]:g.out_offsets[u + 1]].tolist())
    got = set(np.nonzero(res.trace[0])[0].tolist())
    assert got == expect
    assert res.stats["affected_initial"] == len(expect)


def pin_dfp_eq2_one_step(lib):
    """Out-star with the center at its fixed point and the leaves perturbed:
    a leaf's in-neighbours other than itself are fixed, so one Eq. 2 update
    puts it exactly on its fixed point. With tau_p = +inf every updated vertex
    is pruned and with tau_f = +inf nothing expands, so the second iteration
    updates nothing (L-infinity 0) and the run ends after two iterations."""
    k = 5
    n = k + 1
    a = ALPHA
    g = out_star(k)
    s, d = g.edges()
    rc = (1 - a) / (n * (1 - a / (k + 1)))
    rl = (a * rc / (k + 1) + (1 - a) / n) / (1 - a)
    prev = np.full(n, rl * 1.3)
    prev[0] = rc
    leaves = np.arange(1, n, dtype=np.int32)
    # deletion (l, l) marks leaf l and l's out-neighbours (just l itself)
    batch = gg.Batch(leaves, leaves.copy(), np.zeros(0, np.int32), np.zeros(0, np.int32))
    res = oracle.dfp(n, s, d, batch, prev, tol=0.0, tau_f=np.inf, tau_p=np.inf, trace=True,
                     lib=lib)
    assert res.status == oracle.OK and res.iters == 2, (res.status, res.iters)
    assert res.ranks[0] == rc
    assert np.abs(res.ranks[1:] - rl).max() <= 4e-16 * rl
    # the affected set: exactly the leaves, then nothing (all pruned)
    assert res.trace[0].tolist() == [0] + [1] * k and not res.trace[1].any()
    # tau_p = -1 prunes nothing and tau_f = +inf expands nothing: the leaves
    # stay affected in every iteration
    res = oracle.dfp(n, s, d, batch, prev, tol=0.0, tau_f=np.inf, tau_p=-1.0, max_iter=4,
                     trace=True, lib=lib)
    assert all(row.tolist() == [0] + [1] * k for row in res.trace)
    # the relative change divides by max(r, R[v]) (Alg. 3): the center, raised
    # to 1.3 r_c, moves back to r_c in one Eq. 2 step (in-degree 1), so its
    # relative change is 0.3/1.3 < 0.25 < 0.3/1.0 and with tau_f = 0.25 it must
    # not expand to the leaves. Deletion (1, 0) marks the center (target) and
    # out(1) = {1}.
    prev = np.full(n, rl)
    prev[0] = 1.3 * rc
    batch = gg.Batch(np.array([1], np.int32), np.array([0], np.int32),
                     np.zeros(0, np.int32), np.zeros(0, np.int32))
    res = oracle.dfp(n, s, d, batch, prev, tol=0.0, tau_f=0.25, tau_p=-1.0, max_iter=3,
                     trace=True, lib=lib)
    assert abs(res.ranks[0] - rc) <= 4e-16 * rc
    assert res.trace[0].tolist() == [1, 1] + [0] * (k - 1)
    assert res.trace[1].tolist() == [1, 1] + [0] * (k - 1)


def pin_df_eq1_iterate(lib):
    """DF (Sec. 4.3) updates affected vertices with Eq. 1 and never prunes.
    With every vertex affected (a marking batch whose sources are all
    vertices) its iterates from R^{t-1} are the plain Eq. 1 iterates: on the
    in-star they follow the two-variable recurrence, with the same iteration
    count at each tolerance. Eq. 2 would put a leaf (its only in-edge is its
    self-loop) on its fixed point in one step, so its iterates differ."""
    k = 9
    n = k + 1
    g = in_star(k)
    s, d = g.edges()
    x0 = 0.03
    prev = np.full(n, x0)
    prev[0] = 1.0 - k * x0
    seq = _in_star_recurrence(k, x0, prev[0], tol=0.0, max_iter=1)
    res = oracle.dfp(n, s, d, _affected_all(n), prev, tol=0.0, tau_f=-1.0, max_iter=1,
                     prune=False, lib=lib)
    assert res.iters == 1
    _check_star_iterate(res.ranks, seq[0], k)
    for tol in (1e-6, 1e-10):
        seq = _in_star_recurrence(k, x0, prev[0], tol)
        res = oracle.dfp(n, s, d, _affected_all(n), prev, tol=tol, tau_f=-1.0, prune=False,
                         lib=lib)
        assert res.status == oracle.OK and res.iters == len(seq), (tol, res.iters, len(seq))
        _check_star_iterate(res.ranks, seq[-1], k)
        # every vertex is updated in every iteration: in-edges processed = m
        # per iteration, and the affected set is all of V throughout
        assert res.stats["edges_processed"] == res.iters * g.m
        assert res.stats["affected_max"] == n and res.stats["affected_ever"] == n


def _counters_from_trace(g, trace, iters):
    """The affected-set statistics recounted from the per-iteration affected
    flags: initial size, largest size, in-edges of the affected vertices
    summed over the iterations, and the union's size."""
    indeg = g.in_degree().astype(np.int64)
    rows = trace[:iters].astype(bool)
    sizes = rows.sum(axis=1)
    return dict(affected_initial=int(trace[0].sum()), affected_max=int(sizes.max()),
                edges_processed=int(sum(indeg[r].sum() for r in rows)),
                affected_ever=int(rows.any(axis=0).sum()))


def pin_dfp_counters_brute_force(lib):
    """The affected-set counters of DF/DF-P (in-edges processed, largest
    affected set, Sec. 5 measurement) against a recount over the affected
    flags of every iteration. Two cases where the affected set grows after
    the initial marking: frontier reachability on a small graph (tau_f =
    tau_p = -1; the flags themselves are pinned by breadth-first search
    above), and DF-P and DF on an R-MAT graph with a random batch."""
    n = 12
    es = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (6, 7), (7, 8), (8, 6), (9, 10), (5, 11)]
    g = gg.from_edges(n, [e[0] for e in es], [e[1] for e in es])
    s, d = g.edges()
    batch = gg.Batch(np.array([6], np.int32), np.array([9], np.int32),
                     np.array([0], np.int32), np.array([3], np.int32))
    res = oracle.dfp(n, s, d, batch, np.full(n, 1.0 / n), tol=0.0, tau_f=-1.0, tau_p=-1.0,
                     max_iter=5, trace=True, lib=lib)
    expect = _counters_from_trace(g, res.trace, res.iters)
    assert res.stats == expect, (res.stats, expect)
    assert expect["affected_max"] > expect["affected_initial"]
    g0 = gg.rmat_graph(9, 8, seed=13)
    prev = oracle.static(g0.n, *g0.edges(), lib=lib).ranks
    b = gg.random_batch(g0, 12, seed=5)
    g1 = gg.apply_batch(g0, b)
    s1, d1 = g1.edges()
    for prune in (True, False):
        res = oracle.dfp(g1.n, s1, d1, b, prev, prune=prune, trace=True, lib=lib)
        expect = _counters_from_trace(g1, res.trace, res.iters)
        assert res.stats == expect, (prune, res.stats, expect)
        assert expect["affected_max"] > expect["affected_initial"], expect


def pin_dfp_csr_input(lib):
    """DF-P over a given CSR (both views) equals DF-P over the edge list the
    oracle builds its own adjacency from, bit for bit: the CSR entry only
    changes where the rows come from. Scrambled IDs, deletions and
    insertions, DF and DF-P."""
    g0 = gg.rmat_graph(10, 8, seed=21)
    s0, d0 = g0.edges()
    prev = oracle.static(g0.n, s0, d0, tol=1e-12, lib=lib).ranks
    b = gg.random_batch(g0, 200, seed=4)
    g1 = gg.apply_batch(g0, b)
    s1, d1 = g1.edges()
    for prune in (True, False):
        a = oracle.dfp(g1.n, s1, d1, b, prev, prune=prune, lib=lib)
        c = oracle.dfp_csr(g1, b, prev, prune=prune, lib=lib)
        assert a.iters == c.iters and np.array_equal(a.ranks, c.ranks) and a.stats == c.stats


def pin_dfp_accuracy(lib):
    """DF-P from the converged ranks of G^{t-1} lands near the fixed point
    of G^t (dense solve); the error is of the order of the prune tolerance
    times the rank scale (the paper accepts a higher error for DF-P,
    Sec. 5.3). DF (no pruning) is tighter."""
    g0 = gg.rmat_graph(10, 8, seed=6)
    s0, d0 = g0.edges()
    prev = oracle.static(g0.n, s0, d0, tol=1e-14, max_iter=5000, lib=lib).ranks
    b = gg.random_batch(g0, gg.batch_size_for(g0, 1e-3), seed=3)
    g = gg.apply_batch(g0, b)
    s, d = g.edges()
    ref = dense_solve(g.n, s, d)
    res = oracle.dfp(g.n, s, d, b, prev, lib=lib)
    assert res.status == oracle.OK
    err = np.abs(res.ranks - ref).max()
    assert err <= 10 * oracle.TAU_P * ref.max(), (err, ref.max())
    res_df = oracle.dfp(g.n, s, d, b, prev, prune=False, lib=lib)
    err_df = np.abs(res_df.ranks - ref).max()
    assert err_df <= 10 * oracle.TAU_F * ref.max()


# ------------------------------------------------------------------ DT pins
def _reachable(g, seeds):
    """Brute force: every vertex reachable from `seeds` along out-edges."""
    seen = set(seeds)
    stack = list(seeds)
    while stack:
        u = stack.pop()
        for w in g.out_targets[g.out_offsets[u]:g.out_offsets[u + 1]].tolist():
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return seen


def pin_dt_exact_and_reachability(lib):
    """DT (Alg. 7) re-solves only the vertices reachable from the batch. A
    vertex no changed edge reaches has no changed ancestor, so its exact rank
    does not change: started from the exact ranks of G^{t-1}, DT lands on the
    dense solution of G^t, and the unreachable vertices keep their ranks bit
    for bit. The affected count equals brute-force reachability from the
    batch sources and the deletion targets."""
    cases = [(9, 6, 30, 0.8), (10, 8, 5, 1.0), (9, 10, 12, 0.0)]
    for scale, ef, size, ins in cases:
        g0 = gg.rmat_graph(scale, ef, seed=scale + size)
        b = gg.random_batch(g0, size, seed=size, insert_frac=ins)
        g = gg.apply_batch(g0, b)
        s, d = g.edges()
        prev = dense_solve(g0.n, *g0.edges())
        res = oracle.dt(g.n, s, d, b, prev, tol=1e-15, max_iter=5000, lib=lib)
        assert res.status == oracle.OK
        ref = dense_solve(g.n, s, d)
        err = np.abs(res.ranks - ref).max()
        assert err <= 1e-13, (scale, size, err)
        seeds = set(b.del_src.tolist()) | set(b.ins_src.tolist()) | set(b.del_dst.tolist())
        reach = _reachable(g, seeds)
        assert res.stats["affected"] == len(reach), (res.stats, len(reach))
        keep = np.array(sorted(set(range(g.n)) - reach), dtype=np.int64)
        assert np.array_equal(res.ranks[keep], prev[keep])


def pin_dt_empty_batch(lib):
    """Nothing reachable: one iteration with a zero change, ranks unchanged."""
    g = gg.rmat_graph(8, 8, seed=4)
    s, d = g.edges()
    prev = oracle.static(g.n, s, d, lib=lib).ranks
    res = oracle.dt(g.n, s, d, gg.Batch.empty(), prev, tol=0.0, lib=lib)
    assert res.status == oracle.OK and res.iters == 1 and res.delta == 0.0
    assert res.stats["affected"] == 0 and np.array_equal(res.ranks, prev)


# ----------------------------------------------------------------- PPR pins
def pin_ppr_dense_and_linearity(lib):
    g = gg.rmat_graph(9, 8, seed=8)
    s, d = g.edges()
    seeds = gg.distinct_vertices(g.n, 3, 16, seed=2)
    T = np.zeros((g.n, 4))
    for j in range(3):
        T[seeds[j], j] = 1.0 / 16
    T[:, 3] = 0.25 * T[:, 0] + 0.75 * T[:, 1]
    R, its = oracle.ppr(g.n, s, d, T, tol=1e-15, max_iter=5000, lib=lib)
    for j in range(4):
        assert np.abs(R[:, j] - dense_solve(g.n, s, d, s=T[:, j])).max() <= 1e-13
    assert np.abs(R[:, 3] - (0.25 * R[:, 0] + 0.75 * R[:, 1])).max() <= 1e-13
    U = np.full((g.n, 1), 1.0 / g.n)
    Ru, _ = oracle.ppr(g.n, s, d, U, tol=1e-15, max_iter=5000, lib=lib)
    assert np.abs(Ru[:, 0] - dense_solve(g.n, s, d)).max() <= 1e-13


# ------------------------------------------------- weighted forward + adjoint
def weighted_case(scale=8, seed=1):
    g = gg.rmat_graph(scale, 8, seed=seed)
    s, d = g.edges()
    w = gg.edge_weights(s, d, seed=seed)
    W = np.bincount(s, weights=w, minlength=g.n)
    P = w / W[s]
    tele = np.full(g.n, 1.0 / g.n)
    return g, s, d, P, tele


def pin_weighted_dense(lib):
    g, s, d, P, tele = weighted_case()
    res = oracle.weighted(g.n, s, d, P, tele, tol=1e-15, max_iter=5000, lib=lib)
    assert np.abs(res.ranks - dense_solve(g.n, s, d, s=tele, w=P)).max() <= 1e-13
    rng = np.random.default_rng(4)
    tele2 = rng.random(g.n)
    tele2 /= tele2.sum()
    res2 = oracle.weighted(g.n, s, d, P, tele2, tol=1e-15, max_iter=5000, lib=lib)
    assert np.abs(res2.ranks - dense_solve(g.n, s, d, s=tele2, w=P)).max() <= 1e-13


def pin_weighted_start_vector(lib):
    """The weighted forward from a given start vector: on the in-star with
    leaf self-loop weight p, leaf-to-center weight 1 - p and center self-loop
    weight 1, the iterates follow x' = (1-a) s_l + a p x and
    y' = (1-a) s_c + a (y + sum over leaves of (1-p) x) from that vector
    (first iterate and iteration count). The teleport differs per leaf, so
    the leaf values form a vector."""
    k = 7
    n = k + 1
    a = ALPHA
    p = 0.3
    g = in_star(k)
    s, d = g.edges()
    w = np.where(s == d, np.where(s == 0, 1.0, p), 1.0 - p)
    tele = np.linspace(1.0, 2.0, n)
    tele /= tele.sum()
    x0, y0 = 0.05, 1.0 - k * 0.05
    init = np.full(n, x0)
    init[0] = y0

    def step(x, y):
        return (1 - a) * tele[1:] + a * (p * x), (1 - a) * tele[0] + a * (y + ((1 - p) * x).sum())

    x, y = np.full(k, x0), y0
    res = oracle.weighted(n, s, d, w, tele, tol=0.0, max_iter=1, init=init, lib=lib)
    x1, y1 = step(x, y)
    assert res.status == oracle.NOT_CONVERGED
    assert abs(res.ranks[0] - y1) <= 1e-15 and np.abs(res.ranks[1:] - x1).max() <= 1e-15
    for tol in (1e-8, 1e-12):
        x, y = np.full(k, x0), y0
        it = 0
        while True:
            x2, y2 = step(x, y)
            it += 1
            delta = max(np.abs(x2 - x).max(), abs(y2 - y))
            x, y = x2, y2
            if delta <= tol:
                break
        res = oracle.weighted(n, s, d, w, tele, tol=tol, init=init, lib=lib)
        assert res.status == oracle.OK and res.iters == it, (tol, res.iters, it)
        assert abs(res.ranks[0] - y) <= 1e-15 and np.abs(res.ranks[1:] - x).max() <= 1e-15


def pin_adjoint_dense_and_fd(lib):
    """lambda = (I - a A^T)^{-1} g by LU; gradients against central finite
    differences (h = 1e-6) of a dense forward solve of the loss
    L = sum over targets of r_i^2."""
    g, s, d, P, tele = weighted_case(scale=7, seed=3)
    n = g.n
    rng = np.random.default_rng(5)
    targets = rng.choice(n, 20, replace=False)
    r = dense_solve(n, s, d, s=tele, w=P)
    gvec = np.zeros(n)
    gvec[targets] = 2 * r[targets]
    gw, gs, lam, it = oracle.adjoint(n, s, d, P, r, gvec, tol=1e-16, max_iter=5000, lib=lib)
    A = dense_A(n, s, d, P)
    lam_ref = np.linalg.solve((np.eye(n) - ALPHA * A).T, gvec)
    assert np.abs(lam - lam_ref).max() <= 1e-13 * max(1.0, np.abs(lam_ref).max())

    def loss(Pw, t):
        rr = dense_solve(n, s, d, s=t, w=Pw)
        return float((rr[targets] ** 2).sum())

    h = 1e-6
    for e in rng.choice(s.size, 12, replace=False):
        Pp = P.copy(); Pp[e] += h
        Pm = P.copy(); Pm[e] -= h
        fd = (loss(Pp, tele) - loss(Pm, tele)) / (2 * h)
        assert abs(gw[e] - fd) <= 1e-6 * abs(fd) + 1e-10, (e, gw[e], fd)
    for v in rng.choice(n, 6, replace=False):
        tp = tele.copy(); tp[v] += h
        tm = tele.copy(); tm[v] -= h
        fd = (loss(P, tp) - loss(P, tm)) / (2 * h)
        assert abs(gs[v] - fd) <= 1e-6 * abs(fd) + 1e-10, (v, gs[v], fd)


ALL_PINS = [
    pin_static_dense, pin_static_cycle, pin_static_single_vertex, pin_static_in_star,
    pin_static_out_star, pin_static_local_closed_form, pin_static_invariants,
    pin_static_contraction, pin_static_rows_dense, pin_pull_rows_weighted_and_ppr_dense,
    pin_nd_start_vector, pin_df_eq1_iterate, pin_dfp_counters_brute_force,
    pin_weighted_start_vector,
    pin_dfp_empty_batch, pin_dfp_eq2_fixed_point,
    pin_dfp_frontier_reachability, pin_dfp_initial_marking, pin_dfp_eq2_one_step,
    pin_dfp_csr_input,
    pin_dfp_accuracy, pin_dt_exact_and_reachability, pin_dt_empty_batch,
    pin_ppr_dense_and_linearity, pin_weighted_dense, pin_adjoint_dense_and_fd,
]
