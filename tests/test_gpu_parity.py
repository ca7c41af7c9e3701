"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs. Bars: L-infinity <= 1e-9 at tol = 1e-10 for Static and
for DF/DF-P against the oracle's DF/DF-P; when every vertex is in the
lane-per-vertex class the GPU sums in the oracle's order and the results are
bit-identical."""
import numpy as np
import pytest

import oracle
from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_08299_amd import prhip  # noqa: E402

ALL_LANE = dict(lane_max_degree=1 << 30, wave_max_degree=1 << 30, expand_lane_max_degree=1 << 30)
ALL_CLASSES = dict(lane_max_degree=2, wave_max_degree=12, expand_lane_max_degree=2,
                   hub_chunk_edges=16, relabel=1, xcd_split_degree=0)
# die-split class: every row above the lane class, chunking inside segments,
# range-major grouping, fewer workgroups than dies, a grid not a multiple of 8
XSPLIT = [dict(xcd_split_degree=2, lane_max_degree=1),
          dict(xcd_split_degree=8, hub_chunk_edges=4, relabel=1),
          dict(xcd_split_degree=5, grid_blocks=5, relabel=1),
          dict(xcd_split_degree=3, grid_blocks=13, hub_chunk_edges=2, relabel=1),
          dict(xcd_split_degree=16, relabel=0, grid_blocks=64),
          # a wavefront class between the lane class and the die split, relabelled
          dict(lane_max_degree=4, xcd_split_degree=16, relabel=1)]


@pytest.fixture(autouse=True)
def default_tuning():
    prhip.set_tuning()
    yield
    prhip.set_tuning()


def dev(g):
    return prhip.DeviceGraph.from_host(g)


def gpu_static(g, **kw):
    r = prhip.static(dev(g), **kw)
    return r.ranks.cpu().numpy(), r


def ora_static(g, **kw):
    s, d = g.edges()
    return oracle.static(g.n, s, d, **kw)


# ------------------------------------------------------------------ Static
def test_static_rmat14_vs_oracle():
    """R-MAT scale 14, edge factor 8, seed 1 (the small configuration)."""
    g = gg.rmat_graph(14, 8, seed=1)
    r, res = gpu_static(g)
    o = ora_static(g)
    print(f"rmat14 n={g.n} m={g.m} gpu iters={res.iterations} oracle iters={o.iters}")
    assert res.converged and res.status == prhip.PR_OK
    assert np.abs(r - o.ranks).max() <= 1e-9
    assert abs(res.iterations - o.iters) <= 1


@pytest.mark.parametrize("relabel", [0, 1])
def test_static_all_lane_bitwise(relabel):
    prhip.set_tuning(**ALL_LANE, relabel=relabel)
    for g in (gg.rmat_graph(12, 8, seed=1), gg.rmat_graph(10, 16, seed=3, scramble=False)):
        r, res = gpu_static(g)
        o = ora_static(g)
        assert res.iterations == o.iters
        assert np.array_equal(r, o.ranks)


@pytest.mark.parametrize("tuning", [ALL_CLASSES, dict(lane_max_degree=0, wave_max_degree=0,
                                                         expand_lane_max_degree=0,
                                                         xcd_split_degree=0),
                                    dict(lane_max_degree=0, wave_max_degree=0,
                                         expand_lane_max_degree=0),
                                    dict(lane_max_degree=8, wave_max_degree=200,
                                         xcd_split_degree=0),
                                    dict(lane_max_degree=4, wave_max_degree=8, hub_chunk_edges=8,
                                         expand_lane_max_degree=4, grid_blocks=7,
                                         xcd_split_degree=0),
                                    dict(grid_blocks=1), dict(hub_chunk_edges=64, grid_blocks=3000),
                                    dict(relabel=1), dict(relabel=1, grid_blocks=5)] + XSPLIT)
def test_static_every_class(tuning):
    prhip.set_tuning(**tuning)
    g = gg.rmat_graph(13, 8, seed=2)
    r, res = gpu_static(g)
    o = ora_static(g)
    assert np.abs(r - o.ranks).max() <= 1e-9
    assert abs(res.iterations - o.iters) <= 1


@pytest.mark.parametrize("n", [1, 2, 63, 255, 257, 1023, 1025, 4097, 70001])
def test_static_ragged_sizes(n):
    scale = max(1, int(np.ceil(np.log2(max(n, 2)))))
    g = gg.rmat_graph(scale, 6, seed=n, n=n)
    assert g.n == n
    r, res = gpu_static(g)
    o = ora_static(g)
    assert np.abs(r - o.ranks).max() <= 1e-9


def test_static_closed_forms():
    prhip.set_tuning(hub_chunk_edges=512)
    a = 0.85
    # in-star with a hub above every lane/wave threshold (workgroup class)
    k = 6000
    g = gg.from_edges(k + 1, np.arange(1, k + 1, dtype=np.int32), np.zeros(k, np.int32))
    r, res = gpu_static(g, tol=1e-14, max_iter=2000)
    n = k + 1
    rl = 2 * (1 - a) / (n * (2 - a))
    assert abs(r[0] - (1 - k * rl)) <= 1e-12 and np.abs(r[1:] - rl).max() <= 1e-15
    # out-star: the center has out-degree k+1 (wavefront/workgroup class in marking)
    g = gg.from_edges(k + 1, np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32))
    r, _ = gpu_static(g, tol=1e-14, max_iter=2000)
    rc = (1 - a) / (n * (1 - a / (k + 1)))
    assert abs(r[0] - rc) <= 1e-15
    # directed cycle: converges in one iteration to 1/n
    g = gg.from_edges(1000, np.arange(1000, dtype=np.int32), (np.arange(1000, dtype=np.int32) + 1) % 1000)
    r, res = gpu_static(g, tol=1e-15)
    assert res.iterations == 1 and np.abs(r - 1e-3).max() <= 1e-17


def test_static_max_iter_and_determinism():
    g = gg.rmat_graph(12, 8, seed=5)
    with pytest.warns(RuntimeWarning):
        r, res = gpu_static(g, tol=0.0, max_iter=3)
    assert res.status == prhip.PR_NOT_CONVERGED and res.iterations == 3
    o = ora_static(g, tol=0.0, max_iter=3)
    assert np.abs(r - o.ranks).max() <= 1e-15
    a, _ = gpu_static(g)
    b, _ = gpu_static(g)
    assert np.array_equal(a, b)


def test_static_threshold_invariance():
    g = gg.rmat_graph(13, 8, seed=7)
    outs = []
    for t in (dict(), ALL_LANE, ALL_CLASSES, dict(lane_max_degree=16, wave_max_degree=64),
              *XSPLIT):
        prhip.set_tuning()
        prhip.set_tuning(**t)
        outs.append(gpu_static(g, tol=1e-13, max_iter=1000)[0])
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-13


def test_static_iters_per_sync():
    g = gg.rmat_graph(11, 8, seed=9)
    base, rb = gpu_static(g)
    for k in (1, 3, 7):
        prhip.set_tuning(iters_per_sync=k)
        r, res = gpu_static(g)
        assert res.iterations == rb.iterations and np.array_equal(r, base)


def test_validate():
    g = gg.rmat_graph(10, 8, seed=1)
    prhip.validate(dev(g))
    # drop vertex 5's self-loop from the in view
    d = dev(g)
    row = g.in_sources[g.in_offsets[5]:g.in_offsets[6]].copy()
    assert 5 in row
    bad = g.in_sources.copy()
    pos = g.in_offsets[5] + int(np.nonzero(row == 5)[0][0])
    bad[pos] = (5 + 1) % g.n if (5 + 1) % g.n not in row else 0
    d.in_sources = torch.from_numpy(bad).cuda()
    with pytest.raises(prhip.PrError) as e:
        prhip.validate(d)
    assert e.value.code in (prhip.PR_EGRAPH,)
    d2 = dev(g)
    off = g.in_offsets.copy()
    off[-1] += 1
    d2.in_offsets = torch.from_numpy(off).cuda()
    with pytest.raises(prhip.PrError):
        prhip.validate(d2)


# ------------------------------------------------------------------ DF / DF-P
def dynamic_case(scale=12, ef=8, frac=1e-3, seed=1):
    g0 = gg.rmat_graph(scale, ef, seed=seed)
    b = gg.random_batch(g0, gg.batch_size_for(g0, frac), seed=seed + 10)
    g1 = gg.apply_batch(g0, b)
    prev = oracle.static(g0.n, *g0.edges()).ranks
    return g0, g1, b, prev


def gpu_dfp(g1, b, prev, mode="dfp", **kw):
    p = torch.from_numpy(prev).cuda()
    r = prhip.dfp(dev(g1), prhip.DeviceBatch.from_host(b), p, mode=mode, **kw)
    return r.ranks.cpu().numpy(), r


@pytest.mark.parametrize("frac", [1e-4, 1e-3, 1e-2])
def test_dfp_vs_oracle(frac):
    g0, g1, b, prev = dynamic_case(frac=frac)
    r, res = gpu_dfp(g1, b, prev)
    o = oracle.dfp(g1.n, *g1.edges(), b, prev)
    print(f"frac={frac} batch={b.size} gpu iters={res.iterations} oracle iters={o.iters}")
    assert res.converged
    assert np.abs(r - o.ranks).max() <= 1e-9
    ref = oracle.static(g1.n, *g1.edges(), tol=1e-14, max_iter=5000).ranks
    assert np.abs(r - ref).max() <= 10 * 1e-6 * ref.max()


@pytest.mark.parametrize("tol_fp", [1e-7, 1e-8])
@pytest.mark.parametrize("tuning", [dict(), XSPLIT[1]])
def test_dfp_tighter_tolerances(tol_fp, tuning):
    """DF-P with the frontier and prune tolerances (Alg. 3) tightened below
    the paper's 1e-6: the oracle's trajectory at the same tolerances, and an
    error against the exact ranks that shrinks with them (within
    10 * tau_p * max(R), as at 1e-6; the oracle comes to 3.3-4.8 times
    tau_p * max(R) on these cases)."""
    prhip.set_tuning(**tuning)
    for seed, frac in ((5, 1e-3), (6, 1e-2)):
        g0, g1, b, prev = dynamic_case(scale=12, frac=frac, seed=seed)
        r, res = gpu_dfp(g1, b, prev, frontier_tol=tol_fp, prune_tol=tol_fp)
        o = oracle.dfp(g1.n, *g1.edges(), b, prev, tau_f=tol_fp, tau_p=tol_fp)
        assert res.converged
        assert np.abs(r - o.ranks).max() <= 1e-9
        assert abs(res.iterations - o.iters) <= 1
        ref = oracle.static(g1.n, *g1.edges(), tol=1e-14, max_iter=5000).ranks
        assert np.abs(r - ref).max() <= 10 * tol_fp * ref.max()


@pytest.mark.parametrize("relabel", [0, 1])
def test_dfp_all_lane_bitwise(relabel):
    prhip.set_tuning(**ALL_LANE, relabel=relabel)
    g0, g1, b, prev = dynamic_case(scale=11, frac=1e-3, seed=4)
    r, res = gpu_dfp(g1, b, prev)
    o = oracle.dfp(g1.n, *g1.edges(), b, prev)
    assert res.iterations == o.iters
    assert np.array_equal(r, o.ranks)


@pytest.mark.parametrize("mode", ["df", "nd"])
@pytest.mark.parametrize("relabel", [0, 1])
def test_df_nd_vs_oracle(mode, relabel):
    prhip.set_tuning(relabel=relabel)
    g0, g1, b, prev = dynamic_case(scale=12, frac=1e-3, seed=2)
    r, res = gpu_dfp(g1, b, prev, mode=mode)
    if mode == "df":
        o = oracle.dfp(g1.n, *g1.edges(), b, prev, prune=False)
    else:
        o = oracle.static(g1.n, *g1.edges(), init=prev)
    assert np.abs(r - o.ranks).max() <= 1e-9
    assert abs(res.iterations - o.iters) <= 1


@pytest.mark.parametrize("tuning", [ALL_CLASSES, dict(grid_blocks=1), dict(relabel=1),
                                    dict(lane_max_degree=4, wave_max_degree=8, hub_chunk_edges=8,
                                         expand_lane_max_degree=4, grid_blocks=5, relabel=1,
                                         xcd_split_degree=0)] + XSPLIT)
def test_dfp_every_class(tuning):
    prhip.set_tuning(**tuning)
    g0, g1, b, prev = dynamic_case(scale=13, frac=1e-3, seed=3)
    r, res = gpu_dfp(g1, b, prev)
    o = oracle.dfp(g1.n, *g1.edges(), b, prev)
    assert np.abs(r - o.ranks).max() <= 1e-9
    assert abs(res.iterations - o.iters) <= 1


@pytest.mark.parametrize("mode", ["dfp", "df"])
@pytest.mark.parametrize("tuning", [dict(), dict(xcd_split_degree=0),
                                    dict(xcd_split_degree=4, hub_chunk_edges=8, relabel=1),
                                    dict(lane_max_degree=4, wave_max_degree=8, hub_chunk_edges=8,
                                         expand_lane_max_degree=4, xcd_split_degree=0)])
def test_dfp_pull_equals_push(mode, tuning):
    """expandAffected marks the same set pulling over a frontier bitmap as
    pushing over the frontier's out-edges, so the whole DF/DF-P trajectory is
    the same: forced push (0), pull from a frontier of n/1000 (1), never
    pull (1000) and the default give bit-identical ranks."""
    g0, g1, b, prev = dynamic_case(scale=13, frac=1e-2, seed=6)
    outs = []
    for pm in (0, 1, 1000, None):
        prhip.set_tuning()
        prhip.set_tuning(**tuning, **({} if pm is None else dict(expand_pull_per_mille=pm)))
        r, res = gpu_dfp(g1, b, prev, mode=mode)
        outs.append((r, res.iterations))
    o = oracle.dfp(g1.n, *g1.edges(), b, prev, prune=(mode == "dfp"))
    assert np.abs(outs[0][0] - o.ranks).max() <= 1e-9
    for r, it in outs[1:]:
        assert it == outs[0][1] and np.array_equal(r, outs[0][0])


@pytest.mark.parametrize("mode", ["dfp", "df", "dt"])
@pytest.mark.parametrize("tuning", [dict(), ALL_LANE, ALL_CLASSES, dict(grid_blocks=3),
                                    XSPLIT[2]])
def test_affected_list_equals_sweep(mode, tuning):
    """The rank update and the apply/marking step over the compacted affected
    list (frontier_list = 1, the default) give the same bits and iteration
    counts as the sweeps over ID tiles of every vertex (frontier_list = 0)."""
    g0, g1, b, prev = dynamic_case(scale=13, frac=1e-3, seed=8)
    outs = []
    for fl in (0, 1):
        prhip.set_tuning()
        prhip.set_tuning(**tuning, frontier_list=fl)
        r, res = gpu_dfp(g1, b, prev, mode=mode)
        outs.append((r, res.iterations))
    assert outs[0][1] == outs[1][1] and np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("n", [1, 2, 17, 255, 4095, 4097, 70001])
def test_affected_list_ragged(n):
    """Vertex counts around the compaction's 16-vertex words and 4096-vertex
    rounds, every vertex in the lane class: bit-identical to the oracle."""
    prhip.set_tuning(**ALL_LANE)
    scale = max(1, int(np.ceil(np.log2(max(n, 2)))))
    g0 = gg.rmat_graph(scale, 6, seed=n, n=n)
    b = gg.random_batch(g0, max(1, gg.batch_size_for(g0, 1e-2)), seed=n + 1) if n > 2 \
        else gg.Batch.empty()
    g1 = gg.apply_batch(g0, b)
    prev = oracle.static(g0.n, *g0.edges()).ranks
    r, res = gpu_dfp(g1, b, prev, tol=0.0 if n <= 2 else 1e-10)
    o = oracle.dfp(g1.n, *g1.edges(), b, prev, tol=0.0 if n <= 2 else 1e-10)
    assert res.iterations == o.iters and np.array_equal(r, o.ranks)


def test_affected_list_prune_above_frontier_tol():
    """With prune_tol > frontier_tol a vertex can be pruned while its dN flag
    is set; the compaction must clear that flag (Alg. 2 clears delta_N at the
    start of every iteration), so the trajectory stays the oracle's."""
    prhip.set_tuning(**ALL_LANE)
    g0, g1, b, prev = dynamic_case(scale=11, frac=1e-2, seed=9)
    for tau_f, tau_p in ((1e-7, 1e-5), (1e-8, 1e-4)):
        r, res = gpu_dfp(g1, b, prev, frontier_tol=tau_f, prune_tol=tau_p)
        o = oracle.dfp(g1.n, *g1.edges(), b, prev, tau_f=tau_f, tau_p=tau_p)
        assert res.iterations == o.iters and np.array_equal(r, o.ranks)


@pytest.mark.parametrize("frac", [1e-4, 1e-2])
@pytest.mark.parametrize("tuning", [dict(), dict(xcd_split_degree=0), ALL_CLASSES,
                                    dict(grid_blocks=5, relabel=1), XSPLIT[0]])
def test_dt_vs_oracle(tuning, frac):
    """Dynamic Traversal (Alg. 7): the affected set is the closure of the
    batch under out-edges (its size must match exactly), then Eq. 1 over it."""
    prhip.set_tuning(**tuning)
    g0, g1, b, prev = dynamic_case(scale=12, frac=frac, seed=7)
    prhip.set_profiling(True)
    try:
        r, res = gpu_dfp(g1, b, prev, mode="dt")
        aff = prhip.last_stats()["affected_initial"]
    finally:
        prhip.set_profiling(False)
    o = oracle.dt(g1.n, *g1.edges(), b, prev)
    assert res.converged and np.abs(r - o.ranks).max() <= 1e-9
    assert abs(res.iterations - o.iters) <= 1
    assert aff == o.stats["affected"]


def test_dt_bitwise_and_empty():
    prhip.set_tuning(**ALL_LANE)
    g0, g1, b, prev = dynamic_case(scale=11, frac=1e-3, seed=8)
    r, res = gpu_dfp(g1, b, prev, mode="dt")
    o = oracle.dt(g1.n, *g1.edges(), b, prev)
    assert res.iterations == o.iters and np.array_equal(r, o.ranks)
    r, res = gpu_dfp(g1, gg.Batch.empty(), prev, mode="dt", tol=0.0)
    assert res.iterations == 1 and np.array_equal(r, prev)


@pytest.mark.parametrize("mode", ["dfp", "df", "dt"])
def test_affected_counters_match_oracle(mode):
    """With every row summed in the oracle's order the trajectory is the
    oracle's, so the profiling counters must equal its statistics: the
    affected set after the initial marking, the largest affected set of an
    iteration, and the in-edges processed over all iterations."""
    prhip.set_tuning(**ALL_LANE)
    g0, g1, b, prev = dynamic_case(scale=11, frac=1e-3, seed=12)
    prhip.set_profiling(True)
    try:
        r, res = gpu_dfp(g1, b, prev, mode=mode)
        st = prhip.last_stats()
    finally:
        prhip.set_profiling(False)
    s_, d_ = g1.edges()
    if mode == "dt":
        o = oracle.dt(g1.n, s_, d_, b, prev)
        assert st["affected_max"] == st["affected_initial"] == o.stats["affected"]
        # the fixed set's in-edges, once per iteration
        assert st["edges_processed"] % res.iterations == 0
    else:
        o = oracle.dfp(g1.n, s_, d_, b, prev, prune=(mode == "dfp"))
        assert st["affected_initial"] == o.stats["affected_initial"]
        assert st["affected_max"] == o.stats["affected_max"]
        assert st["edges_processed"] == o.stats["edges_processed"]
    assert res.iterations == o.iters and np.array_equal(r, o.ranks)


def test_dfp_empty_batch_and_inplace():
    g0, g1, b, prev = dynamic_case(scale=10, frac=1e-3, seed=5)
    r, res = gpu_dfp(g1, gg.Batch.empty(), prev, tol=0.0)
    assert res.iterations == 1 and np.array_equal(r, prev)
    p = torch.from_numpy(prev).cuda()
    out = prhip.dfp(dev(g1), prhip.DeviceBatch.from_host(b), p, out=p)
    assert out.ranks.data_ptr() == p.data_ptr()
    o = oracle.dfp(g1.n, *g1.edges(), b, prev)
    assert np.abs(p.cpu().numpy() - o.ranks).max() <= 1e-9


def test_dfp_affected_count_and_bad_batch():
    g0, g1, b, prev = dynamic_case(scale=11, frac=1e-3, seed=6)
    prhip.set_profiling(True)
    try:
        r, res = gpu_dfp(g1, b, prev)
    finally:
        prhip.set_profiling(False)
    o = oracle.dfp(g1.n, *g1.edges(), b, prev)
    assert res.stats["affected_initial"] == o.stats["affected_initial"]
    assert res.stats["rank_kernel_launches"] == res.iterations
    assert res.stats["rank_kernel_ms"] > 0
    bad = gg.Batch(b.del_src.copy(), b.del_dst.copy(), b.ins_src.copy(), b.ins_dst.copy())
    bad.del_dst[0] = g1.n + 5
    with pytest.raises(prhip.PrError) as e:
        gpu_dfp(g1, bad, prev)
    assert e.value.code == prhip.PR_EBATCH


def row_aligned_misses(old, new):
    """Entries of new's in-CSR whose source is not at the same place of its
    row in old's in-CSR (position e + old_off[v] - new_off[v], inside old's
    entries): an upper bound, in practice, on what a kept mapping misses."""
    v = np.repeat(np.arange(new.n), np.diff(new.in_offsets))
    e = np.arange(new.m)
    p = e + old.in_offsets[v].astype(np.int64) - new.in_offsets[v]
    ok = (p >= 0) & (p < old.m)
    hit = np.zeros(new.m, bool)
    hit[ok] = old.in_sources[p[ok]] == new.in_sources[e[ok]]
    return int(new.m - hit.sum())


@pytest.mark.parametrize("mode", ["dfp", "df", "dt"])
@pytest.mark.parametrize("tuning", [dict(relabel=1), dict(relabel=1, grid_blocks=13),
                                    dict(relabel=1, lane_max_degree=4, xcd_split_degree=16,
                                         hub_chunk_edges=8)])
def test_chain_numbering_same_bits(mode, tuning):
    """A chain of updates G1 -> G2 -> G3 (each R^t from the previous call),
    then G3 with its vertices renamed at random (same n, rows unrelated to
    the kept ones), then G3 again and a graph of another n. With the
    numbering kept across the calls (chain_numbering = 1) every call gives
    the same bits and iteration count as with it built inside each call
    (chain_numbering = 0). The calls report a kept numbering for G2, G3 and
    the renamed graph, whose mapping misses most entries, so that the next
    call builds it anew, as does the one with another n."""
    # R-MAT plus one row of 6000 in-edges (kept mappings take rows of 4096
    # entries and more item by item, with the in-row search)
    base = gg.rmat_graph(13, 12, seed=21)
    s0, d0 = base.edges()
    hub = np.random.default_rng(21).choice(base.n, 6000, replace=False).astype(np.int32)
    g0 = gg.from_edges(base.n, np.concatenate([s0, hub]),
                       np.concatenate([d0, np.full(hub.size, 5, np.int32)]))
    assert np.diff(g0.in_offsets).max() >= 6000
    b1 = gg.random_batch(g0, gg.batch_size_for(g0, 1e-3), seed=31)
    g1 = gg.apply_batch(g0, b1)
    prev0 = oracle.static(g0.n, *g0.edges()).ranks
    b2 = gg.random_batch(g1, gg.batch_size_for(g1, 1e-4), seed=22)
    g2 = gg.apply_batch(g1, b2)
    b3 = gg.random_batch(g2, gg.batch_size_for(g2, 3e-3), seed=23)
    g3 = gg.apply_batch(g2, b3)
    # the hub row changed within the chain, so its mapping needs the search
    assert np.diff(g3.in_offsets)[5] != np.diff(g1.in_offsets)[5]
    gr = gg.relabel(g3, np.random.default_rng(24).permutation(g3.n))
    br = gg.random_batch(gr, 40, seed=25)
    gr1 = gg.apply_batch(gr, br)
    gs = gg.rmat_graph(12, 12, seed=26)
    bs = gg.random_batch(gs, 30, seed=27)
    gs1 = gg.apply_batch(gs, bs)
    prev_s = oracle.static(gs.n, *gs.edges()).ranks
    # the rebuild rule: misses summed since the build <= 1/8 of its edges
    assert (row_aligned_misses(g1, g2) + row_aligned_misses(g2, g3)) * 8 <= g1.m
    assert row_aligned_misses(g3, gr1) * 8 > g1.m

    def run_chain(keep):
        prhip.set_tuning()
        prhip.set_tuning(**tuning, chain_numbering=keep)
        outs, prev = [], prev0
        steps = [(g1, b1), (g2, b2), (g3, b3), (gr1, br), (g3, b3), (gs1, bs)]
        for k, (g, b) in enumerate(steps):
            p = prev_s if g is gs1 else prev
            r, res = gpu_dfp(g, b, p, mode=mode)
            outs.append((r, res.iterations, prhip.last_stats()["numbering"]))
            if k < 2:
                prev = r  # R^t of the chain
        return outs

    fresh = run_chain(0)   # also releases anything kept by earlier tests
    kept = run_chain(1)
    auto = run_chain(-1)   # the default: below 2^23 vertices, built in each call
    for k, ((rf, itf, nf), (rk, itk, nk), (ra, ita, na)) in enumerate(zip(fresh, kept, auto)):
        assert nf == 1 and na == 1, k
        assert itf == itk == ita and np.array_equal(rf, rk) and np.array_equal(rf, ra), k
    assert [o[2] for o in kept] == [1, 2, 2, 2, 1, 1]
    # the chain's first step against the oracle
    o = oracle.dfp(g1.n, *g1.edges(), b1, prev0, prune=(mode == "dfp")) if mode != "dt" \
        else oracle.dt(g1.n, *g1.edges(), b1, prev0)
    assert np.abs(kept[0][0] - o.ranks).max() <= 1e-9


@pytest.mark.parametrize("mode", ["dfp", "df", "dt"])
@pytest.mark.parametrize("tuning", [dict(expand_lane_max_degree=2),
                                    dict(expand_lane_max_degree=2, xcd_split_degree=0)])
def test_initial_frontier_list_overflow(mode, tuning):
    """A batch of more updates than vertices: the initial frontier's list (an
    entry per batch edge whose source is in the out-degree wavefront class)
    would hold more than n entries, so the initial marking checks the whole
    class instead. Same bits and iterations as the ID-tile sweeps, and the
    oracle's ranks."""
    g0 = gg.rmat_graph(6, 12, seed=41)  # n = 64
    b = gg.random_batch(g0, 200, seed=42)
    g1 = gg.apply_batch(g0, b)
    prev = oracle.static(g0.n, *g0.edges()).ranks
    deg = np.diff(g1.out_offsets)
    src = np.concatenate([b.del_src, b.ins_src])
    assert ((deg[src] > 2) & (deg[src] <= 4096)).sum() > g1.n
    outs = []
    for fl in (0, 1):
        prhip.set_tuning()
        prhip.set_tuning(**tuning, frontier_list=fl)
        r, res = gpu_dfp(g1, b, prev, mode=mode)
        outs.append((r, res.iterations))
    assert outs[0][1] == outs[1][1] and np.array_equal(outs[0][0], outs[1][0])
    o = oracle.dt(g1.n, *g1.edges(), b, prev) if mode == "dt" else \
        oracle.dfp(g1.n, *g1.edges(), b, prev, prune=(mode == "dfp"))
    assert np.abs(outs[1][0] - o.ranks).max() <= 1e-9
