"""Generator invariants: the input contract of the paper (a self-loop on every
vertex, no duplicates, both CSR views consistent, Sec. 3.1 and 5.1.3) and
normalised batch updates (Sec. 3.3, 5.1.4)."""
import numpy as np
import pytest

from paper_2404_08299_amd import graphgen as gg


def check_canonical(g):
    n, m = g.n, g.m
    assert g.out_offsets[0] == 0 and g.out_offsets[-1] == m
    assert g.in_offsets[0] == 0 and g.in_offsets[-1] == m
    src, dst = g.edges()
    key = src.astype(np.int64) * n + dst
    assert np.all(np.diff(key) > 0), "rows sorted, no duplicates"
    assert int((src == dst).sum()) == n, "exactly one self-loop per vertex"
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.in_offsets))
    tkey = g.in_sources.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(tkey), key), "in-CSR is the transpose"
    # sources ascending within every in-row
    inner = np.diff(g.in_sources.astype(np.int64))
    row_start = np.zeros(m, bool)
    row_start[g.in_offsets[:-1][np.diff(g.in_offsets) > 0]] = True
    assert np.all((inner > 0) | row_start[1:])
    assert np.diff(g.out_offsets).sum() == m and np.diff(g.in_offsets).sum() == m


@pytest.mark.parametrize("scale,ef,scr", [(6, 4, True), (10, 8, True), (10, 8, False), (12, 16, True)])
def test_rmat_canonical(scale, ef, scr):
    g = gg.rmat_graph(scale, ef, seed=1, scramble=scr)
    check_canonical(g)
    assert g.n == 1 << scale and g.m <= ef * g.n + g.n


def test_rmat_deterministic():
    a = gg.rmat_graph(11, 8, seed=3)
    b = gg.rmat_graph(11, 8, seed=3)
    c = gg.rmat_graph(11, 8, seed=4)
    assert np.array_equal(a.in_sources, b.in_sources) and a.m == b.m
    assert not (a.m == c.m and np.array_equal(a.in_sources, c.in_sources))


def test_rmat_non_power_of_two():
    g = gg.rmat_graph(10, 8, seed=2, n=700)
    check_canonical(g)
    assert g.n == 700


def test_rmat_skew():
    g = gg.rmat_graph(14, 8, seed=1)
    d = g.in_degree()
    assert d.max() > 50 * d.mean()
    assert (d == 1).mean() > 0.2


def test_tiny_and_empty():
    g = gg.from_edges(1, [], [])
    check_canonical(g)
    assert g.m == 1
    g = gg.from_edges(3, [0, 0, 2, 0], [1, 1, 2, 2])
    check_canonical(g)
    assert g.m == 5


@pytest.mark.parametrize("frac", [1e-4, 1e-3, 1e-2])
def test_random_batch_normalised(frac):
    g = gg.rmat_graph(12, 8, seed=1)
    size = gg.batch_size_for(g, frac)
    b = gg.random_batch(g, size, seed=2)
    assert b.size == size and b.ins_src.size == round(0.8 * size)
    src, dst = g.edges()
    E = set(zip(src.tolist(), dst.tolist()))
    dels = list(zip(b.del_src.tolist(), b.del_dst.tolist()))
    ins = list(zip(b.ins_src.tolist(), b.ins_dst.tolist()))
    assert all(e in E and e[0] != e[1] for e in dels) and len(set(dels)) == len(dels)
    assert all(e not in E and e[0] != e[1] for e in ins) and len(set(ins)) == len(ins)
    g2 = gg.apply_batch(g, b)
    check_canonical(g2)
    s2, d2 = g2.edges()
    E2 = set(zip(s2.tolist(), d2.tolist()))
    assert E2 == (E - set(dels)) | set(ins)


def test_apply_batch_rejects_unnormalised():
    g = gg.rmat_graph(8, 4, seed=1)
    s, d = g.edges()
    bad = gg.Batch(np.zeros(0, np.int32), np.zeros(0, np.int32), s[:1].copy(), d[:1].copy())
    with pytest.raises(ValueError):
        gg.apply_batch(g, bad)


def test_pa_temporal():
    src, dst = gg.pa_temporal_events(20000, 400000, seed=1)
    assert src.size == 400000
    # while vertices arrive (sources non-decreasing), targets precede sources
    brk = np.nonzero(np.diff(src) < 0)[0]
    arrival = src.size if brk.size == 0 else brk[0] + 1
    assert arrival > src.size // 2
    assert np.all(dst[:arrival] < src[:arrival])
    g = gg.from_edges(20000, src, dst)
    check_canonical(g)
    indeg = g.in_degree()
    assert indeg.max() > 100 * np.median(indeg)


def test_temporal_stream_batches_are_set_differences():
    n, ev = 5000, 100000
    src, dst = gg.pa_temporal_events(n, ev, seed=4)
    g0, steps = gg.temporal_stream(n, ev, seed=4, batches=5)
    assert np.array_equal(g0.out_offsets, gg.from_edges(n, src[:90000], dst[:90000]).out_offsets)
    g = g0
    for t, (b, g1) in enumerate(steps):
        have = set(zip(*g.edges()))
        ins = list(zip(b.ins_src.tolist(), b.ins_dst.tolist()))
        dels = list(zip(b.del_src.tolist(), b.del_dst.tolist()))
        # insertions: the unique new non-self-loop pairs of the batch's events
        a, c = 90000 + 2000 * t, 90000 + 2000 * (t + 1)
        want = []
        for e in zip(src[a:c].tolist(), dst[a:c].tolist()):
            if e[0] != e[1] and e not in have and e not in want:
                want.append(e)
        assert ins == want
        assert len(dels) == 200 and len(set(dels)) == 200
        assert all(e in have and e[0] != e[1] for e in dels)
        new = set(zip(*g1.edges()))
        assert new == (have - set(dels)) | set(ins)
        check_canonical(g1)
        g = g1


def test_edge_weights_and_sets():
    g = gg.rmat_graph(8, 8, seed=1)
    s, d = g.edges()
    w = gg.edge_weights(s, d, seed=1)
    assert np.all((w > 0.1) & (w <= 1.0))
    # the weight is a function of the edge, not its position
    perm = np.random.default_rng(0).permutation(s.size)
    assert np.array_equal(gg.edge_weights(s[perm], d[perm], seed=1), w[perm])
    sets = gg.distinct_vertices(g.n, 4, 16, seed=2)
    assert all(len(set(r.tolist())) == 16 for r in sets)
