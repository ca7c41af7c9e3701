"""Batch application on the device (pr_apply_batch): G^t = G^{t-1} minus the
deletions plus the insertions, both CSR views. The expected graph has a plain
definition, the sorted edge set (E - D) | I, built here with numpy; the host
generator's own merge is a second, independent check."""
import numpy as np
import pytest

from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_08299_amd import prhip  # noqa: E402


def expected(g, b):
    s, d = g.edges()
    keep = set(zip(s.tolist(), d.tolist())) - set(zip(b.del_src.tolist(), b.del_dst.tolist()))
    edges = np.array(sorted(keep | set(zip(b.ins_src.tolist(), b.ins_dst.tolist()))), np.int64)
    src, dst = edges[:, 0], edges[:, 1]
    o_in = np.lexsort((src, dst))
    o_out = np.lexsort((dst, src))
    in_off = np.concatenate([[0], np.cumsum(np.bincount(dst, minlength=g.n))])
    out_off = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=g.n))])
    return in_off, src[o_in], out_off, dst[o_out]


def check(g, b, out_view=True):
    dg = prhip.DeviceGraph.from_host(g)
    new = prhip.apply_batch(dg, prhip.DeviceBatch.from_host(b), out_view=out_view)
    in_off, in_src, out_off, out_tgt = expected(g, b)
    assert new.m == in_src.size
    assert np.array_equal(new.in_offsets.cpu().numpy(), in_off)
    assert np.array_equal(new.in_sources.cpu().numpy(), in_src)
    if out_view:
        assert np.array_equal(new.out_offsets.cpu().numpy(), out_off)
        assert np.array_equal(new.out_targets.cpu().numpy(), out_tgt)
    h = gg.apply_batch(g, b)
    assert np.array_equal(new.in_sources.cpu().numpy(), h.in_sources)
    return new


@pytest.mark.parametrize("frac,ins", [(1e-3, 0.8), (1e-2, 0.8), (5e-2, 0.5), (1e-2, 1.0), (1e-2, 0.0)])
def test_random_batches(frac, ins):
    g = gg.rmat_graph(12, 8, seed=3)
    b = gg.random_batch(g, gg.batch_size_for(g, frac), seed=5, insert_frac=ins)
    check(g, b)


@pytest.mark.parametrize("n,size", [(70001, 30000), (300, 2500), (1 << 16, 12289)])
def test_batches_over_many_sort_tiles(n, size):
    """Batches of several 4096-key tiles of the batch sort, with IDs of 17, 9
    and 16 bits (the sort covers only the digits IDs below n can set)."""
    scale = int(np.ceil(np.log2(n)))
    g = gg.rmat_graph(scale, 10, seed=n, n=n)
    b = gg.random_batch(g, size, seed=n + 1, insert_frac=0.7)
    check(g, b)


def test_hub_rows_empty_batch_and_in_view_only():
    k = 5000  # in-star and out-star hubs: rows longer than one lane copies
    src = np.concatenate([np.arange(1, k + 1), np.zeros(k, np.int64)]).astype(np.int32)
    dst = np.concatenate([np.zeros(k, np.int64), np.arange(k + 1, 2 * k + 1)]).astype(np.int32)
    g = gg.from_edges(2 * k + 1, src, dst)
    b = gg.Batch(np.array([5, 0, 0], np.int32), np.array([0, k + 7, 2 * k], np.int32),
                 np.array([0, 3, 9000, 0], np.int32), np.array([2, 7, 0, 4000], np.int32))
    check(g, b)
    check(g, gg.Batch.empty())
    check(g, b, out_view=False)


def test_rows_over_many_chunks():
    """Rows of 20000 entries span several 4096-entry chunks of the long-row
    pass: an unchanged in-hub, and an out-hub whose deletions and insertions
    fall in different chunks, plus a changed row that starts inside a chunk."""
    k = 20000
    hub_in = np.arange(1, k + 1)
    hub_out = np.arange(k + 1, 2 * k + 1)
    src = np.concatenate([hub_in, np.zeros(k, np.int64), [1] * 4500]).astype(np.int32)
    dst = np.concatenate([np.zeros(k, np.int64), hub_out, np.arange(2 * k + 2, 2 * k + 4502)]).astype(np.int32)
    g = gg.from_edges(2 * k + 4502, src, dst)
    ins_dst = np.array([1, 5, 4100, 9000, 2 * k + 1], np.int32)  # out-row 0: new targets (absent)
    del_dst = np.array([k + 1, k + 4097, k + 9000, 2 * k], np.int32)
    b = gg.Batch(np.concatenate([np.zeros(del_dst.size, np.int32), [1, 1]]).astype(np.int32),
                 np.concatenate([del_dst, [2 * k + 2, 2 * k + 4000]]).astype(np.int32),
                 np.concatenate([np.zeros(ins_dst.size, np.int32), [1]]).astype(np.int32),
                 np.concatenate([ins_dst, [3]]).astype(np.int32))
    check(g, b)
    check(g, gg.Batch.empty())


def test_temporal_chain_on_device():
    g0, steps = gg.temporal_stream(20000, 300000, seed=9, batches=5)
    dg = prhip.DeviceGraph.from_host(g0)
    for b, g in steps:
        dg = prhip.apply_batch(dg, prhip.DeviceBatch.from_host(b))
        assert np.array_equal(dg.in_sources.cpu().numpy(), g.in_sources)
        assert np.array_equal(dg.out_offsets.cpu().numpy(), g.out_offsets)
        assert np.array_equal(dg.out_targets.cpu().numpy(), g.out_targets)


def test_invalid_batches_rejected():
    g = gg.rmat_graph(9, 8, seed=4)
    s, d = g.edges()
    present = (int(s[s != d][0]), int(d[s != d][0]))
    dg = prhip.DeviceGraph.from_host(g)
    absent = None
    have = set(zip(s.tolist(), d.tolist()))
    for u in range(g.n):
        if (u, (u + 1) % g.n) not in have:
            absent = (u, (u + 1) % g.n)
            break
    z = np.zeros(0, np.int32)
    a = lambda *x: np.array(x, np.int32)
    bad = [gg.Batch(a(absent[0]), a(absent[1]), z, z),                      # deletion absent
           gg.Batch(z, z, a(present[0]), a(present[1])),                    # insertion present
           gg.Batch(z, z, a(absent[0], absent[0]), a(absent[1], absent[1])),  # repeated pair
           gg.Batch(z, z, a(absent[0]), a(g.n + 3))]                         # ID out of range
    for b in bad:
        with pytest.raises(prhip.PrError) as ei:
            prhip.apply_batch(dg, prhip.DeviceBatch.from_host(b))
        assert ei.value.code == prhip.PR_EBATCH
    check(g, gg.Batch(z, z, a(absent[0]), a(absent[1])))  # the library still works


def test_dfp_on_device_applied_graph():
    g0 = gg.rmat_graph(12, 8, seed=6)
    b = gg.random_batch(g0, gg.batch_size_for(g0, 1e-3), seed=2)
    dg0 = prhip.DeviceGraph.from_host(g0)
    prev = prhip.static(dg0).ranks
    db = prhip.DeviceBatch.from_host(b)
    on_dev = prhip.dfp(prhip.apply_batch(dg0, db), db, prev).ranks
    on_host = prhip.dfp(prhip.DeviceGraph.from_host(gg.apply_batch(g0, b)), db, prev).ranks
    assert torch.equal(on_dev, on_host)
