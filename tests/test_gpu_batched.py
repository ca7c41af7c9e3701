"""GPU batched Static PageRank (pr_static_batched): every graph with the
uniform teleport term is bit-identical to pr_static on that graph alone (same
tuning) and within 1e-9 of the oracle; graphs with a personalised teleport
vector match the oracle's personalised PageRank within 1e-9."""
import numpy as np
import pytest

import oracle
from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2404_08299_amd import prhip  # noqa: E402


@pytest.fixture(autouse=True)
def default_tuning():
    prhip.set_tuning()
    yield
    prhip.set_tuning()


def make_batch(count, seed):
    rng = np.random.default_rng(seed)
    gs = []
    for i in range(count):
        n = int(2 ** rng.uniform(4, 14))
        ef = float(rng.uniform(2, 16))
        scale = max(1, int(np.ceil(np.log2(n))))
        gs.append(gg.rmat_graph(scale, ef, seed=1000 + i, n=n))
    return gs


@pytest.mark.parametrize("tuning", [dict(), dict(relabel=1),
                                    dict(lane_max_degree=2, wave_max_degree=16,
                                         expand_lane_max_degree=2, hub_chunk_edges=32,
                                         relabel=1, xcd_split_degree=0),
                                    dict(xcd_split_degree=4, hub_chunk_edges=8, relabel=1),
                                    dict(xcd_split_degree=2, lane_max_degree=1, grid_blocks=6)])
def test_batched_equals_per_graph(tuning):
    prhip.set_tuning(**tuning)
    gs = make_batch(24, seed=1)
    dgs = [prhip.DeviceGraph.from_host(g) for g in gs]
    res, its = prhip.static_batched(dgs)
    assert res.converged
    for g, dg, r, it in zip(gs, dgs, res.ranks, its):
        single = prhip.static(dg)
        assert single.iterations == it
        assert torch.equal(single.ranks, r)
    for g, r in zip(gs[:6], res.ranks[:6]):
        o = oracle.static(g.n, *g.edges())
        assert np.abs(r.cpu().numpy() - o.ranks).max() <= 1e-9


def test_batched_with_hubs_and_single():
    k = 5000
    star = gg.from_edges(k + 1, np.arange(1, k + 1, dtype=np.int32), np.zeros(k, np.int32))
    gs = [star, gg.rmat_graph(12, 8, seed=3), gg.from_edges(1, [], [])]
    dgs = [prhip.DeviceGraph.from_host(g) for g in gs]
    res, its = prhip.static_batched(dgs)
    for dg, r, it in zip(dgs, res.ranks, its):
        single = prhip.static(dg)
        assert single.iterations == it and torch.equal(single.ranks, r)
    one, its1 = prhip.static_batched(dgs[1:2])
    assert torch.equal(one.ranks[0], prhip.static(dgs[1]).ranks)


@pytest.mark.parametrize("max_iter", [1, 4, 7])
def test_batched_iteration_cap(max_iter):
    gs = make_batch(5, seed=2)
    dgs = [prhip.DeviceGraph.from_host(g) for g in gs]
    with pytest.warns(RuntimeWarning):
        res, its = prhip.static_batched(dgs, tol=0.0, max_iter=max_iter)
    assert res.status == prhip.PR_NOT_CONVERGED and list(its) == [max_iter] * 5
    for g, r in zip(gs, res.ranks):
        o = oracle.static(g.n, *g.edges(), tol=0.0, max_iter=max_iter)
        assert np.abs(r.cpu().numpy() - o.ranks).max() <= 1e-15


def seed_teleport(n, seeds, seed):
    t = np.zeros(n)
    t[gg.distinct_vertices(n, 1, seeds, seed=seed)[0]] = 1.0 / seeds
    return t


@pytest.mark.parametrize("tuning", [dict(), dict(relabel=1, xcd_split_degree=4, hub_chunk_edges=8),
                                    dict(relabel=0, xcd_split_degree=0)])
def test_batched_with_teleports_vs_oracle(tuning):
    """Graphs and personalised vectors in one call. One graph is passed four
    times, each with its own teleport vector (uniform over 16 seed vertices),
    another with a dense non-uniform teleport, the rest with the uniform term.
    Each personalised result matches the oracle's personalised PageRank
    within 1e-9 (iterations within one); the uniform graphs stay bit-identical
    to pr_static; a second call of the same shape with other vectors (the
    kept iteration graph updated in place) matches the oracle as well."""
    prhip.set_tuning(**tuning)
    gs = make_batch(6, seed=3)
    hub = gg.rmat_graph(12, 16, seed=9)
    dg_hub = prhip.DeviceGraph.from_host(hub)
    dgs = [prhip.DeviceGraph.from_host(g) for g in gs]
    rng = np.random.default_rng(4)
    dense = rng.uniform(0.5, 1.5, gs[2].n)
    dense /= dense.sum()

    for call in range(2):
        tele_h = [seed_teleport(hub.n, 16, seed=10 * call + j) for j in range(4)]
        graphs = dgs[:2] + [dg_hub] * 4 + dgs[2:]
        hosts = gs[:2] + [hub] * 4 + gs[2:]
        tele = [None, None] + [torch.from_numpy(t).cuda() for t in tele_h] + \
            [torch.from_numpy(dense if call == 0 else dense[::-1].copy()).cuda()] + [None] * 3
        res, its = prhip.static_batched(graphs, teleports=tele)
        assert res.converged
        for i, (h, dg, t, r, it) in enumerate(zip(hosts, graphs, tele, res.ranks, its)):
            if t is None:
                single = prhip.static(dg)
                assert single.iterations == it and torch.equal(single.ranks, r), i
                continue
            Ro, ito = oracle.ppr(h.n, *h.edges(), t.cpu().numpy())
            err = float(np.abs(r.cpu().numpy() - Ro[:, 0]).max())
            print(f"call {call} graph {i}: n={h.n} iters gpu {it} oracle {ito[0]} Linf {err:.2e}",
                  flush=True)
            assert err <= 1e-9 and abs(int(it) - int(ito[0])) <= 1, i


def test_batched_teleports_all_none_is_uniform():
    gs = make_batch(4, seed=5)
    dgs = [prhip.DeviceGraph.from_host(g) for g in gs]
    a, ia = prhip.static_batched(dgs)
    b, ib = prhip.static_batched(dgs, teleports=[None] * 4)
    assert list(ia) == list(ib)
    for x, y in zip(a.ranks, b.ranks):
        assert torch.equal(x, y)
