"""GPU personalised PageRank (pr_ppr) against the oracle: K teleport vectors,
each uniform over a set of seed vertices; per-vector convergence."""
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


def teleports(n, k, seeds_per, seed):
    sets = gg.distinct_vertices(n, k, seeds_per, seed=seed)
    T = np.zeros((n, k))
    for j in range(k):
        T[sets[j], j] = 1.0 / seeds_per
    return T


@pytest.mark.parametrize("xsplit", [129, 0])
@pytest.mark.parametrize("scale,k,relabel", [(11, 8, 0), (12, 64, 1), (10, 70, 0), (9, 1, 1)])
def test_ppr_vs_oracle(scale, k, relabel, xsplit):
    """Long rows (in-degree > 256) cut into 256-edge chunks, by source range
    first when the die split is on (xcd_split_degree > 0)."""
    prhip.set_tuning(relabel=relabel, xcd_split_degree=xsplit)
    g = gg.rmat_graph(scale, 8, seed=scale)
    T = teleports(g.n, k, min(16, g.n), seed=2)
    res, its = prhip.ppr(prhip.DeviceGraph.from_host(g), torch.from_numpy(T).cuda())
    R = res.ranks.cpu().numpy()
    Ro, ito = oracle.ppr(g.n, *g.edges(), T)
    assert res.converged
    assert np.abs(R - Ro).max() <= 1e-9
    assert np.abs(its - ito).max() <= 1


def test_ppr_bitwise_when_rows_are_short():
    """Rows of in-degree <= 256 are summed in row order: bit-identical."""
    g = gg.rmat_graph(10, 4, seed=3)
    assert g.in_degree().max() <= 256
    T = teleports(g.n, 16, 16, seed=4)
    res, its = prhip.ppr(prhip.DeviceGraph.from_host(g), torch.from_numpy(T).cuda())
    Ro, ito = oracle.ppr(g.n, *g.edges(), T)
    assert np.array_equal(its, ito)
    assert np.array_equal(res.ranks.cpu().numpy(), Ro)


def test_ppr_uniform_teleport_matches_static_and_linearity():
    g = gg.rmat_graph(12, 8, seed=5)
    dg = prhip.DeviceGraph.from_host(g)
    T = teleports(g.n, 3, 16, seed=6)
    T = np.concatenate([T, np.full((g.n, 1), 1.0 / g.n), 0.3 * T[:, :1] + 0.7 * T[:, 1:2]], axis=1)
    res, _ = prhip.ppr(dg, torch.from_numpy(np.ascontiguousarray(T)).cuda(), tol=1e-14,
                       max_iter=2000)
    R = res.ranks.cpu().numpy()
    st = prhip.static(dg, tol=1e-14, max_iter=2000).ranks.cpu().numpy()
    assert np.abs(R[:, 3] - st).max() <= 1e-13
    assert np.abs(R[:, 4] - (0.3 * R[:, 0] + 0.7 * R[:, 1])).max() <= 1e-13


@pytest.mark.parametrize("tuning", [dict(), dict(xcd_split_degree=0), dict(grid_blocks=5),
                                    dict(grid_blocks=13, relabel=1)])
def test_ppr_hub_rows_split(tuning):
    """In-star with a center of in-degree 3000 (> 256): chunked rows."""
    prhip.set_tuning(**tuning)
    k = 3000
    g = gg.from_edges(k + 1, np.arange(1, k + 1, dtype=np.int32), np.zeros(k, np.int32))
    T = teleports(g.n, 5, 4, seed=1)
    res, its = prhip.ppr(prhip.DeviceGraph.from_host(g), torch.from_numpy(T).cuda())
    Ro, ito = oracle.ppr(g.n, *g.edges(), T)
    assert np.abs(res.ranks.cpu().numpy() - Ro).max() <= 1e-12


def test_ppr_max_iter():
    g = gg.rmat_graph(9, 8, seed=7)
    T = teleports(g.n, 4, 8, seed=8)
    with pytest.warns(RuntimeWarning):
        res, its = prhip.ppr(prhip.DeviceGraph.from_host(g), torch.from_numpy(T).cuda(), tol=0.0,
                             max_iter=3)
    assert res.status == prhip.PR_NOT_CONVERGED and list(its) == [3] * 4
    Ro, _ = oracle.ppr(g.n, *g.edges(), T, tol=0.0, max_iter=3)
    assert np.abs(res.ranks.cpu().numpy() - Ro).max() <= 1e-15


@pytest.mark.parametrize("tuning", [dict(ppr_chunk_edges=16), dict(ppr_chunk_edges=64),
                                    dict(ppr_chunk_edges=1024, grid_blocks=13),
                                    dict(ppr_chunk_edges=64, xcd_split_degree=0),
                                    # a die-split threshold above the chunk size and a lane
                                    # class above it: PPR still splits every row longer than
                                    # the chunk, by source range
                                    dict(xcd_split_degree=1000),
                                    dict(lane_max_degree=512, relabel=1)])
def test_ppr_chunk_sizes(tuning):
    """Rows split at the tuned chunk size (ppr_chunk_edges), with and without
    the die split, on R-MAT plus an in-star hub of in-degree 3000: the
    oracle's ranks, and the vectors stop in the oracle's iteration."""
    prhip.set_tuning(**tuning)
    base = gg.rmat_graph(12, 16, seed=5)
    s0, d0 = base.edges()
    hub = np.random.default_rng(5).choice(base.n, 3000, replace=False).astype(np.int32)
    g = gg.from_edges(base.n, np.concatenate([s0, hub]),
                      np.concatenate([d0, np.full(hub.size, 7, np.int32)]))
    deg = np.diff(g.in_offsets)
    assert ((deg > 256) & (deg < 1000)).any() and deg.max() >= 3000
    T = teleports(g.n, 24, 16, seed=3)
    res, its = prhip.ppr(prhip.DeviceGraph.from_host(g), torch.from_numpy(T).cuda())
    Ro, ito = oracle.ppr(g.n, *g.edges(), T)
    assert np.abs(res.ranks.cpu().numpy() - Ro).max() <= 1e-9
    assert np.abs(np.asarray(its) - np.asarray(ito)).max() <= 1
