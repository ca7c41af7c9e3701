"""GPU weighted forward (pr_weighted), adjoint (pr_adjoint) and the autograd
Function, against the oracle, a dense LU gradient and central finite
differences."""
import numpy as np
import pytest

import oracle
from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2404_08299_amd import prhip  # noqa: E402
from paper_2404_08299_amd.autograd import pagerank  # noqa: E402

ALPHA = 0.85


@pytest.fixture(autouse=True)
def default_tuning():
    prhip.set_tuning()
    yield
    prhip.set_tuning()


def weighted_graph(scale, seed, ef=8):
    """Weights U(0.1, 1] per edge, row-normalised by the source's row sum;
    returned in in-CSR order together with that order's edge list."""
    g = gg.rmat_graph(scale, ef, seed=seed)
    dst = np.repeat(np.arange(g.n, dtype=np.int32), g.in_degree())
    src = g.in_sources.copy()
    w = gg.edge_weights(src, dst, seed=seed)
    W = np.bincount(src, weights=w, minlength=g.n)
    P = w / W[src]
    return g, src, dst, w, P


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("scale,relabel,tuning", [(11, 0, {}), (12, 1, {}),
                                                  (11, 1, dict(lane_max_degree=2,
                                                               wave_max_degree=16,
                                                               expand_lane_max_degree=2,
                                                               hub_chunk_edges=32,
                                                               xcd_split_degree=0)),
                                                  (11, 1, dict(xcd_split_degree=3,
                                                               hub_chunk_edges=4)),
                                                  (12, 0, dict(xcd_split_degree=2,
                                                               lane_max_degree=1,
                                                               grid_blocks=9))])
def test_weighted_forward_vs_oracle(scale, relabel, tuning):
    prhip.set_tuning(relabel=relabel, **tuning)
    g, src, dst, w, P = weighted_graph(scale, seed=scale)
    s = np.random.default_rng(1).random(g.n)
    s /= s.sum()
    dg = prhip.DeviceGraph.from_host(g)
    r = prhip.weighted(dg, cu(P), cu(s))
    o = oracle.weighted(g.n, src, dst, P, s)
    assert np.abs(r.ranks.cpu().numpy() - o.ranks).max() <= 1e-9
    assert abs(r.iterations - o.iters) <= 1


def test_weighted_bitwise_all_lane():
    prhip.set_tuning(lane_max_degree=1 << 30, wave_max_degree=1 << 30,
                     expand_lane_max_degree=1 << 30)
    g, src, dst, w, P = weighted_graph(10, seed=3)
    s = np.full(g.n, 1.0 / g.n)
    r = prhip.weighted(prhip.DeviceGraph.from_host(g), cu(P), cu(s))
    o = oracle.weighted(g.n, src, dst, P, s)
    assert r.iterations == o.iters and np.array_equal(r.ranks.cpu().numpy(), o.ranks)


def test_weighted_unit_weights_equal_static():
    g = gg.rmat_graph(11, 8, seed=4)
    dg = prhip.DeviceGraph.from_host(g)
    P = 1.0 / g.out_degree()[g.in_sources]
    r = prhip.weighted(dg, cu(P), None, tol=1e-14, max_iter=2000).ranks.cpu().numpy()
    st = prhip.static(dg, tol=1e-14, max_iter=2000).ranks.cpu().numpy()
    assert np.abs(r - st).max() <= 1e-14


@pytest.mark.parametrize("relabel,xsplit", [(0, 257), (1, 257), (1, 2), (0, 3)])
def test_adjoint_vs_oracle_and_dense(relabel, xsplit):
    prhip.set_tuning(relabel=relabel, xcd_split_degree=xsplit)
    g, src, dst, w, P = weighted_graph(9, seed=5)
    n = g.n
    s = np.full(n, 1.0 / n)
    dg = prhip.DeviceGraph.from_host(g)
    r = prhip.weighted(dg, cu(P), cu(s), tol=1e-15, max_iter=3000).ranks
    rng = np.random.default_rng(2)
    targets = rng.choice(n, 40, replace=False)
    gvec = np.zeros(n)
    rh = r.cpu().numpy()
    gvec[targets] = 2 * rh[targets]
    gw, gs, lam = prhip.adjoint(dg, cu(P), r, cu(gvec), tol=1e-15, max_iter=3000,
                                want_lambda=True)
    gw, gs, lam = gw.cpu().numpy(), gs.cpu().numpy(), lam.cpu().numpy()
    ow, os_, olam, oit = oracle.adjoint(n, src, dst, P, rh, gvec, tol=1e-15, max_iter=3000)
    scale = np.abs(olam).max()
    assert np.abs(lam - olam).max() <= 1e-12 * scale
    assert np.abs(gs - os_).max() <= 1e-12 * scale
    assert np.abs(gw - ow).max() <= 1e-12 * np.abs(ow).max()
    # dense: lambda = (I - alpha A^T)^{-1} g with A[v][u] = P_uv
    A = np.zeros((n, n))
    np.add.at(A, (dst.astype(np.int64), src.astype(np.int64)), P)
    lam_ref = np.linalg.solve((np.eye(n) - ALPHA * A).T, gvec)
    assert np.abs(lam - lam_ref).max() <= 1e-12 * scale


def test_autograd_matches_finite_differences():
    """Loss = sum of squared ranks of random targets; gradients with respect to
    the weights and the teleport vector through PageRankFn, against central
    differences (h = 1e-6) of forward solves run to 1e-15."""
    g, src, dst, w, P = weighted_graph(10, seed=6)
    n, m = g.n, g.m
    dg = prhip.DeviceGraph.from_host(g)
    rng = np.random.default_rng(3)
    targets = torch.from_numpy(rng.choice(n, 64, replace=False)).cuda()
    Pt = cu(P).requires_grad_(True)
    st = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda", requires_grad=True)
    r = pagerank(Pt, st, dg, tol=1e-15, max_iter=3000)
    loss = (r[targets] ** 2).sum()
    loss.backward()
    gP, gS = Pt.grad.cpu().numpy(), st.grad.cpu().numpy()

    def L(Pv, sv):
        rr = prhip.weighted(dg, cu(Pv), cu(sv), tol=1e-15, max_iter=3000).ranks
        return float((rr[targets] ** 2).sum())

    h = 1e-6
    s0 = np.full(n, 1.0 / n)
    for e in rng.choice(m, 24, replace=False):
        Pp, Pm = P.copy(), P.copy()
        Pp[e] += h
        Pm[e] -= h
        fd = (L(Pp, s0) - L(Pm, s0)) / (2 * h)
        assert abs(gP[e] - fd) <= 1e-5 * abs(fd) + 1e-9, (e, gP[e], fd)
    for v in rng.choice(n, 8, replace=False):
        sp, sm = s0.copy(), s0.copy()
        sp[v] += h
        sm[v] -= h
        fd = (L(P, sp) - L(P, sm)) / (2 * h)
        assert abs(gS[v] - fd) <= 1e-5 * abs(fd) + 1e-9, (v, gS[v], fd)


def test_autograd_through_row_normalisation():
    """Raw weights normalised in torch outside the Function: autograd adds
    the normalisation's chain rule (raw-weight gradients vs central FD)."""
    g, src, dst, w, P = weighted_graph(9, seed=7)
    n, m = g.n, g.m
    dg = prhip.DeviceGraph.from_host(g)
    srcs = torch.from_numpy(src.astype(np.int64)).cuda()
    rng = np.random.default_rng(4)
    targets = torch.from_numpy(rng.choice(n, 32, replace=False)).cuda()

    def loss_of(wraw):
        rowsum = torch.zeros(n, dtype=torch.float64, device="cuda").index_add_(0, srcs, wraw)
        Pn = wraw / rowsum[srcs]
        r = pagerank(Pn, None, dg, tol=1e-15, max_iter=3000)
        return (r[targets] ** 2).sum()

    wt = cu(w).requires_grad_(True)
    loss_of(wt).backward()
    gw = wt.grad.cpu().numpy()
    h = 1e-6
    for e in rng.choice(m, 16, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        with torch.no_grad():
            fd = (float(loss_of(cu(wp))) - float(loss_of(cu(wm)))) / (2 * h)
        assert abs(gw[e] - fd) <= 1e-5 * abs(fd) + 1e-9, (e, gw[e], fd)
