"""Parity at full size: R-MAT scale 24, edge factor 16, seed 1, scrambled IDs
(n = 16,777,216, m = 280,209,285), with the default tuning and launch shape
the benchmark times.

Static is compared element by element with the oracle's whole run (Alg. 1,
about 61 x 2.8e8 edge steps, a minute or two on one host core). It is also
checked one step at a time on samples: the GPU
iterate R_k (a run stopped after k iterations) fed to the oracle's Eq. 1 for
a sample of rows (every degree class, the largest hubs, random rows) must give
the GPU's R_{k+1} on those rows within the rounding bound of a sum of
positive terms in any order, 2 (deg + 2) u with u = 2^-53, relative. The
converged ranks are checked by properties that hold at any size: they sum to
1 and none is below (1 - alpha)/N.

DF-P is checked element by element against the oracle's whole DF-P run from
the same previous ranks, for the batch decades where that run takes seconds,
and for every decade against a Static recompute of G^t within 1e-8 (DF-P's
accepted error, Sec. 5.3). The batches are the benchmark's: seed j + 1 for the
j-th decade, 80 % insertions.
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
FRACS = [1e-7, 1e-6, 1e-5, 1e-4, 1e-3]


@pytest.fixture(scope="module")
def full():
    prhip.set_tuning()
    g = gg.rmat_graph(24, 16, seed=1)
    print(f"scale 24: n={g.n} m={g.m}", flush=True)
    dg = prhip.DeviceGraph.from_host(g)
    res = prhip.static(dg)
    assert res.converged
    yield g, dg, res
    prhip.set_tuning()


def sample_rows(g, seed=0):
    """The largest hubs, rows on both sides of every class boundary of the
    default tuning (lane up to 128, die split from 129), and random rows."""
    d = g.in_degree()
    rng = np.random.default_rng(seed)
    picks = [np.argsort(-d, kind="stable")[:256], [0, g.n - 1], rng.choice(g.n, 4096, replace=False)]
    for lo, hi in [(1, 1), (2, 32), (33, 127), (128, 128), (129, 129), (130, 1024),
                   (1025, 4096), (4097, 1 << 30)]:
        cand = np.flatnonzero((d >= lo) & (d <= hi))
        if cand.size:
            picks.append(rng.choice(cand, min(256, cand.size), replace=False))
    return np.unique(np.concatenate(picks)).astype(np.int32)


def stopped_after(dg, k):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        res = prhip.static(dg, tol=0.0, max_iter=k)
    assert res.iterations == k
    return res.ranks.cpu().numpy()


def test_static_full_size_sampled_steps(full):
    g, dg, _ = full
    rows = sample_rows(g)
    deg = g.in_degree()[rows].astype(np.float64)
    iterate = {0: np.full(g.n, 1.0 / g.n)}
    for k in (1, 2, 3, 30, 31):
        prev = iterate.get(k - 1)
        if prev is None:
            prev = stopped_after(dg, k - 1)
        cur = iterate[k] = stopped_after(dg, k)
        o = oracle.static_rows(g.n, g.in_offsets, g.in_sources, g.out_offsets, prev, rows)
        rel = np.abs(cur[rows] - o) / o
        bound = 2 * (deg + 2) * U
        print(f"step {k - 1} -> {k}: {rows.size} rows, max rel diff {rel.max():.2e}, "
              f"max rel/bound {(rel / bound).max():.3f}", flush=True)
        assert (rel <= bound).all(), rows[np.argmax(rel / bound)]


def test_static_full_size_whole_run_vs_oracle(full):
    """The converged Static vector against the oracle's whole Static run over
    the same in-CSR (Alg. 1, Eq. 1, tol 1e-10): L-infinity <= 1e-9 and the
    same iteration count up to one (Delta can land within rounding of tol)."""
    g, _, res = full
    print("oracle Static over the scale-24 CSR (one host core) ...", flush=True)
    o, sec = oracle.static_csr(g.n, g.in_offsets, g.in_sources, g.out_offsets)
    r = res.ranks.cpu().numpy()
    err = float(np.abs(r - o.ranks).max())
    rel = float((np.abs(r - o.ranks) / o.ranks).max())
    print(f"Static whole run: gpu iters {res.iterations} oracle iters {o.iters} "
          f"({sec:.1f} s), Linf {err:.2e}, max rel {rel:.2e}", flush=True)
    assert o.status == oracle.OK
    assert err <= 1e-9
    assert abs(res.iterations - o.iters) <= 1


def test_static_full_size_invariants(full):
    g, dg, res = full
    r = res.ranks.cpu().numpy()
    print(f"Static: {res.iterations} iterations, delta {res.final_delta:.2e}", flush=True)
    assert 50 <= res.iterations <= 80 and res.final_delta <= 1e-10
    assert abs(math.fsum(r) - 1.0) <= 1e-9
    assert r.min() >= (1 - ALPHA) / g.n * (1 - 1e-12)
    # deterministic: a second run gives the same bits
    assert torch.equal(prhip.static(dg).ranks, res.ranks)


def batch_of(g, j):
    return gg.random_batch(g, gg.batch_size_for(g, FRACS[j]), seed=j + 1)


@pytest.mark.parametrize("j", [0, 1, 2])
def test_dfp_full_size_vs_oracle(full, j):
    g, _, res = full
    b = batch_of(g, j)
    g1 = gg.apply_batch(g, b)
    prev = res.ranks
    d = prhip.dfp(prhip.DeviceGraph.from_host(g1), prhip.DeviceBatch.from_host(b), prev)
    o = oracle.dfp_csr(g1, b, prev.cpu().numpy())
    err = float(np.abs(d.ranks.cpu().numpy() - o.ranks).max())
    print(f"DF-P {FRACS[j]:g}|E| ({b.size} updates): gpu iters {d.iterations}, oracle iters "
          f"{o.iters}, affected max {o.stats['affected_max']}, Linf {err:.2e}", flush=True)
    assert d.converged and o.status == oracle.OK
    assert err <= 1e-9
    assert abs(d.iterations - o.iters) <= 1


@pytest.mark.parametrize("j", range(len(FRACS)))
def test_dfp_full_size_vs_static(full, j):
    g, dg, res = full
    db = prhip.DeviceBatch.from_host(batch_of(g, j))
    dg1 = prhip.apply_batch(dg, db)
    d = prhip.dfp(dg1, db, res.ranks)
    s = prhip.static(dg1)
    err = float((d.ranks - s.ranks).abs().max())
    print(f"DF-P {FRACS[j]:g}|E|: {d.iterations} iterations, |DF-P - Static| {err:.2e}", flush=True)
    assert d.converged and err <= 1e-8


def test_apply_full_size_vs_host(full):
    """The batch applied on the device (both views) equals the host merge at
    scale 24, where rows reach 2.4e5 entries, for the largest decade."""
    g, dg, _ = full
    b = batch_of(g, len(FRACS) - 1)
    new = prhip.apply_batch(dg, prhip.DeviceBatch.from_host(b))
    h = gg.apply_batch(g, b)
    assert new.m == h.m
    for dev, host in ((new.in_offsets, h.in_offsets), (new.in_sources, h.in_sources),
                      (new.out_offsets, h.out_offsets), (new.out_targets, h.out_targets)):
        assert np.array_equal(dev.cpu().numpy(), host)
