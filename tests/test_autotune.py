"""Autotuner search logic and cache (no GPU: the measurement is replaced by
a synthetic cost), plus the GPU check that a tuned call returns the same
ranks."""
import json

import numpy as np
import pytest

from paper_2404_08299_amd import autotune, prhip


@pytest.fixture(autouse=True)
def restore():
    prhip.set_tuning()
    yield
    prhip.set_tuning()


def test_size_class():
    assert autotune.size_class(1 << 24, 16 << 24) == "n2^24_d2^4"
    assert autotune.size_class(1000, 1000) == "n2^10_d2^0"


def test_coordinate_descent_finds_separable_minimum(monkeypatch):
    target = dict(lane_max_degree=64, wave_max_degree=16384, hub_chunk_edges=1024, relabel=1,
                  iters_per_sync=4, xcd_split_degree=257)

    def fake_score(run, tuning, k1, k2, expected, repeats=2):
        prhip.set_tuning(**tuning)  # the real score applies the candidate
        return 1.0 + sum(abs(np.log2(tuning[f] + 2) - np.log2(v + 2)) for f, v in target.items())

    monkeypatch.setattr(autotune, "score", fake_score)
    best, s = autotune.coordinate_descent(lambda k: None, autotune.DEFAULT_SPACE)
    for f, v in target.items():
        assert best[f] == v
    assert s == pytest.approx(1.0)
    assert prhip.get_tuning()["wave_max_degree"] == 16384


def test_coordinate_descent_skips_invalid(monkeypatch):
    calls = []

    def fake_score(run, tuning, k1, k2, expected, repeats=2):
        assert tuning["lane_max_degree"] <= tuning["wave_max_degree"]
        calls.append(dict(tuning))
        return float(tuning["wave_max_degree"])  # prefers the smallest wave threshold

    monkeypatch.setattr(autotune, "score", fake_score)
    # a wavefront threshold of 16 is below the default lane (32) and expand
    # (32) thresholds: never scored; the smallest valid one wins
    space = {"wave_max_degree": [16, 1024], "lane_max_degree": [8, 64]}
    best, _ = autotune.coordinate_descent(lambda k: None, space)
    assert best["wave_max_degree"] == 1024
    assert all(c["wave_max_degree"] != 16 for c in calls)


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "tune.json")
    tuned = dict(prhip.get_tuning(), lane_max_degree=8)
    calls = []

    def tune():
        calls.append(1)
        return tuned, 0.5

    got = autotune._cached("static", 1 << 20, 16 << 20, tune, path, False)
    assert got == tuned and len(calls) == 1
    got2 = autotune._cached("static", 1 << 20, 16 << 20, tune, path, False)
    assert got2 == tuned and len(calls) == 1  # served from the cache
    assert prhip.get_tuning()["lane_max_degree"] == 8
    data = json.load(open(path))
    assert "static:n2^20_d2^4" in data
    autotune._cached("static", 1 << 20, 16 << 20, tune, path, True)
    assert len(calls) == 2


@pytest.mark.gpu
def test_tuned_static_same_ranks(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08299_amd import graphgen as gg
    g = gg.rmat_graph(14, 8, seed=1)
    dg = prhip.DeviceGraph.from_host(g)
    ref = prhip.static(dg, tol=1e-13, max_iter=1000).ranks.clone()
    best = autotune.tune_static(dg, cache_path=str(tmp_path / "t.json"))
    assert prhip.get_tuning() == best
    got = prhip.static(dg, tol=1e-13, max_iter=1000).ranks
    assert float((got - ref).abs().max()) <= 1e-13


def test_ppr_space_is_valid():
    """Every value of the PPR search space is a tuning the library accepts,
    and the space's fields are tuning fields."""
    for field, values in autotune.PPR_SPACE.items():
        assert field in prhip.TUNING_FIELDS
        for v in values:
            prhip.set_tuning(**{field: v})
            assert prhip.get_tuning()[field] == v
            prhip.set_tuning()


@pytest.mark.gpu
def test_tuned_ppr_same_ranks(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_08299_amd import graphgen as gg
    g = gg.rmat_graph(13, 8, seed=2)
    dg = prhip.DeviceGraph.from_host(g)
    sets = gg.distinct_vertices(g.n, 8, 16, seed=3)
    T = np.zeros((g.n, 8))
    for j in range(8):
        T[sets[j], j] = 1.0 / 16
    Td = torch.from_numpy(T).cuda()
    ref = prhip.ppr(dg, Td, tol=1e-13, max_iter=1000)[0].ranks.clone()
    best = autotune.tune_ppr(dg, Td, cache_path=str(tmp_path / "t.json"))
    assert prhip.get_tuning() == best
    got = prhip.ppr(dg, Td, tol=1e-13, max_iter=1000)[0].ranks
    assert float((got - ref).abs().max()) <= 1e-13
