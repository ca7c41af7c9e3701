"""Every entry point of the binding refuses, with TypeError or ValueError and
before the library is called, tensors that are of the wrong kind, on the
host, strided or of the wrong size, so no such pointer reaches a kernel."""
import numpy as np
import pytest

from paper_2404_08299_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_08299_amd import prhip  # noqa: E402


@pytest.fixture(scope="module")
def case():
    g = gg.rmat_graph(8, 8, seed=1)
    dg = prhip.DeviceGraph.from_host(g)
    b = gg.random_batch(g, 6, seed=2)
    g1 = gg.apply_batch(g, b)
    return g, dg, prhip.DeviceGraph.from_host(g1), prhip.DeviceBatch.from_host(b)


def f64(n, device="cuda"):
    return torch.zeros(n, dtype=torch.float64, device=device)


def test_static_refuses_bad_outputs(case):
    g, dg, _, _ = case
    with pytest.raises(ValueError, match="out"):
        prhip.static(dg, out=f64(g.n, "cpu"))
    with pytest.raises(TypeError, match="out"):
        prhip.static(dg, out=torch.zeros(g.n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="out"):
        prhip.static(dg, out=f64(g.n + 1))
    with pytest.raises(ValueError, match="contiguous"):
        prhip.static(dg, out=f64(2 * g.n)[::2])
    # the same call with a good output still works
    assert prhip.static(dg, out=f64(g.n)).converged


def test_dfp_refuses_bad_inputs(case):
    g, dg, dg1, db = case
    prev = prhip.static(dg).ranks
    with pytest.raises(ValueError, match="ranks_prev"):
        prhip.dfp(dg1, db, prev[:-1].clone())
    with pytest.raises(ValueError, match="ranks_prev"):
        prhip.dfp(dg1, db, prev.cpu())
    with pytest.raises(ValueError, match="mode"):
        prhip.dfp(dg1, db, prev, mode="push")
    bad = prhip.DeviceBatch(db.del_src, db.del_dst[:-1], db.ins_src, db.ins_dst)
    with pytest.raises(ValueError, match="del_dst"):
        prhip.dfp(dg1, bad, prev)
    assert prhip.dfp(dg1, db, prev).converged


def test_apply_batch_refuses_host_batches(case):
    g, dg, _, db = case
    host = prhip.DeviceBatch(db.del_src.cpu(), db.del_dst.cpu(), db.ins_src.cpu(),
                             db.ins_dst.cpu())
    with pytest.raises(ValueError, match="del_src"):
        prhip.apply_batch(dg, host)


def test_ppr_refuses_bad_teleports(case):
    g, dg, _, _ = case
    with pytest.raises(ValueError, match="teleport"):
        prhip.ppr(dg, torch.zeros((g.n - 1, 4), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="teleport"):
        prhip.ppr(dg, torch.zeros((g.n, 4), dtype=torch.float64))
    tele = torch.full((g.n, 4), 1.0 / g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="out"):
        prhip.ppr(dg, tele, out=torch.zeros((g.n, 3), dtype=torch.float64, device="cuda"))


def test_batched_refuses_bad_outputs(case):
    g, dg, dg1, _ = case
    with pytest.raises(ValueError, match="at least one"):
        prhip.static_batched([])
    with pytest.raises(ValueError, match="outs"):
        prhip.static_batched([dg, dg1], outs=[f64(g.n)])
    with pytest.raises(ValueError, match="outs"):
        prhip.static_batched([dg, dg1], outs=[f64(g.n), f64(g.n - 1)])


def test_weighted_and_adjoint_refuse_bad_sizes(case):
    g, dg, _, _ = case
    w = torch.rand(g.m, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="in_weights"):
        prhip.weighted(dg, w[:-1].clone())
    with pytest.raises(ValueError, match="teleport"):
        prhip.weighted(dg, w, teleport=f64(g.n - 1))
    r = f64(g.n)
    with pytest.raises(ValueError, match="grad_ranks"):
        prhip.adjoint(dg, w, r, f64(g.n + 1))
    with pytest.raises(ValueError, match="ranks"):
        prhip.adjoint(dg, w, f64(g.n, "cpu"), f64(g.n))


def test_graph_arrays_are_checked(case):
    g, dg, _, _ = case
    bad = prhip.DeviceGraph(g.n, g.m, dg.in_offsets, dg.in_sources.to(torch.int64),
                            dg.out_offsets, dg.out_targets)
    with pytest.raises(TypeError, match="in_sources"):
        prhip.static(bad)
    bad = prhip.DeviceGraph(g.n, g.m + 1, dg.in_offsets, dg.in_sources, dg.out_offsets,
                            dg.out_targets)
    with pytest.raises(ValueError, match="in_sources"):
        prhip.static(bad)
    mixed = prhip.DeviceGraph(g.n, g.m, dg.in_offsets, dg.in_sources.cpu(), dg.out_offsets,
                              dg.out_targets)
    with pytest.raises(ValueError, match="in_sources"):
        prhip.validate(mixed)


def test_c_abi_refuses_host_outputs(case):
    """Straight through the C ABI (no binding checks): a device graph with a
    pageable or pinned host output array gets PR_EINVAL, and no kernel runs."""
    import ctypes
    g, dg, _, _ = case
    lib = prhip.load_library()
    csr = dg.csr()
    host = np.zeros(g.n)
    pinned = torch.zeros(g.n, dtype=torch.float64).pin_memory()
    for addr in (host.ctypes.data, pinned.data_ptr()):
        rc = lib.pr_static(ctypes.byref(csr), 0.85, 1e-10, 500, ctypes.c_void_p(addr))
        assert rc == prhip.PR_EINVAL
        assert b"ranks_out is not device memory" in lib.pr_last_error()
    assert np.all(host == 0.0) and bool((pinned == 0).all())
    # the library is still usable afterwards
    assert prhip.static(dg).converged
