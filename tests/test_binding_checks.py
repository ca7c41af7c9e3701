"""The binding's argument checks, on the CPU: the C ABI receives raw data
pointers, so every tensor is checked for kind, place, layout and size before
one is handed over. These checks need no GPU (they run on CPU tensors here);
tests/test_gpu_binding_checks.py drives the same refusals through every entry
point on a GPU."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2404_08299_amd import graphgen as gg  # noqa: E402
from paper_2404_08299_amd import prhip  # noqa: E402

CPU = torch.device("cpu")


def test_tensor_check_accepts_the_expected_kind():
    x = torch.zeros(6, dtype=torch.float64)
    assert prhip._tensor(x, "x", torch.float64, CPU, numel=6) is x
    y = torch.zeros((3, 2), dtype=torch.float64)
    assert prhip._tensor(y, "y", torch.float64, CPU, shape=(3, 2)) is y


@pytest.mark.parametrize("bad, exc, words", [
    (np.zeros(6), TypeError, "torch tensor"),
    (torch.zeros(6, dtype=torch.float32), TypeError, "float64"),
    (torch.zeros(7, dtype=torch.float64), ValueError, "6 elements"),
    (torch.zeros(12, dtype=torch.float64)[::2], ValueError, "contiguous"),
])
def test_tensor_check_refuses(bad, exc, words):
    with pytest.raises(exc, match=words):
        prhip._tensor(bad, "x", torch.float64, CPU, numel=6)


def test_tensor_check_refuses_another_device():
    x = torch.zeros(6, dtype=torch.float64)
    with pytest.raises(ValueError, match="expected a tensor on"):
        prhip._tensor(x, "x", torch.float64, torch.device("cuda", 0), numel=6)


def host_graph():
    g = gg.rmat_graph(6, 4, seed=1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32))
    return g, prhip.DeviceGraph(g.n, g.m, t(g.in_offsets), t(g.in_sources), t(g.out_offsets),
                                t(g.out_targets))


def test_graph_view_checks_its_arrays():
    g, dg = host_graph()
    csr = dg.csr()
    assert (csr.n, csr.m) == (g.n, g.m)
    dg.in_sources = dg.in_sources.to(torch.int64)
    with pytest.raises(TypeError, match="in_sources"):
        dg.csr()
    _, dg = host_graph()
    dg.in_offsets = dg.in_offsets[:-1]
    with pytest.raises(ValueError, match="in_offsets"):
        dg.csr()
    _, dg = host_graph()
    dg.out_targets = dg.out_targets[1:]
    with pytest.raises(ValueError, match="out_targets"):
        dg.csr()
    _, dg = host_graph()
    dg.out_offsets = None
    dg.out_targets = None
    dg.csr()  # the out view is optional (pr_static reads out_offsets only when present)


def test_batch_view_checks_its_arrays():
    i32 = lambda *v: torch.tensor(v, dtype=torch.int32)
    b = prhip.DeviceBatch(i32(1, 2), i32(3, 4), i32(5), i32(6))
    de, ie = b.edges()
    assert (de.count, ie.count) == (2, 1)
    b = prhip.DeviceBatch(i32(1, 2), i32(3), i32(5), i32(6))
    with pytest.raises(ValueError, match="del_dst"):
        b.edges()
    b = prhip.DeviceBatch(i32(1), i32(3), torch.tensor([5], dtype=torch.int64), i32(6))
    with pytest.raises(TypeError, match="ins_src"):
        b.edges()
    empty = torch.zeros(0, dtype=torch.int32)
    de, ie = prhip.DeviceBatch(empty, empty, empty, empty).edges()
    assert de.count == 0 and de.src is None and ie.count == 0
