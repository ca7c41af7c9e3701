"""The CPU oracle against facts fixed outside it (tests/pins.py)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin, lib):
    pin(lib)


def test_static_csr_entry_matches(lib):
    """The CSR entry point runs the same iteration: bit-identical ranks."""
    from paper_2404_08299_amd import graphgen as gg
    import numpy as np
    g = gg.rmat_graph(11, 8, seed=3)
    a = oracle.static(g.n, *g.edges(), lib=lib)
    b, sec = oracle.static_csr(g.n, g.in_offsets, g.in_sources, g.out_offsets, lib=lib)
    assert a.iters == b.iters and np.array_equal(a.ranks, b.ranks) and sec > 0
