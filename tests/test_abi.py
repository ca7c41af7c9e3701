"""The C-ABI library loads and exports every symbol include/prhip.h declares,
and argument validation answers before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2404_08299_amd import prhip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prhip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return prhip.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(prhip.EXPORTED) == sorted(names)


def test_status_codes_match_header():
    text = open(HEADER).read()
    for name, val in [("PR_OK", 0), ("PR_NOT_CONVERGED", 1), ("PR_EINVAL", -1),
                      ("PR_EGRAPH", -2), ("PR_EBATCH", -3), ("PR_ENOMEM", -4), ("PR_EHIP", -5)]:
        m = re.search(r"#define %s \(?(-?\d+)\)?" % name, text)
        assert m and int(m.group(1)) == val
        assert getattr(prhip, name) == val


def test_struct_layouts():
    assert ctypes.sizeof(prhip.PrCsr) == 8 + 4 * 8
    assert ctypes.sizeof(prhip.PrEdges) == 24
    assert ctypes.sizeof(prhip.PrTuning) == 12 * 4
    # the binding's tuning fields are the header's, in order
    text = open(os.path.join(ROOT, "include", "prhip.h")).read()
    body = re.search(r"typedef struct pr_tuning \{(.*?)\} pr_tuning;", text, re.S).group(1)
    names = re.findall(r"int32_t (\w+);", body)
    assert names == [f for f, _ in prhip.PrTuning._fields_] == list(prhip.TUNING_FIELDS)
    assert ctypes.sizeof(prhip.PrStats) == 4 + 4 + 8 + 8 + 8 + 4 + 4 + 8 + 32


def test_argument_errors_before_hip(lib):
    assert lib.pr_static(None, 0.85, 1e-10, 500, None) == prhip.PR_EINVAL
    assert b"NULL" in lib.pr_last_error()
    csr = prhip.PrCsr(0, 0, None, None, None, None)
    assert lib.pr_static(ctypes.byref(csr), 0.85, 1e-10, 500, None) == prhip.PR_EINVAL
    csr = prhip.PrCsr(4, 4, 8, 8, 8, None)  # non-NULL fake pointers: never dereferenced
    # each refusal names its reason: scalar and structural checks come before
    # the arrays' memory is examined
    for alpha, tol, it, why in [(0.0, 1e-10, 5, b"alpha"), (1.0, 1e-10, 5, b"alpha"),
                                (0.85, -1.0, 5, b"tol"), (0.85, 1e-10, 0, b"max_iter"),
                                (float("nan"), 1e-10, 5, b"alpha")]:
        assert lib.pr_static(ctypes.byref(csr), alpha, tol, it, ctypes.c_void_p(8)) == prhip.PR_EINVAL
        assert why in lib.pr_last_error()
    # pr_dfp needs out_targets
    assert lib.pr_dfp(None, ctypes.byref(csr), None, None, ctypes.c_void_p(8), 0.85, 1e-10, 1e-6,
                      1e-6, ctypes.c_void_p(8)) == prhip.PR_EINVAL
    assert b"out_targets" in lib.pr_last_error()
    csr2 = prhip.PrCsr(4, 4, 8, 8, 8, 8)
    bad = prhip.PrEdges(None, None, 3)
    assert lib.pr_dfp(None, ctypes.byref(csr2), ctypes.byref(bad), None, ctypes.c_void_p(8), 0.85,
                      1e-10, 1e-6, 1e-6, ctypes.c_void_p(8)) == prhip.PR_EINVAL
    assert b"src is NULL" in lib.pr_last_error()
    # pr_apply_batch: output sizes and required arrays are checked before any HIP call
    out = prhip.PrCsrOut(4, 5, 8, 8, None, None)  # m must be 4 - 0 + 0
    assert lib.pr_apply_batch(ctypes.byref(csr2), None, None, ctypes.byref(out)) == prhip.PR_EINVAL
    assert b"out->m" in lib.pr_last_error()
    out = prhip.PrCsrOut(4, 5, 8, 8, None, None)
    ins = prhip.PrEdges(8, None, 1)  # insertion targets are required here
    assert lib.pr_apply_batch(ctypes.byref(csr2), None, ctypes.byref(ins),
                              ctypes.byref(out)) == prhip.PR_EINVAL
    assert b"insertions.dst" in lib.pr_last_error()
    assert lib.pr_apply_batch(ctypes.byref(csr2), None, None, None) == prhip.PR_EINVAL
    for mode in (-1, 4, 7):  # PR_MODE_DFP, _DF, _ND, _DT are 0 .. 3
        assert lib.pr_dfp_ex(None, ctypes.byref(csr2), None, None, ctypes.c_void_p(8), 0.85,
                             1e-10, 1e-6, 1e-6, 500, mode, ctypes.c_void_p(8)) == prhip.PR_EINVAL
        assert b"mode" in lib.pr_last_error()
    text = open(os.path.join(ROOT, "include", "prhip.h")).read()
    for name, val in prhip.MODES.items():
        assert re.search(r"#define PR_MODE_%s %d\b" % (name.upper(), val), text), name


def test_tuning_validation(lib):
    t = prhip.PrTuning()
    assert lib.pr_get_tuning(ctypes.byref(t)) == 0
    default = prhip.get_tuning()
    assert default["hub_chunk_edges"] > 0
    for bad in [prhip.PrTuning(10, 5, 3, 1, 4096, 0),   # lane > wave
                prhip.PrTuning(1, 5, 3, 0, 4096, 0),    # iters_per_sync < 1
                prhip.PrTuning(1, 5, 9, 1, 4096, 0),    # expand lane > wave
                prhip.PrTuning(1, 5, 3, 1, -1, 0),      # chunk < 0
                prhip.PrTuning(1, 5, 3, 1, 64, -2),     # grid < 0
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 2),   # relabel not in {-1, 0, 1}
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, -1),  # die-split degree < 0
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 1),   # die-split degree 1
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, -1),   # pull threshold < 0
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 1001),   # pull threshold > 1000
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 2),   # frontier_list not 0/1
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 1, 2),  # chain_numbering > 1
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 1, -2),  # chain_numbering < -1
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 1, 1, 8),  # PPR chunk < 16
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 1, 1, (1 << 20) + 1),
                prhip.PrTuning(1, 5, 3, 1, 64, 0, 0, 0, 0, 1, 1, -1)]:
        assert lib.pr_set_tuning(ctypes.byref(bad)) == prhip.PR_EINVAL
    assert default["xcd_split_degree"] == 129 and default["expand_pull_per_mille"] == 20
    good = prhip.PrTuning(4, 64, 8, 3, 0, 100, 1, 2)
    assert lib.pr_set_tuning(ctypes.byref(good)) == 0
    got = prhip.get_tuning()
    assert got["wave_max_degree"] == 64 and got["hub_chunk_edges"] == 4096 and got["grid_blocks"] == 100
    assert got["xcd_split_degree"] == 2
    assert got["ppr_chunk_edges"] == 256 and default["ppr_chunk_edges"] == 256  # 0: default
    assert default["chain_numbering"] == -1 and default["frontier_list"] == 1
    prhip.set_tuning(ppr_chunk_edges=16)
    assert prhip.get_tuning()["ppr_chunk_edges"] == 16
    prhip.set_tuning(hub_chunk_edges=128)
    assert prhip.get_tuning()["hub_chunk_edges"] == 128
    with pytest.raises(KeyError):
        prhip.set_tuning(bogus=1)
    assert lib.pr_set_tuning(None) == 0
    assert prhip.get_tuning() == default


def test_binding_has_no_cpu_fallback():
    """The product modules never import the oracle."""
    pkg = os.path.join(ROOT, "paper_2404_08299_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f


def test_ppr_argument_errors(lib):
    csr = prhip.PrCsr(4, 4, 8, 8, 8, None)
    assert lib.pr_ppr(ctypes.byref(csr), ctypes.c_void_p(8), 0, 0.85, 1e-10, 10,
                      ctypes.c_void_p(8), None) == prhip.PR_EINVAL
    assert lib.pr_ppr(ctypes.byref(csr), None, 4, 0.85, 1e-10, 10, ctypes.c_void_p(8),
                      None) == prhip.PR_EINVAL
    assert lib.pr_ppr(ctypes.byref(csr), ctypes.c_void_p(8), 4, 1.5, 1e-10, 10,
                      ctypes.c_void_p(8), None) == prhip.PR_EINVAL


def test_weighted_adjoint_argument_errors(lib):
    csr = prhip.PrCsr(4, 4, 8, 8, 8, None)
    assert lib.pr_weighted(ctypes.byref(csr), None, None, 0.85, 1e-10, 10,
                           ctypes.c_void_p(8)) == prhip.PR_EINVAL
    # the adjoint needs out_targets and at least one output
    assert lib.pr_adjoint(ctypes.byref(csr), ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), 0.85, 1e-10, 10, ctypes.c_void_p(8), None,
                          None) == prhip.PR_EINVAL
    csr2 = prhip.PrCsr(4, 4, 8, 8, 8, 8)
    assert lib.pr_adjoint(ctypes.byref(csr2), ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), 0.85, 1e-10, 10, None, None,
                          None) == prhip.PR_EINVAL


def test_noalloc_argument_errors(lib):
    """The allocation-free entry point checks its arguments like pr_static and
    refuses graphs beyond its fixed limit before any HIP call."""
    assert lib.pr_static_noalloc(None, 0.85, 1e-10, 500, None) == prhip.PR_EINVAL
    big = prhip.PrCsr(prhip.NOALLOC_MAX_N + 1, prhip.NOALLOC_MAX_N + 1, 8, 8, 8, None)
    assert lib.pr_static_noalloc(ctypes.byref(big), 0.85, 1e-10, 500,
                                 ctypes.c_void_p(8)) == prhip.PR_EINVAL
    assert b"n must be <=" in lib.pr_last_error()
    text = open(HEADER).read()
    assert re.search(r"#define PR_NOALLOC_MAX_N \(1 << 20\)", text)
    assert prhip.NOALLOC_MAX_N == 1 << 20
    ok = prhip.PrCsr(4, 4, 8, 8, 8, None)
    assert lib.pr_static_noalloc(ctypes.byref(ok), 1.5, 1e-10, 500,
                                 ctypes.c_void_p(8)) == prhip.PR_EINVAL


def test_batched_argument_errors(lib):
    csr = (prhip.PrCsr * 2)(prhip.PrCsr(4, 4, 8, 8, 8, None), prhip.PrCsr(0, 4, 8, 8, 8, None))
    outs = (ctypes.c_void_p * 2)(8, 8)
    assert lib.pr_static_batched(csr, 0, None, 0.85, 1e-10, 10, outs, None) == prhip.PR_EINVAL
    assert lib.pr_static_batched(csr, 5000, None, 0.85, 1e-10, 10, outs, None) == prhip.PR_EINVAL
    assert lib.pr_static_batched(csr, 2, None, 0.85, 1e-10, 10, outs, None) == prhip.PR_EINVAL  # n = 0


def test_host_memory_is_refused(lib):
    """With valid scalars, arrays that are not device memory of the current
    device (here host addresses; on a machine without a GPU nothing is) are
    refused with PR_EINVAL before any work is enqueued."""
    import numpy as np
    off = np.array([0, 1, 2, 3, 4], np.int32)
    src = np.array([0, 1, 2, 3], np.int32)
    r = np.zeros(4)
    p = lambda a: a.ctypes.data
    csr = prhip.PrCsr(4, 4, p(off), p(src), p(off), p(src))
    assert lib.pr_static(ctypes.byref(csr), 0.85, 1e-10, 5, ctypes.c_void_p(p(r))) == prhip.PR_EINVAL
    assert b"not device memory" in lib.pr_last_error()
    assert lib.pr_validate_csr(ctypes.byref(csr)) == prhip.PR_EINVAL
    assert b"not device memory" in lib.pr_last_error()
    assert lib.pr_dfp(None, ctypes.byref(csr), None, None, ctypes.c_void_p(p(r)), 0.85, 1e-10,
                      1e-6, 1e-6, ctypes.c_void_p(p(r))) == prhip.PR_EINVAL
    assert b"not device memory" in lib.pr_last_error()
