"""Host-side checks of libsttsm: it loads, exports every symbol the header
declares, validates arguments before launching, and its plan's counts equal
the oracle's enumeration of the paper's loops.  Nothing here touches a GPU."""
import ctypes
import os
import re
from math import comb

import pytest

import paper_1301_7744_amd as st
from oracle import costs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "sttsm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"if", "sizeof"})


def test_library_exports_every_declared_symbol():
    lib = st.load()
    names = header_functions()
    assert "sttsm" in names and "bcss_pack" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(st.exported_symbols())


def test_version():
    assert "gfx950" in st.version()


@pytest.mark.parametrize("m,nbar", [(1, 1), (2, 3), (3, 16), (4, 8), (6, 6), (8, 5)])
def test_num_blocks(m, nbar):
    assert st.bcss_num_blocks(m, nbar) == comb(nbar + m - 1, m)


def test_num_elems_padded():
    assert st.bcss_num_elems(3, 256, 16) == 816 * 16 ** 3
    assert st.bcss_num_elems(4, 130, 16) == comb(9 + 3, 4) * 16 ** 4   # nbar = 9
    assert st.bcss_num_elems(0, 4, 2) == -1
    assert st.bcss_num_blocks(0, 3) == -1


SHAPES = [(m, n, p, bA, bC) for m in (1, 2, 3, 4, 5, 6) for (n, p) in ((8, 8), (12, 6), (7, 10))
          for bA in (1, 2, 4) for bC in (2, 3)]


@pytest.mark.parametrize("m,n,p,bA,bC", SHAPES)
def test_flop_counts_match_oracle(m, n, p, bA, bC):
    """The library's closed form and its plan's per-level sums both equal the
    oracle's enumeration of Figure 6's loops with partial symmetry."""
    levels = costs.enumerate_stage_work(m, n, p, bA, bC)
    assert st.sttsm_flops(m, n, p, bA, bC) == sum(lv["flops"] for lv in levels)
    for lv in levels:
        info = st.sttsm_plan_info(m, n, p, bA, bC, st.PREC_FP32, lv["d"])
        assert info["flops"] == lv["flops"]
        # one row group per (trailing C-block tuple of length d, unique prefix)
        assert info["groups"] == lv["prefixes"] * comb(-(-p // bC) + lv["d"] - 1, lv["d"])


@pytest.mark.parametrize("m,n,p,bA,bC", [(3, 256, 256, 16, 16), (4, 130, 32, 16, 8), (6, 24, 24, 4, 4)])
def test_temporary_shapes(m, n, p, bA, bC):
    """T^(k): binom(pbar+d, d+1) tuples of C-block indices (d = m-1-k) times
    binom(nbar+k-1, k) unique prefixes times bA^k bC^(m-k) entries."""
    nbar, pbar = -(-n // bA), -(-p // bC)
    for k in range(1, m):
        d = m - 1 - k
        info = st.sttsm_workspace_temp(m, n, p, bA, bC, st.PREC_FP32, k)
        assert info["num_jtuples"] == comb(pbar + d, d + 1)
        assert info["num_prefixes"] == comb(nbar + k - 1, k)
        assert info["block_elems"] == bA ** k * bC ** (m - k)
        assert info["byte_offset"] % 256 == 0
    assert st.sttsm_workspace_bytes(m, n, p, bA, bC) > 0


def test_config2_plan():
    """m=3, n=p=256, b=16: level 0 has 136 sorted prefixes (all 16 output
    block indices in one group), level 1 has 16 x 16 (jbar_2, ibar_0) groups,
    level 2 has 136 sorted (jbar_1, jbar_2) groups."""
    g = [st.sttsm_plan_info(3, 256, 256, 16, 16, st.PREC_FP32, d)["groups"] for d in range(3)]
    assert g == [136, 16 * 16, 136]


def _call_sttsm(LA, LC, prec=0, A=1, X=1, C=1, ws=256, wsb=1 << 30):
    lib = st.load()
    return lib.sttsm(ctypes.byref(LA), A, X, 1, 1, ctypes.byref(LC), C, prec, ws, wsb, None)


@pytest.mark.parametrize("bad", [
    dict(LA=(0, 8, 2, 0)), dict(LA=(9, 8, 2, 0)), dict(LA=(3, 0, 2, 0)), dict(LA=(3, 8, 0, 0)),
    dict(LA=(3, 8, 2, 7)), dict(LC=(3, 8, 2, 1)), dict(LC=(2, 8, 2, 0)), dict(prec=9),
    dict(LA=(3, 8, 2, 1)), dict(A=0), dict(X=0), dict(C=0), dict(ws=3),
])
def test_invalid_arguments_rejected(bad):
    LA = st.Layout(*bad.get("LA", (3, 8, 2, 0)))
    LC = st.Layout(*bad.get("LC", (3, 8, 2, 0)))
    rc = _call_sttsm(LA, LC, prec=bad.get("prec", 0), A=bad.get("A", 1), X=bad.get("X", 1), C=bad.get("C", 1),
                     ws=bad.get("ws", 256))
    assert rc == -1
    assert st.load().sttsm_last_error()


def test_bf16_input_needs_bf16_form():
    with pytest.raises(st.SttsmError):
        st.sttsm_plan_info(3, 8, 8, 2, 2, st.PREC_FP32, 0, dtype=st.BF16)
    assert st.sttsm_plan_info(3, 8, 8, 2, 2, st.PREC_BF16, 0, dtype=st.BF16)["groups"] > 0


# ------------------------------------------------------------------ serving (host side)
def test_server_argument_validation():
    lib = st.load()
    h = ctypes.c_void_p()
    assert lib.sttsm_server_create(None, 1 << 20, 4, ctypes.byref(h)) == -1
    assert lib.sttsm_server_create(256, 1 << 20, 0, ctypes.byref(h)) == -1
    assert lib.sttsm_server_create(257, 1 << 20, 4, ctypes.byref(h)) == -1
    t = ctypes.c_uint64()
    assert lib.sttsm_submit(None, None, ctypes.byref(t)) == -1
    assert lib.sttsm_poll(None, 1, ctypes.byref(ctypes.c_int32())) == -1
    assert lib.sttsm_server_destroy(None) == -1


def test_request_footprint():
    """Footprint = A + X + workspace + tables + C, growing with the shape;
    invalid requests report 0."""
    f1 = st.request_footprint(3, 32, 32, 8, 8, st.PREC_BF16, st.BF16)
    f2 = st.request_footprint(3, 64, 32, 8, 8, st.PREC_BF16, st.BF16)
    f3 = st.request_footprint(4, 64, 32, 8, 8, st.PREC_BF16, st.BF16)
    assert 0 < f1 < f2 < f3
    ws = st.sttsm_workspace_bytes(3, 64, 32, 8, 8, st.PREC_BF16, st.BF16)
    assert f2 > ws + st.bcss_num_elems(3, 32, 8) * 4
    assert st.request_footprint(0, 64, 32, 8, 8, st.PREC_BF16, st.BF16) == 0


def test_all_but_one_host_checks():
    """All modes but one: element count is T^(1)'s, m = 1 is rejected before
    any launch."""
    lib = st.load()
    LA, LC = st.layout(3, 35, 16), st.layout(3, 20, 8)
    info = st.sttsm_workspace_temp(3, 35, 20, 16, 8, st.PREC_FP32, 1)
    ne = lib.sttsm_all_but_one_elems(ctypes.byref(LA), ctypes.byref(LC), st.PREC_FP32)
    assert ne == info["num_jtuples"] * info["num_prefixes"] * info["block_elems"]
    assert info["num_jtuples"] == comb(3 + 2 - 1, 2) and info["num_prefixes"] == 3
    L1A, L1C = st.layout(1, 10, 4), st.layout(1, 6, 4)
    assert lib.sttsm_all_but_one_elems(ctypes.byref(L1A), ctypes.byref(L1C), st.PREC_FP32) == -1
    rc = lib.sttsm_all_but_one(ctypes.byref(L1A), 1, 1, 10, 1, ctypes.byref(L1C), 1, st.PREC_FP32, None, 0, None)
    assert rc == -1


@pytest.mark.parametrize("m,n,b,V", [(2, 10, 3, 4), (3, 35, 16, 7), (4, 9, 2, 3), (3, 256, 16, 64)])
def test_vector_work_count(m, n, b, V):
    """sttsm_vectors' term count: per vector, b^m for every stored block and
    every distinct block index it holds (enumerated here independently)."""
    import itertools
    nbar = -(-n // b)
    distinct = sum(len(set(t)) for t in itertools.combinations_with_replacement(range(nbar), m))
    assert st.sttsm_vectors_flops(m, n, b, V) == 2 * V * b ** m * distinct
    assert st.sttsm_vectors_flops(1, n, b, V) == -1


@pytest.mark.parametrize("m,n,p,bA,bC", [(2, 100, 70, 16, 8), (3, 35, 20, 16, 8), (4, 13, 11, 3, 3)])
def test_rank_update_workspace(m, n, p, bA, bC, monkeypatch):
    """The rank-update form's workspace: the generic chain's, with T^(1)
    (the last temporary) cut to the rows of one pass; one pass of all rows
    needs exactly the chain's workspace."""
    monkeypatch.setenv("STTSM_GENERIC_KERNELS", "1")
    info = st.sttsm_workspace_temp(m, n, p, bA, bC, st.PREC_FP32, 1)
    chain = st.sttsm_workspace_bytes(m, n, p, bA, bC, st.PREC_FP32)
    nbar = -(-n // bA)
    for rows in (1, 2, nbar, nbar + 5):
        pass_bytes = info["num_jtuples"] * min(rows, nbar) * info["block_elems"] * 4
        want = info["byte_offset"] + -(-pass_bytes // 256) * 256
        assert st.sttsm_rank_update_workspace_bytes(m, n, p, bA, bC, st.PREC_FP32, rows) == want
    assert st.sttsm_rank_update_workspace_bytes(m, n, p, bA, bC, st.PREC_FP32, nbar) == chain
    monkeypatch.delenv("STTSM_GENERIC_KERNELS")
    # independent of the kernel choice sttsm itself would make
    assert st.sttsm_rank_update_workspace_bytes(m, n, p, bA, bC, st.PREC_FP32, nbar) == chain


def test_rank_update_host_checks():
    """m = 1 and rows < 1 are rejected before any launch."""
    lib = st.load()
    L1A, L1C = st.layout(1, 10, 4), st.layout(1, 6, 4)
    assert lib.sttsm_rank_update_workspace_bytes(ctypes.byref(L1A), ctypes.byref(L1C), st.PREC_FP32, 1) == 0
    rc = lib.sttsm_rank_update(ctypes.byref(L1A), 1, 1, 10, 1, ctypes.byref(L1C), 1, st.PREC_FP32, 1, None, 0, None)
    assert rc == -1
    LA, LC = st.layout(2, 10, 4), st.layout(2, 6, 4)
    assert lib.sttsm_rank_update_workspace_bytes(ctypes.byref(LA), ctypes.byref(LC), st.PREC_FP32, 0) == 0
    rc = lib.sttsm_rank_update(ctypes.byref(LA), 1, 1, 10, 1, ctypes.byref(LC), 1, st.PREC_FP32, 0, None, 0, None)
    assert rc == -1
    assert "rows" in lib.sttsm_last_error().decode()
