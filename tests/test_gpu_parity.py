"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Integer/byte work (pack, unpack, padding) is compared bit for bit; floating
point results by relative Frobenius error over the dense C with the bounds in
gpu_util (FP32 1e-5; BF16 sqrt(2m) 2^-8; split-BF16x3 2e-5) and, entry by
entry, by |C_gpu - C_ref| <= TAU u S_j with S_j the oracle's per-entry error
scale and u the precision form's unit roundoff (gpu_util.check_entries).  At
every full-size workload 256 output entries are also evaluated by the
literal n^m-term sum of Eq. (cob) (O3) and checked the same way."""
import numpy as np
import pytest

import oracle
from oracle import bcss_ref, closed_forms
import synth
from gpu_util import (P32, PBF, PX3B, PX3F, TOL_FP32, TOL_X3_FIRST_FP32, TOL_X3_STAGE0, check_entries,
                      check_literal_entries, dev_dense, err, padding_mask, ref_bcss, reference, run, say, tol_bf16)

pytestmark = pytest.mark.gpu


def st():
    import paper_1301_7744_amd
    return paper_1301_7744_amd


# ------------------------------------------------------------------ pack / unpack
PACK_CASES = [(1, 5, 2), (2, 7, 3), (3, 16, 4), (3, 10, 4), (4, 9, 2), (5, 6, 2), (6, 5, 2), (3, 3, 4),
              (2, 130, 16), (3, 256, 16), (8, 2, 1)]


@pytest.mark.parametrize("m,n,b", PACK_CASES)
def test_pack_bitexact(m, n, b):
    import torch
    say("pack", m, n, b)
    A = synth.symmetric_uniform(m, n, (m, n, b, 1))
    got = st().bcss_pack(dev_dense(A), m, n, b)
    torch.cuda.synchronize()
    ref = bcss_ref.pack(A, b)
    assert np.array_equal(got.cpu().numpy().reshape(ref.shape), ref)


@pytest.mark.parametrize("dt", ["bf16", "f64"])
def test_pack_unpack_other_dtypes(dt):
    import torch
    tdt = {"bf16": torch.bfloat16, "f64": torch.float64}[dt]
    m, n, b = 3, 11, 4
    A = synth.symmetric_uniform(m, n, 5)
    if dt == "bf16":
        A = synth.round_to_bf16(A)
    Ad = dev_dense(A.astype(np.float64 if dt == "f64" else np.float32), tdt)
    P = st().bcss_pack(Ad, m, n, b)
    D = st().bcss_unpack(P, m, n, b)
    torch.cuda.synchronize()
    assert torch.equal(D, Ad)
    ref = bcss_ref.pack(A, b)
    assert np.array_equal(P.to(torch.float64).cpu().numpy().reshape(ref.shape), ref)


@pytest.mark.parametrize("m,n,b", PACK_CASES)
def test_unpack_bitexact(m, n, b):
    """unpack(pack(A)) == A, and unpack of an arbitrary (non-symmetric) BCSS
    array equals the oracle's unpack, which shows the permuted reads."""
    import torch
    say("unpack", m, n, b)
    A = synth.symmetric_uniform(m, n, (m, n, b, 2))
    Ad = dev_dense(A)
    D = st().bcss_unpack(st().bcss_pack(Ad, m, n, b), m, n, b)
    torch.cuda.synchronize()
    assert torch.equal(D, Ad)
    if n ** m <= 300_000:
        nb = st().bcss_num_blocks(m, -(-n // b))
        B = synth.rng((m, n, b, 3)).standard_normal((nb, b ** m)).astype(np.float32)
        Dd = st().bcss_unpack(torch.from_numpy(B.ravel()).cuda(), m, n, b)
        torch.cuda.synchronize()
        ref = bcss_ref.unpack(B, m, n, b)
        assert np.array_equal(Dd.cpu().numpy(), ref.ravel(order="F"))


# ------------------------------------------------------------------ FP32 sttsm
SMALL = [(m, n, p, bA, bC) for m, n, p, bA, bC in [
    (1, 5, 3, 2, 2), (1, 40, 33, 16, 8),
    (2, 5, 3, 2, 1), (2, 7, 7, 3, 3), (2, 17, 9, 4, 8), (2, 33, 40, 16, 16), (2, 70, 65, 64, 64),
    (3, 5, 5, 2, 2), (3, 6, 4, 3, 2), (3, 9, 11, 4, 4), (3, 16, 16, 4, 4), (3, 20, 13, 8, 4), (3, 35, 35, 16, 16),
    (4, 5, 4, 2, 3), (4, 9, 9, 4, 4), (4, 12, 7, 4, 2), (4, 17, 10, 8, 4),
    (5, 4, 5, 2, 2), (5, 7, 6, 4, 3),
    (6, 4, 4, 2, 2), (6, 5, 3, 2, 1),
    (7, 3, 3, 1, 2), (8, 2, 2, 1, 1), (3, 3, 2, 4, 4), (3, 1, 1, 1, 1),
]]


@pytest.mark.parametrize("m,n,p,bA,bC", SMALL)
def test_fp32_small_vs_oracle(m, n, p, bA, bC):
    """Several tiles and ragged tails, p != n, bA != bC, n < b, m = 1..8."""
    say("fp32", m, n, p, bA, bC)
    A = synth.symmetric_uniform(m, n, (m, n, p, 11))
    X = synth.change_of_basis(p, n, (m, n, p, 12))
    got = run(A, X, bA, bC, P32)
    ref, S = reference(A, X, bC)
    e = err(got, ref, m, p, bC)
    say("  rel err", e)
    assert e <= TOL_FP32
    check_entries(got, ref, S, P32, -(-n // bA) * bA)
    mask = padding_mask(m, p, bC)
    assert np.all(got[mask] == 0.0)


def test_fp32_config1_vs_direct_sum():
    """m=3, n=p=16, b=4 against the literal direct sum (O1)."""
    A, X = synth.make_config_inputs("m3_n16_b4")
    got = run(A, X, 4, 4, P32)
    ref = ref_bcss(A.astype(np.float64), X.astype(np.float64), 4, method="direct")
    e = err(got, ref, 3, 16, 4)
    say("config1 fp32 rel err", e)
    assert e <= TOL_FP32
    _, S = reference(A, X, 4)
    check_entries(got, ref, S, P32, 16)


def test_fp32_config2_full():
    """m=3, n=p=256, b=16 (the measured workload): full C against O2, entry
    by entry, and 256 sampled entries against the literal per-entry sum (O3)."""
    A, X = synth.make_config_inputs("m3_n256_b16")
    got = run(A, X, 16, 16, P32)
    ref, S = reference(A, X, 16)
    e = err(got, ref, 3, 256, 16)
    say("config2 fp32 rel err", e)
    assert e <= TOL_FP32
    check_entries(got, ref, S, P32, 256)
    check_literal_entries({P32: got}, A, X, 16, ref, S, 256)


def test_temporaries_match_oracle():
    """Every stored block of every GPU temporary T^(k) equals O2's dense T^(k)
    restricted to that block (FP32 tolerance per block set)."""
    import torch
    for (m, n, p, bA, bC) in [(3, 16, 16, 4, 4), (4, 9, 7, 4, 3), (3, 35, 20, 16, 8)]:
        say("temps", m, n, p, bA, bC)
        A = synth.symmetric_uniform(m, n, (m, n, 21))
        X = synth.change_of_basis(p, n, (m, n, 22))
        _, ws = run(A, X, bA, bC, P32, keep_ws=True)
        _, temps = oracle.chain(A.astype(np.float64), X.astype(np.float64), keep_temps=True)
        nbar, pbar = -(-n // bA), -(-p // bC)
        for k in range(1, m):
            T = st().temporary(ws, m, n, p, bA, bC, P32, k).double().cpu().numpy()
            dense = temps[k]
            pad = np.zeros((nbar * bA,) * k + (pbar * bC,) * (m - k))
            pad[tuple(slice(0, n) for _ in range(k)) + tuple(slice(0, p) for _ in range(m - k))] = dense
            jt = bcss_ref.sorted_block_tuples(m - k, pbar)
            pf = bcss_ref.sorted_block_tuples(k, nbar) if k else [()]
            shape = (bA,) * k + (bC,) * (m - k)
            num = den = 0.0
            for r, J in enumerate(jt):
                for q, s in enumerate(pf):
                    sl = tuple(slice(si * bA, (si + 1) * bA) for si in s) + \
                        tuple(slice(ji * bC, (ji + 1) * bC) for ji in J)
                    ref = pad[sl].ravel(order="F")
                    num += float(np.sum((T[r, q] - ref) ** 2))
                    den += float(np.sum(ref ** 2))
            e = (num / den) ** 0.5
            say("  T^(%d) rel err" % k, e)
            assert e <= TOL_FP32
        del ws
        torch.cuda.empty_cache()


# ------------------------------------------------------------------ reduced precision
@pytest.mark.parametrize("prec", [PBF, PX3F, PX3B])
@pytest.mark.parametrize("case", [(3, 16, 16, 4, 4), (3, 35, 20, 16, 8), (4, 17, 10, 8, 4), (2, 70, 65, 64, 64),
                                  (5, 7, 6, 4, 3)])
def test_reduced_precision_small(prec, case):
    m, n, p, bA, bC = case
    say("prec", prec, case)
    A = synth.symmetric_uniform(m, n, (m, n, 31))
    X = synth.change_of_basis(p, n, (m, n, 32))
    got = run(A, X, bA, bC, prec)
    ref, S = reference(A, X, bC)
    e = err(got, ref, m, p, bC)
    bound = {PBF: tol_bf16(m), PX3F: TOL_X3_FIRST_FP32, PX3B: tol_bf16(m)}[prec]
    say("  rel err", e, "bound", bound)
    assert e <= bound
    check_entries(got, ref, S, prec, -(-n // bA) * bA)
    assert np.all(got[padding_mask(m, p, bC)] == 0.0)


def test_bf16_inputs():
    """BF16 A and X (the served precision): the oracle gets the same bf16 values."""
    import torch
    m, n, p, b = 3, 40, 24, 8
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, 41))
    X = synth.round_to_bf16(synth.change_of_basis(p, n, 42))
    got = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    ref, S = reference(A, X, b)
    e = err(got, ref, m, p, b)
    say("bf16-input rel err", e)
    assert e <= tol_bf16(m)
    check_entries(got, ref, S, PBF, n)


def test_split_stage0_recovers_fp32():
    """split-BF16x3: the first temporary T^(m-1) alone is within 1e-5 of O2,
    while plain BF16 is not."""
    m, n, p, b = 3, 64, 64, 16
    A = synth.symmetric_uniform(m, n, 51)
    X = synth.change_of_basis(p, n, 52)
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    _, temps = oracle.chain(A64, X64, keep_temps=True)
    ref = temps[m - 1]
    scale = oracle.error_scale(A64, X64, last_mode=m - 1)     # the first level alone
    errs = {}
    for prec in (PX3F, PBF):
        _, ws = run(A, X, b, b, prec, keep_ws=True)
        T = st().temporary(ws, m, n, p, b, b, prec, m - 1).double().cpu().numpy()
        nbar = n // b
        pf = bcss_ref.sorted_block_tuples(m - 1, nbar)
        got_l, ref_l, sc_l = [], [], []
        for jb in range(p // b):
            for q, s in enumerate(pf):
                sl = tuple(slice(si * b, (si + 1) * b) for si in s) + (slice(jb * b, (jb + 1) * b),)
                got_l.append(T[jb, q])
                ref_l.append(ref[sl].ravel(order="F"))
                sc_l.append(scale[sl].ravel(order="F"))
        got_a, ref_a = np.array(got_l), np.array(ref_l)
        errs[prec] = float(np.linalg.norm(got_a - ref_a) / np.linalg.norm(ref_a))
        if prec == PX3F:
            check_entries(got_a, ref_a, np.array(sc_l), PX3F, n, what="T^(m-1)")
    say("T^(m-1) errors", errs)
    assert errs[PX3F] <= TOL_X3_STAGE0
    assert errs[PBF] > 10 * errs[PX3F]


# ------------------------------------------------------------------ full-size sweep
SWEEP = ["m2_n4096_b64", "m4_n64_b8", "m5_n32_b4", "m6_n24_b4"]


@pytest.fixture(scope="module")
def sweep_refs():
    return {}


@pytest.mark.parametrize("prec", [P32, PBF, PX3F, PX3B])
@pytest.mark.parametrize("name", SWEEP)
def test_order_sweep_full(name, prec, sweep_refs):
    """Each order-sweep workload in every precision form: the whole C by
    relative Frobenius error and entry by entry, and 256 entries against the
    literal sum (O3)."""
    c = synth.CONFIGS[name]
    m, n, p, b = c["m"], c["n"], c["p"], c["bA"]
    say("sweep", name, prec)
    A, X = synth.make_config_inputs(name)
    if sweep_refs.get("name") != name:
        sweep_refs.clear()
        sweep_refs["name"] = name
        sweep_refs["ref"], sweep_refs["S"] = reference(A, X, b)
    ref, S = sweep_refs["ref"], sweep_refs["S"]
    got = run(A, X, b, b, prec)
    e = err(got, ref, m, p, b)
    bound = {P32: TOL_FP32, PBF: tol_bf16(m), PX3F: TOL_X3_FIRST_FP32, PX3B: tol_bf16(m)}[prec]
    say("  rel err", e, "bound", bound)
    assert e <= bound
    check_entries(got, ref, S, prec, n)
    check_literal_entries({prec: got}, A, X, b, ref, S, n, cache=sweep_refs)


_RECT = {}


def _rect_inputs(case):
    """A (fp32), X, the oracle's C on those values, its per-entry error scale
    and the closed form, per (n, seed): shared by the block-size and
    precision variants (and so are the O3 literal sums, in the cache)."""
    key = (case["m"], case["n"], case["p"], case["rank"], case["seed"])
    if key not in _RECT:
        _RECT.clear()
        m = case["m"]
        A, X, lams, vecs = synth.rect_inputs(case)
        A64, X64 = A.astype(np.float64), X.astype(np.float64)
        Cref, temps = oracle.chain(A64, X64, keep_temps=True)
        S = oracle.error_scale(A64, X64, temps=temps)
        del temps, A64
        Cclosed = closed_forms.rank_r(lams, vecs, X64, m)
        _RECT[key] = (A, X, Cref, Cclosed, S, {})
    return _RECT[key]


@pytest.mark.parametrize("prec", [P32, PBF])
@pytest.mark.parametrize("case", synth.rect_cases(), ids=lambda c: c["name"])
def test_rank8_rectangular(case, prec):
    """m=4, p=32, rank-8 A: against the closed form sum lam (X a)^{o4}."""
    m, n, p, bA, bC = case["m"], case["n"], case["p"], case["bA"], case["bC"]
    say("rect", case["name"], prec)
    A, X, Cref, Cclosed, S, cache = _rect_inputs(case)
    got = run(A, X, bA, bC, prec)
    # the GPU sees A rounded to fp32: compare with the exact result for those values
    ref, Sb = bcss_ref.pack(Cref, bC), bcss_ref.pack(S, bC)
    e = err(got, ref, m, p, bC)
    closed = bcss_ref.pack(Cclosed, bC)
    e_closed = err(got, closed, m, p, bC)
    bound = TOL_FP32 if prec == P32 else tol_bf16(m)
    say("  rel err", e, "vs closed form", e_closed)
    assert e <= bound and e_closed <= bound
    kpad = -(-n // bA) * bA
    check_entries(got, ref, Sb, prec, kpad)
    check_literal_entries({prec: got}, A, X, bC, ref, Sb, kpad, cache=cache)
    assert np.all(got[padding_mask(m, p, bC)] == 0.0)


# ------------------------------------------------------------------ edge cases
def test_zero_inputs_give_exact_zero():
    m, n, p, b = 3, 20, 18, 8
    A = synth.symmetric_uniform(m, n, 61)
    assert np.all(run(A, np.zeros((p, n), np.float32), b, b, P32) == 0.0)
    assert np.all(run(np.zeros_like(A), synth.change_of_basis(p, n, 62), b, b, PBF) == 0.0)


def test_deterministic_reruns():
    m, n, p, b = 3, 48, 48, 16
    A = synth.symmetric_uniform(m, n, 71)
    X = synth.change_of_basis(p, n, 72)
    for prec in (P32, PBF, PX3F):
        assert np.array_equal(run(A, X, b, b, prec), run(A, X, b, b, prec))


def test_workspace_too_small_rejected():
    """Through the raw C ABI: a workspace one byte short returns EINVAL."""
    import ctypes
    import torch
    lib = st().load()
    m, n, p, b = 3, 16, 16, 4
    A = synth.symmetric_uniform(m, n, 81)
    Ab = st().bcss_pack(dev_dense(A), m, n, b)
    X = torch.zeros(p, n, device="cuda")
    C = torch.empty(st().bcss_num_elems(m, p, b), device="cuda")
    need = st().sttsm_workspace_bytes(m, n, p, b, b)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    LA, LC = st().layout(m, n, b), st().layout(m, p, b)
    rc = lib.sttsm(ctypes.byref(LA), Ab.data_ptr(), X.data_ptr(), n, 1, ctypes.byref(LC), C.data_ptr(), P32,
                   ws.data_ptr(), need - 1, None)
    assert rc == -1 and b"workspace" in lib.sttsm_last_error()
    rc = lib.sttsm(ctypes.byref(LA), Ab.data_ptr(), X.data_ptr(), n, 1, ctypes.byref(LC), C.data_ptr(), P32,
                   ws.data_ptr(), need, None)
    torch.cuda.synchronize()
    assert rc == 0


# ------------------------------------------------------------------ both staging kernels
FAST_SHAPES = [(3, 35, 35, 16, 16), (3, 40, 24, 16, 16), (3, 100, 70, 16, 16), (5, 9, 10, 4, 4), (5, 13, 7, 4, 4)]


@pytest.mark.parametrize("generic", [False, True], ids=["blockcopy", "generic"])
@pytest.mark.parametrize("m,n,p,bA,bC", FAST_SHAPES)
def test_block_copy_and_generic_kernels(m, n, p, bA, bC, generic, monkeypatch):
    """Shapes the block-copy kernel takes (256 entries per block row, bA | 16),
    run through it and through the generic kernel: both match the oracle."""
    if generic:
        monkeypatch.setenv("STTSM_GENERIC_KERNELS", "1")
    else:
        monkeypatch.delenv("STTSM_GENERIC_KERNELS", raising=False)
    say("kernels", "generic" if generic else "block-copy", m, n, p, bA, bC)
    A = synth.symmetric_uniform(m, n, (m, n, p, 91))
    X = synth.change_of_basis(p, n, (m, n, p, 92))
    got = run(A, X, bA, bC, P32)
    e = err(got, ref_bcss(A.astype(np.float64), X.astype(np.float64), bC), m, p, bC)
    say("  rel err", e)
    assert e <= TOL_FP32
    assert np.all(got[padding_mask(m, p, bC)] == 0.0)


# Every instantiated tile of the FP32 block-copy kernel that a level can
# take (STTSM_FAST_TILE, one entry per level, empty = default): prefetch
# depths 1-4, K chunks of 16 and 32, 32- to 128-column tiles.  The first
# level (k = m-1) takes whole 256-row block rows only.  Each test checks,
# through sttsm_plan_info, that the plan took the requested tile.
FAST_TILE_CASES = [
    ("256x64x16x2,128x128x16x2,128x64x16x2", 3, 101, 71),
    (",128x128x16x3,128x64x16x3", 3, 103, 75),
    (",128x64x16x4,128x64x16x4", 3, 105, 81),
    ("256x32x16x1,128x32x16x1,128x32x16x2", 3, 99, 83),
    ("256x128x16x1,128x64x32x1,128x64x32x1", 3, 97, 87),
    (",128x64x16x2,256x64x16x1", 3, 94, 90),
    ("256x64x16x2,256x64x16x1,256x64x16x2", 5, 11, 9),
]


@pytest.mark.parametrize("tiles,m,n,p", FAST_TILE_CASES, ids=[c[0] or "default" for c in FAST_TILE_CASES])
def test_block_copy_tile_variants(tiles, m, n, p, monkeypatch):
    """Each block-copy tile variant against the oracle on a ragged shape."""
    monkeypatch.delenv("STTSM_GENERIC_KERNELS", raising=False)
    monkeypatch.setenv("STTSM_FAST_TILE", tiles)
    b = 16 if m == 3 else 4
    say("tile variant", tiles, m, n, p, b)
    for d, want in enumerate(tiles.split(",")):
        if want:
            info = st().sttsm_plan_info(m, n, p, b, b, P32, d)
            assert info["kernel"] == "fp32_block_copy"
            assert info["tile"] == tuple(int(v) for v in want.split("x")), (d, info)
    A = synth.symmetric_uniform(m, n, (m, n, p, 93))
    X = synth.change_of_basis(p, n, (m, n, p, 94))
    got = run(A, X, b, b, P32)
    e = err(got, ref_bcss(A.astype(np.float64), X.astype(np.float64), b), m, p, b)
    say("  rel err", e)
    assert e <= TOL_FP32
    assert np.all(got[padding_mask(m, p, b)] == 0.0)


# ------------------------------------------------------------------ bf16 block-copy kernel
# (m, n, p, b): ragged n and p, K chunks that run past nbar, m = 4 M tiles.
BF16_FAST_SHAPES = [(3, 40, 24, 8), (3, 35, 35, 16), (3, 100, 70, 16), (3, 130, 60, 16), (4, 33, 20, 8),
                    (4, 48, 16, 8), (4, 40, 37, 16), (4, 64, 64, 8)]


def bf16_fast_level0_tasks(m, n, p, b):
    """Workgroup tasks of level 0 under the bf16 block-copy tiling:
    unique prefixes x column tiles (b = 16: 64 wide, b = 8: 128) x M tiles
    (b^(m-3) of b^2 rows each)."""
    from math import comb
    import os
    nbar, pbar = -(-n // b), -(-p // b)
    nt = 64 if b == 16 else 128
    # b = 16 with Kpad <= 256 on bf16 input: the X-resident form, 96-column tiles by default
    xres = os.environ.get("STTSM_BF16_XRES", "")
    if b == 16 and nbar * b <= 256 and not os.environ.get("STTSM_BF16_TILE") and xres != "0":
        nt = int(xres.split("x")[0]) if "x" in xres else 96
    override = os.environ.get("STTSM_BF16_TILE", "")   # "NTxKTxPD", a measurement override
    if override and "," not in override:
        o_nt = int(override.split("x")[0])
        if (b == 16 and override in ("128x32x1", "64x32x1", "64x32x2", "64x16x1", "64x16x3", "128x16x2",
                                       "32x16x1")) or \
                (b == 8 and override in ("256x32x1", "128x32x1", "128x32x2", "128x16x3")):
            nt = o_nt
    return comb(nbar + m - 2, m - 1) * (-(-(pbar * b) // nt)) * b ** (m - 3)


@pytest.mark.parametrize("generic", [False, True], ids=["blockcopy", "generic"])
@pytest.mark.parametrize("m,n,p,b", BF16_FAST_SHAPES)
def test_bf16_block_copy_and_generic_kernels(m, n, p, b, generic, monkeypatch):
    """BF16 inputs and temporaries (the served form) through the bf16
    block-copy kernel and through the generic kernel: both within the bf16
    bound of the oracle run on the same bf16 values; padding exactly zero."""
    import torch
    if generic:
        monkeypatch.setenv("STTSM_GENERIC_KERNELS", "1")
    else:
        monkeypatch.delenv("STTSM_GENERIC_KERNELS", raising=False)
    info = st().sttsm_plan_info(m, n, p, b, b, PBF, 0, dtype=st().BF16)
    if not generic:
        assert info["tasks"] == bf16_fast_level0_tasks(m, n, p, b)
    say("bf16 kernels", "generic" if generic else "block-copy", m, n, p, b, info)
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, (m, n, p, 93)))
    X = synth.round_to_bf16(synth.change_of_basis(p, n, (m, n, p, 94)))
    got = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    ref, S = reference(A, X, b)
    e = err(got, ref, m, p, b)
    say("  rel err", e, "bound", tol_bf16(m))
    assert e <= tol_bf16(m)
    check_entries(got, ref, S, PBF, -(-n // b) * b)
    assert np.all(got[padding_mask(m, p, b)] == 0.0)


# bf16 tile variants (STTSM_BF16_TILE, "NTxKTxPD" per level): 32-wide K chunks
# hold two b = 16 blocks, each staged in its own region with its own layout.
# Plans are cached per shape, so every case has a shape no other test uses.
BF16_TILE_CASES = [("64x32x1", 3, 101, 69, 16), ("64x32x2,128x32x1,64x32x2", 3, 131, 61, 16),
                   ("128x32x1", 4, 41, 36, 16), ("64x16x3,64x16x1,32x16x1", 3, 36, 34, 16),
                   ("128x32x2,256x32x1,128x16x3", 3, 41, 23, 8)]


@pytest.mark.parametrize("tiles,m,n,p,b", BF16_TILE_CASES, ids=[c[0] for c in BF16_TILE_CASES])
def test_bf16_tile_variants(tiles, m, n, p, b, monkeypatch):
    """Each bf16 block-copy tile variant against the oracle on a ragged shape."""
    import torch
    monkeypatch.delenv("STTSM_GENERIC_KERNELS", raising=False)
    monkeypatch.setenv("STTSM_BF16_TILE", tiles)
    say("bf16 tile variant", tiles, m, n, p, b)
    parts = tiles.split(",")
    for d in range(m):
        want = parts[0] if len(parts) == 1 else (parts[d] if d < len(parts) else "")
        if want:
            info = st().sttsm_plan_info(m, n, p, b, b, PBF, d, dtype=st().BF16)
            assert info["kernel"] == "bf16_block_copy"
            assert info["tile"][1:] == tuple(int(v) for v in want.split("x")), (d, info)
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, (m, n, p, 95)))
    X = synth.round_to_bf16(synth.change_of_basis(p, n, (m, n, p, 96)))
    got = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    ref, S = reference(A, X, b)
    e = err(got, ref, m, p, b)
    say("  rel err", e, "bound", tol_bf16(m))
    assert e <= tol_bf16(m)
    check_entries(got, ref, S, PBF, -(-n // b) * b)
    assert np.all(got[padding_mask(m, p, b)] == 0.0)


# The X-resident form of the bf16 block-copy kernel (b = 16, bf16 input,
# Kpad <= 256) runs the same MFMA sequence on the same operands for every
# output entry as the chunk-staged kernel, so both give the same C.
XRES_SHAPES = [(3, 35, 35), (3, 100, 70), (3, 130, 60), (4, 40, 37), (4, 64, 64), (3, 256, 256), (3, 250, 17)]


@pytest.mark.parametrize("m,n,p", XRES_SHAPES)
def test_bf16_xres_matches_chunk_staged(m, n, p, monkeypatch):
    import torch
    b = 16
    monkeypatch.delenv("STTSM_GENERIC_KERNELS", raising=False)
    monkeypatch.delenv("STTSM_BF16_TILE", raising=False)
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, (m, n, p, 97)))
    X = synth.round_to_bf16(synth.change_of_basis(p, n, (m, n, p, 98)))
    got = {}
    modes = ("0", "64x2", "64x4", "96x2", "96x4", "128x2", "128x4")
    for mode in modes:
        monkeypatch.setenv("STTSM_BF16_XRES", mode)
        for d in range(m):
            info = st().sttsm_plan_info(m, n, p, b, b, PBF, d, dtype=st().BF16)
            if mode == "0":
                assert info["kernel"] == "bf16_block_copy"
            else:
                assert info["kernel"] == "bf16_xres"
                assert (info["tile"][1], info["tile"][3]) == tuple(int(v) for v in mode.split("x"))
        say("xres", mode, m, n, p)
        got[mode] = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    for mode in modes[1:]:
        assert np.array_equal(got["0"], got[mode]), mode
    ref, S = reference(A, X, b)
    e = err(got["96x2"], ref, m, p, b)
    say("  rel err", e, "bound", tol_bf16(m))
    assert e <= tol_bf16(m)
    check_entries(got["96x2"], ref, S, PBF, -(-n // b) * b)
    assert np.all(got["96x2"][padding_mask(m, p, b)] == 0.0)


def test_bf16_block_copy_config2_full():
    """m = 3, n = p = 256, b = 16 in bf16 through the block-copy kernel (the
    bench workload at bf16): the whole C against the oracle chain on the same
    bf16 values, by Frobenius error and entry by entry, and 256 entries
    against the literal sum (O3)."""
    import torch
    m, n, p, b = 3, 256, 256, 16
    A, X = synth.make_config_inputs("m3_n256_b16")
    A, X = synth.round_to_bf16(A), synth.round_to_bf16(X)
    got = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    ref, S = reference(A, X, b)
    e = err(got, ref, m, p, b)
    say("config m3_n256_b16 bf16 rel err", e, "bound", tol_bf16(m))
    assert e <= tol_bf16(m)
    check_entries(got, ref, S, PBF, n)
    check_literal_entries({PBF: got}, A, X, b, ref, S, n)


# ------------------------------------------------------------------ all modes but one
def _blocks_of_T1(dense, m, n, p, bA, bC):
    """Oracle's dense A x_1 X ... x_{m-1} X cut into the [J][ibar][block] layout."""
    nbar, pbar = -(-n // bA), -(-p // bC)
    pad = np.zeros((nbar * bA,) + (pbar * bC,) * (m - 1))
    pad[(slice(0, n),) + tuple(slice(0, p) for _ in range(m - 1))] = dense
    out = []
    for J in bcss_ref.sorted_block_tuples(m - 1, pbar):
        row = []
        for i in range(nbar):
            sl = (slice(i * bA, (i + 1) * bA),) + tuple(slice(j * bC, (j + 1) * bC) for j in J)
            row.append(pad[sl].ravel(order="F"))
        out.append(row)
    return np.array(out)


@pytest.mark.parametrize("case", [(3, 16, 16, 4, 4, P32), (4, 9, 7, 4, 3, P32), (3, 35, 20, 16, 8, P32),
                                  (2, 70, 33, 16, 8, P32), (3, 70, 40, 16, 16, PBF), (4, 33, 20, 8, 8, PBF)])
def test_all_but_one_vs_oracle(case):
    """sttsm_all_but_one (the chain stopped before mode 0) against the
    oracle's mode products in modes m-1..1, block by block."""
    import torch
    m, n, p, bA, bC, prec = case
    say("all-but-one", case)
    A = synth.symmetric_uniform(m, n, (m, n, 71))
    X = synth.change_of_basis(p, n, (m, n, 72))
    tdt = torch.float32
    if prec == PBF:
        A, X, tdt = synth.round_to_bf16(A), synth.round_to_bf16(X), torch.bfloat16
    Ab = st().bcss_pack(dev_dense(np.asarray(A, np.float32), tdt), m, n, bA)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(tdt).cuda()
    T, _ = st().sttsm_all_but_one(Ab, Xd, m, n, p, bA, bC, prec)
    torch.cuda.synchronize()
    got = T.double().cpu().numpy()
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    ref = _blocks_of_T1(oracle.all_but_one(A64, X64), m, n, p, bA, bC)
    scale = _blocks_of_T1(oracle.error_scale(A64, X64, last_mode=1), m, n, p, bA, bC)
    e = float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
    bound = TOL_FP32 if prec == P32 else tol_bf16(m)
    say("  rel err", e, "bound", bound)
    assert got.shape == ref.shape
    assert e <= bound
    check_entries(got, ref, scale, prec, -(-n // bA) * bA)


# ------------------------------------------------------------------ symmetrisation
@pytest.mark.parametrize("m,n,b,dt", [(2, 7, 3, "f32"), (3, 10, 4, "f32"), (4, 9, 2, "f32"), (3, 16, 4, "f64"),
                                      (3, 40, 8, "bf16"), (5, 6, 2, "f32")])
def test_symmetrize_vs_oracle(m, n, b, dt):
    """bcss_symmetrize on a BCSS array that is not symmetric inside its
    blocks: equal to the oracle (dense average over all m! permutations,
    packed), mirrored entries bitwise equal, blocks without repeated block
    indices untouched."""
    import itertools
    import torch
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[dt]
    nb = st().bcss_num_blocks(m, -(-n // b))
    raw = synth.rng((m, n, b, 81)).standard_normal((nb, b ** m))
    X = bcss_ref.pack(bcss_ref.unpack(raw, m, n, b), b)       # zero padding
    if dt == "bf16":
        X = synth.round_to_bf16(X.astype(np.float32)).astype(np.float64)
    dev = torch.from_numpy(X.ravel()).to(tdt).cuda()
    X = dev.double().cpu().numpy().reshape(nb, b ** m)          # the values the GPU holds
    st().bcss_symmetrize(dev, m, n, b)
    torch.cuda.synchronize()
    got = dev.double().cpu().numpy().reshape(nb, b ** m)
    ref = bcss_ref.symmetrize(X, m, n, b)
    tol = {"f32": 1e-6, "f64": 1e-14, "bf16": 2 ** -8}[dt]
    say("symmetrize", m, n, b, dt, "max diff", np.abs(got - ref).max())
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    D = bcss_ref.unpack(got, m, n, b)
    for p in itertools.permutations(range(m)):
        assert np.array_equal(np.transpose(D, p), D)
    for r, s in enumerate(bcss_ref.sorted_block_tuples(m, -(-n // b))):
        if len(set(s)) == m:
            assert np.array_equal(got[r], X[r])


def test_symmetrize_after_sttsm():
    """C from sttsm, symmetrised: exactly symmetric, still within the FP32
    bound of the oracle."""
    import itertools
    import torch
    m, n, p, b = 3, 35, 20, 8
    A = synth.symmetric_uniform(m, n, 91)
    X = synth.change_of_basis(p, n, 92)
    Ab = st().bcss_pack(dev_dense(A), m, n, b)
    Xd = torch.from_numpy(X).cuda()
    C, _ = st().sttsm(Ab, Xd, m, n, p, b, b, P32)
    st().bcss_symmetrize(C, m, p, b)
    torch.cuda.synchronize()
    nb = st().bcss_num_blocks(m, -(-p // b))
    got = C.double().cpu().numpy().reshape(nb, b ** m)
    D = bcss_ref.unpack(got, m, p, b)
    for q in itertools.permutations(range(m)):
        assert np.array_equal(np.transpose(D, q), D)
    assert err(got, ref_bcss(A.astype(np.float64), X.astype(np.float64), b), m, p, b) <= TOL_FP32


# ------------------------------------------------------------------ vector case
@pytest.mark.parametrize("m,n,b,V,dt", [(2, 33, 8, 4, "f32"), (3, 16, 4, 5, "f32"), (3, 35, 16, 7, "f32"),
                                        (4, 9, 2, 3, "f32"), (5, 7, 3, 6, "f32"), (3, 256, 16, 64, "f32"),
                                        (3, 40, 8, 9, "bf16"), (3, 30, 4, 70, "f32"), (3, 21, 8, 40, "f32"),
                                        (3, 100, 16, 17, "bf16")])
def test_vectors_vs_oracle(m, n, b, V, dt):
    """y_v = A x_v^(m-1), s_v = A x_v^m on the GPU against the oracle (FP64
    mode products) on the same values; repeated calls give identical bits."""
    import torch
    tdt = torch.float32 if dt == "f32" else torch.bfloat16
    A = synth.symmetric_uniform(m, n, (m, n, 95))
    X = synth.rng((m, n, 96)).standard_normal((V, n)).astype(np.float32)
    if dt == "bf16":
        A, X = synth.round_to_bf16(A), synth.round_to_bf16(X)
    Ab = st().bcss_pack(dev_dense(np.asarray(A, np.float32), tdt), m, n, b)
    Xd = torch.from_numpy(X).to(tdt).cuda()
    y, s, ws = st().sttsm_vectors(Ab, Xd, m, n, b)
    y2, s2, _ = st().sttsm_vectors(Ab, Xd, m, n, b, ws=ws)
    torch.cuda.synchronize()
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    Y, S = oracle.vectors(A64, X64)
    gy, gs = y.double().cpu().numpy(), s.double().cpu().numpy()
    ey = float(np.linalg.norm(gy - Y) / np.linalg.norm(Y))
    es = float(np.linalg.norm(gs - S) / np.linalg.norm(S))
    tol = TOL_FP32 if dt == "f32" else tol_bf16(m)
    say("vectors", m, n, b, V, dt, "rel err y", ey, "s", es)
    assert ey <= tol and es <= tol
    # entry by entry: y_v sums up to n^(m-1) terms and s_v n^m terms in one
    # FP32 accumulation each; the inputs are exact in the kernel's precision
    sy = np.array([oracle.error_scale(A64, X64[v:v + 1], last_mode=1).ravel() for v in range(V)])
    ss = np.array([oracle.error_scale(A64, X64[v:v + 1]).ravel()[0] for v in range(V)])
    check_entries(gy, Y, sy, P32, n ** (m - 1), what="y")
    check_entries(gs, S, ss, P32, n ** m, what="s")
    assert torch.equal(y, y2) and torch.equal(s, s2)


# ------------------------------------------------------------------ rank-update form (§8, second variant)
RANK_CASES = [(2, 37, 29, 8, 8, 1, P32), (2, 64, 64, 16, 16, 3, P32), (2, 100, 70, 16, 8, 2, PBF),
              (2, 50, 50, 8, 8, 2, PX3F), (3, 23, 19, 4, 4, 2, P32), (3, 40, 40, 8, 8, 1, PBF),
              (4, 13, 11, 3, 3, 2, P32), (2, 300, 200, 64, 64, 2, P32), (3, 35, 20, 16, 8, 5, P32)]


def _rank_inputs(m, n, p, prec, seed):
    import torch
    A = synth.symmetric_uniform(m, n, (m, n, seed))
    X = synth.change_of_basis(p, n, (m, n, seed + 1))
    tdt = torch.float32
    if prec == PBF:
        A, X, tdt = synth.round_to_bf16(A), synth.round_to_bf16(X), torch.bfloat16
    return A, X, tdt


@pytest.mark.parametrize("case", RANK_CASES)
def test_rank_update_vs_oracle(case):
    """sttsm_rank_update against the oracle's rank-update form (passes of the
    same size), over a C that starts as NaN: every entry is written, the
    padding comes out exactly zero."""
    import torch
    m, n, p, bA, bC, rows, prec = case
    say("rank-update", case)
    A, X, tdt = _rank_inputs(m, n, p, prec, 91)
    Ab = st().bcss_pack(dev_dense(np.asarray(A, np.float32), tdt), m, n, bA)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(tdt).cuda()
    nc = st().bcss_num_elems(m, p, bC)
    C0 = torch.full((nc,), float("nan"), dtype=torch.float32, device="cuda")
    C, _ = st().sttsm_rank_update(Ab, Xd, m, n, p, bA, bC, prec, rows, C=C0)
    torch.cuda.synchronize()
    got = C.double().cpu().numpy().reshape(-1, bC ** m)
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    ref = bcss_ref.pack(oracle.rank_update(A64, X64, bA, rows), bC)
    e = err(got, ref, m, p, bC)
    bound = {P32: TOL_FP32, PBF: tol_bf16(m), PX3F: TOL_X3_FIRST_FP32}[prec]
    say("  rel err", e, "bound", bound)
    assert e <= bound
    check_entries(got, ref, bcss_ref.pack(oracle.error_scale(A64, X64), bC), prec, -(-n // bA) * bA)
    assert np.all(got[padding_mask(m, p, bC)] == 0.0)


@pytest.mark.parametrize("case", [(2, 100, 70, 16, 8, P32), (3, 35, 20, 16, 8, P32), (3, 40, 40, 8, 8, PBF),
                                  (2, 300, 200, 64, 64, P32)])
def test_rank_update_one_pass_is_the_chain(case, monkeypatch):
    """One pass of every block row is the chain on the generic kernels, bit
    for bit; several passes give the same bits on every call."""
    import torch
    m, n, p, bA, bC, prec = case
    say("rank-update bitwise", case)
    monkeypatch.setenv("STTSM_GENERIC_KERNELS", "1")
    A, X, tdt = _rank_inputs(m, n, p, prec, 93)
    Ab = st().bcss_pack(dev_dense(np.asarray(A, np.float32), tdt), m, n, bA)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(tdt).cuda()
    nbar = -(-n // bA)
    C1, _ = st().sttsm(Ab, Xd, m, n, p, bA, bC, prec)
    C2, _ = st().sttsm_rank_update(Ab, Xd, m, n, p, bA, bC, prec, nbar)
    C2b, _ = st().sttsm_rank_update(Ab, Xd, m, n, p, bA, bC, prec, nbar + 3)   # more rows than there are
    C3, ws = st().sttsm_rank_update(Ab, Xd, m, n, p, bA, bC, prec, 2)
    C4, _ = st().sttsm_rank_update(Ab, Xd, m, n, p, bA, bC, prec, 2, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    assert torch.equal(C1, C2b)
    assert torch.equal(C3, C4)


# ------------------------------------------------------------------ m = 2, 64 x 64 blocks, bf16
B64_SHAPES = [(2, 64, 64), (2, 70, 65), (2, 200, 300), (2, 1000, 900), (2, 4096, 4096)]


@pytest.mark.parametrize("m,n,p", B64_SHAPES)
def test_bf16_b64_kernel(m, n, p):
    """bf16 inputs and temporaries, bA = bC = 64, through the kernel that
    stacks four row groups per tile (both levels, every tile width it picks):
    the whole C within the bf16 bound of the oracle run on the same bf16
    values and entry by entry, padding exactly zero; at n = p = 4096 also
    256 entries against the literal sum (O3)."""
    import torch
    b = 64
    for d in range(m):
        info = st().sttsm_plan_info(m, n, p, b, b, PBF, d, dtype=st().BF16)
        say("b64", (m, n, p), d, info)
        assert info["kernel"] == "bf16_b64"
    if n == 4096:
        A, X = synth.make_config_inputs("m2_n4096_b64")
    else:
        A = synth.symmetric_uniform(m, n, (m, n, p, 151))
        X = synth.change_of_basis(p, n, (m, n, p, 152))
    A, X = synth.round_to_bf16(A), synth.round_to_bf16(X)
    got = run(A, X, b, b, PBF, dtype=torch.bfloat16)
    ref, S = reference(A, X, b)
    e = err(got, ref, m, p, b)
    say("  rel err", e, "bound", tol_bf16(m))
    assert e <= tol_bf16(m)
    check_entries(got, ref, S, PBF, -(-n // b) * b)
    assert np.all(got[padding_mask(m, p, b)] == 0.0)
    if n == 4096:
        check_literal_entries({PBF: got}, A, X, b, ref, S, n)


# ------------------------------------------------------------------ X read in place
X_PLACE_CASES = [(3, 256, 256, 16, P32), (3, 100, 70, 16, P32), (3, 130, 60, 16, P32), (3, 64, 64, 16, PBF),
                 (2, 256, 256, 64, P32), (2, 256, 256, 64, PBF), (4, 40, 37, 8, P32)]


@pytest.mark.parametrize("m,n,p,b,prec", X_PLACE_CASES)
def test_x_in_place_equals_panels(m, n, p, b, prec, monkeypatch):
    """X read in place (an X of the panel's layout, or the FP32 block-copy
    kernel staging X itself, zeros past p and n) gives C bit for bit equal to
    the padded panels (STTSM_X_PANEL=1), for shapes that take either path."""
    import torch
    A = synth.symmetric_uniform(m, n, (m, n, p, 171))
    X = synth.change_of_basis(p, n, (m, n, p, 172))
    tdt = torch.bfloat16 if prec == PBF else torch.float32
    if prec == PBF:
        A, X = synth.round_to_bf16(A), synth.round_to_bf16(X)
    monkeypatch.delenv("STTSM_X_PANEL", raising=False)
    got = run(A, X, b, b, prec, dtype=tdt)
    monkeypatch.setenv("STTSM_X_PANEL", "1")
    ref = run(A, X, b, b, prec, dtype=tdt)
    say("x in place", (m, n, p, b, prec))
    assert np.array_equal(got, ref)
