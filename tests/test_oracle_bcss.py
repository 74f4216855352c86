"""Pins for the oracle's BCSS reference and its cost counts."""
import itertools
import json
import os
from math import comb

import numpy as np
import pytest

from oracle import bcss_ref, costs
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_packed_order_matches_section_3_3():
    """At b=1, m=2 the block order is the printed packing order 0 1 3 / 2 4 / 5."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "packed_order_m2.txt"))
            if ln.strip() and not ln.startswith("#")]
    index = bcss_ref.block_index(2, 3)
    for i, row in enumerate(rows):
        for j, tok in enumerate(row):
            if tok == ".":
                assert i > j
            else:
                assert index[(i, j)] == int(tok)


@pytest.mark.parametrize("m,nbar", [(m, nb) for m in range(1, 7) for nb in (1, 2, 3, 5, 8)])
def test_block_count(m, nbar):
    """Stored blocks = binom(nbar+m-1, m) (Table 1), by brute force."""
    assert len(bcss_ref.sorted_block_tuples(m, nbar)) == comb(nbar + m - 1, m)
    assert costs.enumerate_bcss_blocks(m, nbar) == comb(nbar + m - 1, m)


def test_storage_table_rows():
    """Table 1: compact count by enumerating sorted element tuples; BCSS count
    as b^m times the block count."""
    for m in range(1, 6):
        for n in (1, 3, 7):
            brute = sum(1 for _ in itertools.combinations_with_replacement(range(n), m))
            assert costs.storage_compact(n, m) == brute
            for b in (1, 2, 3):
                nbar = -(-n // b)
                assert costs.storage_bcss(n, m, b) == b ** m * len(bcss_ref.sorted_block_tuples(m, nbar))


def test_fig2_printed_ratios():
    """Figure 2's printed storage ratios at n=512, m=2, from the storage counts."""
    g = json.load(open(os.path.join(GOLDEN, "fig2_storage_ratios.json")))
    n = g["n"]
    for nbar, r_min, r_dense in zip(g["nbar"], g["relative_to_minimal"], g["relative_to_dense"]):
        b = n // nbar
        bcss = costs.storage_bcss(n, 2, b)
        assert round(costs.storage_compact(n, 2) / bcss, 2) == r_min
        assert round(n * n / bcss, 2) == r_dense
        a, d = costs.fig2_ratios(n, b)
        assert round(a, 2) == r_min and round(d, 2) == r_dense


@pytest.mark.parametrize("m,n,b", [(2, 6, 2), (2, 7, 3), (3, 5, 2), (3, 6, 3), (4, 5, 2), (5, 4, 3), (3, 4, 4), (2, 3, 5)])
def test_pack_unpack_roundtrip(m, n, b):
    """unpack(pack(A)) == A bit for bit for symmetric A, ragged n included;
    padding entries of the packed array are exactly zero."""
    A = synth.symmetric_uniform(m, n, (m, n, b))
    P = bcss_ref.pack(A, b)
    assert np.array_equal(bcss_ref.unpack(P, m, n, b), A)
    nbar = -(-n // b)
    # every padded position holds zero
    for r, s in enumerate(bcss_ref.sorted_block_tuples(m, nbar)):
        blk = P[r].reshape((b,) * m, order="F")
        for l in itertools.product(range(b), repeat=m):
            if any(sk * b + lk >= n for sk, lk in zip(s, l)):
                assert blk[l] == 0.0


@pytest.mark.parametrize("m,nbar,b", [(2, 3, 2), (3, 3, 2), (4, 2, 3)])
def test_pack_of_unpack_is_identity(m, nbar, b):
    """pack(unpack(B)) == B for ANY array B (stable sort leaves a sorted block
    unpermuted, so every stored block lands back in place)."""
    nb = comb(nbar + m - 1, m)
    B = synth.rng(m + nbar).standard_normal((nb, b ** m))
    n = nbar * b
    assert np.array_equal(bcss_ref.pack(bcss_ref.unpack(B, m, n, b), b), B)


def test_unpack_permutes_nonstored_blocks():
    """A non-symmetric block tensor shows the permutation: logical block (1,0)
    of an m=2 BCSS matrix is the transpose of stored block (0,1)."""
    b = 3
    B = np.arange(3 * b * b, dtype=np.float64).reshape(3, b * b)
    D = bcss_ref.unpack(B, 2, 2 * b, b)
    s01 = B[bcss_ref.block_index(2, 2)[(0, 1)]].reshape((b, b), order="F")
    assert np.array_equal(D[:b, b:], s01)
    assert np.array_equal(D[b:, :b], s01.T)


def test_rel_frobenius_bcss_matches_dense():
    """The multiplicity-weighted BCSS error equals the error of the unpacked
    dense tensors."""
    m, n, b = 3, 7, 3
    A = synth.symmetric_uniform(m, n, 1).astype(np.float64)
    B = A + 1e-3 * synth.symmetric_uniform(m, n, 2)
    e = bcss_ref.rel_frobenius_bcss(bcss_ref.pack(B, b), bcss_ref.pack(A, b), m, n, b)
    ref = np.linalg.norm((B - A).ravel()) / np.linalg.norm(A.ravel())
    assert abs(e - ref) <= 1e-12 * ref


# ------------------------------------------------------------------ cost counts
CASES = [(m, n, p, bA, bC) for m in range(1, 7) for (n, p) in ((8, 8), (12, 6), (7, 10))
         for bA in (1, 2, 4) for bC in (1, 2, 3)]


@pytest.mark.parametrize("m,n,p,bA,bC", CASES)
def test_enumerated_flops_equal_table2(m, n, p, bA, bC):
    """Walking the loops of Figure 6 with partial symmetry exploited gives
    exactly Table 2's BCSS flop count (integers, padded sizes)."""
    nbar, pbar = -(-n // bA), -(-p // bC)
    assert costs.enumerate_flops(m, n, p, bA, bC) == costs.flops_table_mincosts(m, nbar, pbar, bA, bC)


@pytest.mark.parametrize("m,n", [(2, 6), (3, 5), (4, 4), (5, 3), (6, 3)])
def test_unit_blocks_reach_the_minimum(m, n):
    """bA = bC = 1, p = n: Table 2 equals the minimum cost of §6.5."""
    assert costs.flops_table_mincosts(m, n, n, 1, 1) == costs.flops_minimum(m, n)


@pytest.mark.parametrize("n,b", [(8, 2), (12, 4), (16, 16), (9, 3)])
def test_matrix_case_matches_figure3(n, b):
    """m=2 (nothing left to exploit in T^(1)): Table 2 equals Figure 3's total
    2 bC n^2 pbar + 2 bC^2 n pbar(pbar+1)/2."""
    pbar = n // b
    fig3 = 2 * b * n * n * pbar + 2 * b * b * n * pbar * (pbar + 1) // 2
    assert costs.flops_table_mincosts(2, n // b, pbar, b, b) == fig3 == costs.flops_fig_mD(2, n, pbar, b)


@pytest.mark.parametrize("m", [3, 4, 5])
def test_partial_symmetry_saves_work(m):
    """For m >= 3 the partial symmetry of the temporaries strictly lowers the
    flop count below Figure 6's total, which forms every temporary block."""
    n, b = 16, 4
    assert costs.flops_table_mincosts(m, n // b, n // b, b, b) < costs.flops_fig_mD(m, n, n // b, b)


def test_stage_counts_match_figure6_column():
    """Level d runs binom(pbar+d, d+1) times (Figure 6's '# times executed'
    column) over binom(nbar+m-d-2, m-d-1) unique output prefixes."""
    m, n, p, b = 5, 12, 9, 3
    for lv in costs.enumerate_stage_work(m, n, p, b, b):
        d = lv["d"]
        assert lv["jtuples"] == comb(-(-p // b) + d, d + 1)
        assert lv["prefixes"] == comb(n // b + m - d - 2, m - d - 1)


def test_workload_flop_totals():
    """Symmetry-aware GFLOP of the measured workloads (Table 2)."""
    # m=3, n=p=256, b=16: 16 x 136 + 136 x 16 + 816 x 1 block updates of
    # 2 * 256 * 16^3 flops each
    per_block = 2 * 256 * 16 ** 3
    assert costs.flops_table_mincosts(3, 16, 16, 16, 16) == (16 * 136 + 136 * 16 + 816) * per_block
    assert costs.flops_table_mincosts(3, 16, 16, 16, 16) == 10_838_081_536
    assert costs.flops_table_mincosts(3, 4, 4, 4, 4) == 204_800
    # Dense temporaries algorithm for comparison (§5.2): 25.8 GFLOP at n=p=256
    assert costs.flops_dense(3, 256, 256) == 6 * 256 ** 4


def test_limit_approximation_of_table3():
    """Table 3 (§6.4) approximates the BCSS count by (2n)^(m+1)/m! via the
    Vandermonde identity.  At bA = bC = 1, p = n, the exact count of Table 2
    stays below that estimate, and the gap closes as m grows (the estimate
    drops lower-order terms).  The dense-to-BCSS ratio of the exact counts
    grows with m, as the O((m+1)!/2^m) claim says."""
    from math import factorial
    n = 4096
    gaps, ratios = [], []
    for m in (2, 3, 4, 5):
        exact = costs.flops_table_mincosts(m, n, n, 1, 1)
        approx = (2 * n) ** (m + 1) / factorial(m)
        assert exact < approx
        gaps.append(approx / exact)
        ratios.append(costs.flops_dense(m, n, n) / exact)
    assert gaps == sorted(gaps, reverse=True) and gaps[-1] < 1.04
    assert ratios == sorted(ratios)


# ------------------------------------------------------------------ symmetrisation (end of §5.4)
def test_symmetrize_matrix_case():
    """m = 2: a diagonal block becomes (M + M^T)/2, other blocks are kept."""
    m, n, b = 2, 6, 3
    tuples = bcss_ref.sorted_block_tuples(m, 2)
    X = synth.rng(5).standard_normal((len(tuples), b * b))
    Y = bcss_ref.symmetrize(X, m, n, b)
    for r, s in enumerate(tuples):
        M = X[r].reshape(b, b, order="F")
        want = (M + M.T) / 2 if s[0] == s[1] else M
        assert np.allclose(Y[r].reshape(b, b, order="F"), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("m,n,b", [(3, 6, 2), (3, 7, 3), (4, 5, 2)])
def test_symmetrize_invariants(m, n, b):
    """Output is a symmetric tensor; symmetrising twice changes nothing; an
    exactly symmetric input is returned (to rounding); the sum over every
    dense permutation orbit is kept."""
    nb = len(bcss_ref.sorted_block_tuples(m, -(-n // b)))
    X = synth.rng((m, n, b)).standard_normal((nb, b ** m))
    Y = bcss_ref.symmetrize(X, m, n, b)
    D = bcss_ref.unpack(Y, m, n, b)
    for p in itertools.permutations(range(m)):
        assert np.allclose(np.transpose(D, p), D, rtol=0, atol=1e-14)
    assert np.allclose(bcss_ref.symmetrize(Y, m, n, b), Y, rtol=0, atol=1e-14)
    A = synth.symmetric_uniform(m, n, (m, n, 3)).astype(np.float64)
    P = bcss_ref.pack(A, b)
    assert np.allclose(bcss_ref.symmetrize(P, m, n, b), P, rtol=0, atol=1e-15)
    assert abs(bcss_ref.unpack(X, m, n, b).sum() - D.sum()) <= 1e-10 * np.abs(D).sum()
