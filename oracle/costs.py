"""Storage and work counts for BCSS sttsm: by enumeration and by the paper's
closed forms.  Each closed form is typed from the passage it cites; each
enumeration walks the loops it counts.  Tests pin one against the other and
against the numbers the paper prints.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import itertools
from math import comb


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


# ---------------------------------------------------------------- closed forms
def storage_compact(n: int, m: int) -> int:
    """Unique entries of an order-m symmetric tensor, binom(n+m-1, m)
    (Table 1, 'Compact (Minimum)' column)."""
    return comb(n + m - 1, m)


def storage_bcss(n: int, m: int, b: int) -> int:
    """BCSS entries b^m binom(nbar+m-1, m) (Table 1, BCSS column)."""
    return b ** m * comb(ceil_div(n, b) + m - 1, m)


def storage_bcss_m2_formula(n: int, b: int) -> float:
    """m=2 BCSS entries n(n+b)/2 (§3.3), valid when b divides n."""
    return n * (n + b) / 2


def fig2_ratios(n: int, b: int):
    """Figure 2 rows: minimal/BCSS = (n(n+1)/2)/(n(n+b)/2) and
    dense/BCSS = n^2/(n(n+b)/2)."""
    bc = storage_bcss_m2_formula(n, b)
    return (n * (n + 1) / 2) / bc, (n * n) / bc


def flops_table_mincosts(m: int, nbar: int, pbar: int, bA: int, bC: int) -> int:
    """Table 2 (§6.4), BCSS computation row, in exact integers:
    2 nbar bC bA^m sum_{d=0}^{m-1} binom(pbar+d, d+1) binom(nbar+m-d-2, m-d-1) (bC/bA)^d.
    Multiplying through by bA^d keeps it integral: bA^m (bC/bA)^d = bA^(m-d) bC^d."""
    total = 0
    for d in range(m):
        total += comb(pbar + d, d + 1) * comb(nbar + m - d - 2, m - d - 1) * bA ** (m - d) * bC ** d
    return 2 * nbar * bC * total


def flops_fig_mD(m: int, n: int, pbar: int, bC: int) -> int:
    """Figure 6 total (no partial symmetry in the temporaries):
    sum_{d=0}^{m-1} 2 bC^(d+1) n^(m-d) binom(pbar+d, d+1)."""
    return sum(2 * bC ** (d + 1) * n ** (m - d) * comb(pbar + d, d + 1) for d in range(m))


def flops_minimum(m: int, n: int) -> int:
    """§6.5, bA=bC=1 and p=n: 2n sum_d binom(n+d, d+1) binom(n+m-d-2, m-d-1)."""
    return 2 * n * sum(comb(n + d, d + 1) * comb(n + m - d - 2, m - d - 1) for d in range(m))


def flops_dense(m: int, n: int, p: int) -> int:
    """Dense temporaries algorithm, 2 sum_{i=0}^{m-1} p^(i+1) n^(m-i) (§5.2)."""
    return 2 * sum(p ** (i + 1) * n ** (m - i) for i in range(m))


def flops_naive(m: int, n: int, p: int) -> int:
    """Naive algorithm over every output entry, (m+1) p^m n^m (§5.2)."""
    return (m + 1) * p ** m * n ** m


# ----------------------------------------------------------------- enumeration
def enumerate_stage_work(m: int, n: int, p: int, bA: int, bC: int):
    """Walk the loops of the algorithm-by-blocks (Figure 6) with the partial
    symmetry of the temporaries exploited (§6.1-6.3).

    Loop level d = 0..m-1 forms T^(m-1-d) (level m-1 forms C).  It runs once per
    sorted tuple (jbar_{m-1-d} <= ... <= jbar_{m-1}) of C-block indices, and in
    each run updates only the unique output blocks: the sorted prefixes
    (ibar_0 <= ... <= ibar_{m-2-d}) of the symmetric modes 0..m-2-d (Theorem 1).
    Each output block has bA^(m-1-d) bC^(d+1) entries and takes 2 * nbar*bA
    flops per entry (one multiply and one add per term of the mode product over
    the full padded dimension).

    Returns a list of dicts, one per level, with the enumerated counts.
    """
    nbar, pbar = ceil_div(n, bA), ceil_div(p, bC)
    levels = []
    for d in range(m):
        k = m - 1 - d                      # mode contracted at this level
        jtuples = sum(1 for _ in itertools.combinations_with_replacement(range(pbar), d + 1))
        prefixes = sum(1 for _ in itertools.combinations_with_replacement(range(nbar), k))
        block_entries = bA ** k * bC ** (d + 1)
        flops = 0
        for _j in range(jtuples):
            for _s in range(prefixes):
                flops += 2 * nbar * bA * block_entries
        levels.append(dict(d=d, mode=k, jtuples=jtuples, prefixes=prefixes,
                           block_entries=block_entries, flops=flops))
    return levels


def enumerate_flops(m: int, n: int, p: int, bA: int, bC: int) -> int:
    return sum(lv["flops"] for lv in enumerate_stage_work(m, n, p, bA, bC))


def enumerate_bcss_blocks(m: int, nbar: int) -> int:
    """Count blocks in the upper hypertriangle by brute force over all nbar^m."""
    return sum(1 for t in itertools.product(range(nbar), repeat=m)
               if all(t[i] <= t[i + 1] for i in range(m - 1)))
