"""Independent reference for Blocked Compact Symmetric Storage (BCSS).

TEST INFRASTRUCTURE ONLY (see the package docstring).

BCSS (§3.3 for m=2, §4.3 for m=3, §5.3 for general m): partition the
symmetric tensor into b^m blocks and store only the blocks whose block index is
sorted, s_0 <= s_1 <= ... <= s_{m-1} (the "upper hypertriangle"); each block is
stored whole, in dimensional order, with no use of symmetry inside it.

Readings where the paper leaves a choice open:
  * Block order: colex, i.e. sorted by the reversed tuple.  At b=1, m=2 this is
    exactly the element packing order printed in §3.3 (0 1 3 / 2 4 / 5).
  * Ragged n (n not a multiple of b): the tensor is padded with zeros to
    ceil(n/b)*b in every mode; padding is never read back by unpack.
  * A non-stored block t is read from the stored block sort(t), whose modes are
    permuted by the STABLE argsort of t.

Everything here is plain enumeration (itertools) and NumPy slicing: no closed
form ranking, no stride tables.
"""
from __future__ import annotations

import itertools

import numpy as np


def sorted_block_tuples(m: int, nbar: int):
    """All sorted m-tuples over [0, nbar), in colex order (key: reversed tuple)."""
    tuples = list(itertools.combinations_with_replacement(range(nbar), m))
    tuples.sort(key=lambda t: tuple(reversed(t)))
    return tuples


def block_index(m: int, nbar: int):
    """dict sorted tuple -> position in the BCSS block list."""
    return {t: r for r, t in enumerate(sorted_block_tuples(m, nbar))}


def _padded(dense: np.ndarray, b: int) -> np.ndarray:
    m = dense.ndim
    n = dense.shape[0]
    nbar = -(-n // b)
    out = np.zeros((nbar * b,) * m, dtype=dense.dtype, order="F")
    out[tuple(slice(0, n) for _ in range(m))] = dense
    return out


def pack(dense: np.ndarray, b: int) -> np.ndarray:
    """Dense symmetric tensor -> BCSS array of shape (num_blocks, b^m).

    Row r holds the r-th sorted block (colex order) flattened in dimensional
    order; entries beyond n are zero.  Only sorted blocks are read.
    """
    m = dense.ndim
    n = dense.shape[0]
    nbar = -(-n // b)
    pad = _padded(np.asfortranarray(dense), b)
    blocks = sorted_block_tuples(m, nbar)
    out = np.zeros((len(blocks), b ** m), dtype=dense.dtype)
    for r, s in enumerate(blocks):
        sub = pad[tuple(slice(sk * b, (sk + 1) * b) for sk in s)]
        out[r] = sub.ravel(order="F")
    return out


def unpack(bcss: np.ndarray, m: int, n: int, b: int) -> np.ndarray:
    """BCSS array -> dense tensor (Fortran order), every block from a stored one.

    Logical block t is the stored block u = sorted(t) with its modes permuted:
    with sigma the stable argsort of t (u_i = t_{sigma_i}), logical element
    (l_0..l_{m-1}) equals stored element (l_{sigma_0}, ..., l_{sigma_{m-1}}).
    """
    nbar = -(-n // b)
    index = block_index(m, nbar)
    if bcss.shape != (len(index), b ** m):
        raise ValueError("BCSS array has the wrong shape")
    pad = np.zeros((nbar * b,) * m, dtype=bcss.dtype, order="F")
    for t in itertools.product(range(nbar), repeat=m):
        sigma = sorted(range(m), key=lambda i: t[i])          # stable
        u = tuple(t[i] for i in sigma)
        stored = bcss[index[u]].reshape((b,) * m, order="F")
        # logical[l] = stored[l[sigma_0], ..., l[sigma_{m-1}]]
        inv = np.argsort(sigma)
        logical = np.transpose(stored, axes=inv)
        pad[tuple(slice(tk * b, (tk + 1) * b) for tk in t)] = logical
    return np.asfortranarray(pad[tuple(slice(0, n) for _ in range(m))])


def block_multiplicity(s) -> int:
    """Number of distinct permutations of the block tuple s (how many dense
    blocks the stored block s stands for)."""
    from math import factorial
    from collections import Counter
    out = factorial(len(s))
    for c in Counter(s).values():
        out //= factorial(c)
    return out


def rel_frobenius_bcss(got: np.ndarray, ref: np.ndarray, m: int, p: int, b: int) -> float:
    """Relative Frobenius error of two BCSS arrays measured over the dense
    tensor they stand for: each stored block is weighted by its multiplicity.
    Padding entries are included, and are exactly zero in a correct result."""
    nbar = -(-p // b)
    w = np.array([block_multiplicity(s) for s in sorted_block_tuples(m, nbar)], dtype=np.float64)
    d = (np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    num = float(np.sum(w * np.sum(d * d, axis=1)))
    den = float(np.sum(w * np.sum(np.asarray(ref, np.float64) ** 2, axis=1)))
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


def symmetrize(bcss: np.ndarray, m: int, n: int, b: int) -> np.ndarray:
    """The post-processing of §5.4 that removes the asymmetry inside blocks:
    the dense tensor BCSS represents (unpack), averaged over all m! mode
    permutations, packed again.  FP64; returns (num_blocks, b^m)."""
    D = unpack(np.asarray(bcss, dtype=np.float64), m, n, b)
    acc = np.zeros_like(D)
    perms = list(itertools.permutations(range(m)))
    for p in perms:
        acc += np.transpose(D, p)
    return pack(acc / len(perms), b)
