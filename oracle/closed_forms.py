"""Closed forms for sttsm that hold without any algorithm (O4).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def matrix_case(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """m = 2: [A; X, X] = X A X^T (§3.1), by a library matrix product in FP64."""
    A64 = np.asarray(A, dtype=np.float64)
    X64 = np.asarray(X, dtype=np.float64)
    return X64 @ A64 @ X64.T


def outer_power(v: np.ndarray, m: int) -> np.ndarray:
    """v o v o ... o v (m factors) as a Fortran-ordered dense tensor."""
    out = np.asarray(v, dtype=np.float64)
    for _ in range(m - 1):
        out = np.multiply.outer(out, v)
    return np.asfortranarray(out)


def rank_r(lams, vecs, X: np.ndarray, m: int) -> np.ndarray:
    """C for A = sum_i lam_i a_i^{o m}:  sum_i lam_i (X a_i)^{o m}.

    Follows from the multilinearity of the defining sum in §2.5: every mode
    multiplies the same vector a_i by X.  This is the symmetric CP form the
    paper names as a use of sttsm (§2.5)."""
    X64 = np.asarray(X, dtype=np.float64)
    out = None
    for lam, a in zip(lams, vecs):
        term = lam * outer_power(X64 @ np.asarray(a, dtype=np.float64), m)
        out = term if out is None else out + term
    return np.asfortranarray(out)


def rank_r_all_but_one(lams, vecs, X: np.ndarray, m: int) -> np.ndarray:
    """A x_1 X ... x_{m-1} X for A = sum_i lam_i a_i^{o m}:
    sum_i lam_i a_i o (X a_i)^{o (m-1)} (multilinearity of the mode products;
    mode 0 keeps a_i)."""
    X64 = np.asarray(X, dtype=np.float64)
    out = None
    for lam, a in zip(lams, vecs):
        a64 = np.asarray(a, dtype=np.float64)
        term = lam * np.multiply.outer(a64, outer_power(X64 @ a64, m - 1)) if m > 1 else lam * a64
        out = term if out is None else out + term
    return np.asfortranarray(out)


def rank_r_vectors(lams, vecs, X: np.ndarray, m: int):
    """For A = sum_i lam_i a_i^{o m} and rows x of X:
    A x^(m-1) = sum_i lam_i (a_i . x)^(m-1) a_i and A x^m = sum_i lam_i (a_i . x)^m."""
    X64 = np.asarray(X, dtype=np.float64)
    Av = np.asarray(vecs, dtype=np.float64)          # r x n
    dots = X64 @ Av.T                                  # V x r
    lam = np.asarray(lams, dtype=np.float64)
    Y = (dots ** (m - 1) * lam) @ Av
    s = (dots ** m) @ lam
    return Y, s
