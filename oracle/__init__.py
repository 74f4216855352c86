"""FP64 CPU oracle for the sttsm operation C := [A; X, ..., X].

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1301_7744_amd``) and never imports it.

Paper: Schatz, Low, van de Geijn, Kolda, "Exploiting Symmetry in Tensors for
High Performance: Multiplication with Symmetric Tensors" (arXiv:1301.7744).

Dense tensors here are NumPy arrays in Fortran order, indexed naturally as
``T[i_0, ..., i_{m-1}]``; their memory order is then the paper's dimensional
order (App. A).  X is a (p, n) array, ``X[j, i] = chi_{j i}``.

Components
  direct_sum  (O1)  literal sum of §2.5 over all n^m terms, every output entry
  chain       (O2)  successive dense mode products (§5.2, Figure 1 bottom right)
  rank_update       the rank-update form of §8 (C as a sum of rank-b updates)
  entry       (O3)  one output entry by the literal sum
  entries     (O3)  many entries by the literal sum, each with its
                    root-sum-square of terms (the rounding-error scale)
  term_rss          that root-sum-square for every entry (O2 on A*A, X*X)
  error_scale       per-entry 2-norm of the first-order sensitivities to every
                    operand entry of the chain (the entry-by-entry error scale)
  closed_forms (O4) m=2 matrix identity, rank-1 / rank-r forms
  bcss_ref          independent BCSS enumerator, pack and unpack
  costs             storage / work counts by enumeration and by the paper's formulas
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O3, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_entry.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, i64p, dp]
        lib.oracle_entries.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_int64,
                                       i64p, dp, dp]
        lib.oracle_direct_sum.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, dp]
        lib.oracle_mode_product.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int, dp, ctypes.c_int64, dp]
        lib.oracle_chain.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, dp,
                                     ctypes.POINTER(dp)]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        for f in (lib.oracle_entry, lib.oracle_entries, lib.oracle_direct_sum, lib.oracle_mode_product,
                  lib.oracle_chain, lib.oracle_num_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_dense_f64(T: np.ndarray) -> np.ndarray:
    return np.asfortranarray(np.asarray(T, dtype=np.float64))


def _check(A: np.ndarray, X: np.ndarray):
    m = A.ndim
    p, n = X.shape
    if m < 1 or m > 8 or any(d != n for d in A.shape):
        raise ValueError("A must be order 1..8 with every extent equal to X.shape[1]")
    return m, n, p


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for the oracle's following OpenMP loops."""
    _load().oracle_set_num_threads(int(n))


def entry(A: np.ndarray, X: np.ndarray, j) -> float:
    """O3: one entry gamma_j by the literal n^m-term sum (§2.5)."""
    m, n, p = _check(A, X)
    A64, X64 = _as_dense_f64(A), np.ascontiguousarray(X, dtype=np.float64)
    jj = np.ascontiguousarray(j, dtype=np.int64)
    if jj.shape != (m,):
        raise ValueError("j must have m entries")
    out = ctypes.c_double(0.0)
    rc = _load().oracle_entry(m, n, p, _dptr(A64), _dptr(X64),
                              jj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(out))
    if rc:
        raise ValueError("oracle_entry rejected its arguments")
    return out.value


def entries(A: np.ndarray, X: np.ndarray, js):
    """O3 for many output tuples (js: (count, m) integers): each entry by the
    literal n^m-term sum of §2.5, and the root-sum-square of the same terms,
    sqrt(sum_i t_i^2), the scale against which an entry's rounding error is
    measured.  Returns (sums, rss), float64 arrays of length count."""
    m, n, p = _check(A, X)
    A64, X64 = _as_dense_f64(A), np.ascontiguousarray(X, dtype=np.float64)
    J = np.ascontiguousarray(js, dtype=np.int64).reshape(-1, m)
    sums = np.zeros(J.shape[0])
    rss = np.zeros(J.shape[0])
    rc = _load().oracle_entries(m, n, p, _dptr(A64), _dptr(X64), J.shape[0],
                                J.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(sums), _dptr(rss))
    if rc:
        raise ValueError("oracle_entries rejected its arguments")
    return sums, rss


def term_rss(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """For every output entry j, sqrt(sum_i t_i^2) over the n^m terms
    t_i = alpha_i chi_{j_0 i_0} ... chi_{j_{m-1} i_{m-1}} of §2.5: the
    squared terms are the terms of the same operation on the entrywise
    squares of A and X, so this is the O2 chain on (A*A, X*X), then a square
    root.  Dense, FP64, Fortran order, extent p in every mode."""
    A64, X64 = _as_dense_f64(A), np.asarray(X, dtype=np.float64)
    return np.sqrt(chain(A64 * A64, X64 * X64))


def error_scale(A: np.ndarray, X: np.ndarray, last_mode: int = 0, temps=None) -> np.ndarray:
    """Per-entry rounding-error scale of the chain of mode products (§5.2,
    §6), for a symmetric A.

    The chain runs modes m-1, m-2, ..., last_mode (last_mode = 0 is sttsm,
    last_mode = 1 the product in every mode but mode 0 of §2.5).  Its
    operands are the entries of A, the entries of every temporary
    T^(k) = A x_(m-1) X ... x_k X (k = last_mode+1 .. m-1) and the entries of
    X used in each contracted mode.  A relative change delta of one operand
    entry e changes output entry j by delta * e * d(out_j)/de to first order.
    This returns, for every output entry j,

        S_j = sqrt( sum over every operand entry e of (e * d(out_j)/de)^2 ),

    the 2-norm of those sensitivities, computed as sums of squared terms:
      * A entries:   (A*A) x_(m-1) (X*X) ... x_last (X*X)  (the terms of the
        same operation on entrywise squares);
      * T^(k) entries: (T^(k)*T^(k)) x_(k-1) (X*X) ... x_last (X*X);
      * X entries in mode l: the sensitivity to chi_(j_l, i) is the output
        with mode l left uncontracted, which for symmetric A is T^(last+1)
        with its free mode `last` moved to l (Theorem 1 and the symmetry of
        A), so this part is (T^(last+1)^2 x_last (X*X)) with mode `last`
        moved to l, summed over l = last..m-1 (T^(m) meaning A).
    An independent relative rounding of every operand entry by at most u
    then gives an error of about u * S_j / sqrt(3) in entry j (sharing of one
    rounded value between mirrored positions raises this by at most the
    square root of the number of positions that share it).

    Dense, FP64, Fortran order, the shape of the chain's output.  `temps`
    may pass the {k: T^(k)} of chain(A, X, keep_temps=True) to skip
    recomputing them."""
    A = _as_dense_f64(A)
    X = np.asarray(X, dtype=np.float64)
    m, n, p = _check(A, X)
    s = int(last_mode)
    if s < 0 or s >= m:
        raise ValueError("last_mode must be in 0..m-1")
    if m == 2 and s == 0:
        # The same three parts by library matrix products (§3.1: the m = 2
        # chain is T^(1) = A X^T, C = X T^(1)); X2 A2 X2^T is the A part,
        # X2 (T^(1))^2 the T^(1) part and the mode-0 X part, its transpose
        # the mode-1 X part.
        X2 = X * X
        T1 = A @ X.T
        Q = X2 @ (T1 * T1)
        return np.asfortranarray(np.sqrt(X2 @ (A * A) @ X2.T + 2.0 * Q + Q.T))
    if temps is None and s + 1 < m:
        _, temps = chain(A, X, keep_temps=True)
    X2 = X * X

    def contract(T, hi):
        for k in range(hi, s - 1, -1):
            T = mode_product(T, k, X2)
        return T

    S2 = contract(A * A, m - 1)
    for k in range(s + 1, m):
        S2 += contract(temps[k] * temps[k], k - 1)
    W = temps[s + 1] if s + 1 < m else A
    Q = mode_product(W * W, s, X2)
    del W
    for l in range(s, m):
        S2 += np.moveaxis(Q, s, l)
    return np.sqrt(S2)


def direct_sum(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """O1: every entry of C by the literal sum of §2.5; cost (m+1) n^m p^m."""
    m, n, p = _check(A, X)
    A64, X64 = _as_dense_f64(A), np.ascontiguousarray(X, dtype=np.float64)
    C = np.zeros((p,) * m, dtype=np.float64, order="F")
    rc = _load().oracle_direct_sum(m, n, p, _dptr(A64), _dptr(X64), _dptr(C))
    if rc:
        raise ValueError("oracle_direct_sum rejected its arguments")
    return C


def mode_product(T: np.ndarray, k: int, B: np.ndarray) -> np.ndarray:
    """out = T x_k B (App. A): B is (J, T.shape[k]); out has extent J in mode k."""
    T64 = _as_dense_f64(T)
    B64 = np.ascontiguousarray(B, dtype=np.float64)
    if B64.ndim != 2 or B64.shape[1] != T64.shape[k]:
        raise ValueError("B must be (J, T.shape[k])")
    dims = np.asarray(T64.shape, dtype=np.int64)
    shape = list(T64.shape)
    shape[k] = B64.shape[0]
    out = np.zeros(shape, dtype=np.float64, order="F")
    rc = _load().oracle_mode_product(T64.ndim, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     _dptr(T64), k, _dptr(B64), B64.shape[0], _dptr(out))
    if rc:
        raise ValueError("oracle_mode_product rejected its arguments")
    return out


def chain(A: np.ndarray, X: np.ndarray, keep_temps: bool = False):
    """O2: C by successive dense mode products, mode m-1 first (§5.2, Figure 1).

    With keep_temps, also returns {k: T^(k)} for k = 1..m-1, where T^(k) has
    extent n in modes 0..k-1 and p in modes k..m-1.
    """
    m, n, p = _check(A, X)
    A64, X64 = _as_dense_f64(A), np.ascontiguousarray(X, dtype=np.float64)
    C = np.zeros((p,) * m, dtype=np.float64, order="F")
    temps = {}
    tptrs = None
    if keep_temps and m > 1:
        arr_t = ctypes.POINTER(ctypes.c_double) * m
        tptrs = arr_t()
        for k in range(1, m):
            temps[k] = np.zeros((n,) * k + (p,) * (m - k), dtype=np.float64, order="F")
            tptrs[k] = _dptr(temps[k])
    rc = _load().oracle_chain(m, n, p, _dptr(A64), _dptr(X64), _dptr(C), tptrs)
    if rc:
        raise MemoryError("oracle_chain failed (%d)" % rc)
    return (C, temps) if keep_temps else C


def all_but_one(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """A x_1 X x_2 X ... x_{m-1} X: the product in every mode but mode 0, the
    related operation §2.5 names beside sttsm; dense FP64, Fortran order,
    extent n in mode 0 and p in the others.  Computed as the same mode
    products as chain(), in the same order, stopping before mode 0."""
    A = _as_dense_f64(A)
    X = np.asarray(X, dtype=np.float64)
    _check(A, X)
    m = A.ndim
    if m < 2:
        raise ValueError("needs order m >= 2")
    T = A
    for k in range(m - 1, 0, -1):
        T = mode_product(T, k, X)
    return T



def rank_update(A: np.ndarray, X: np.ndarray, b: int, rows: int = 1) -> np.ndarray:
    """The rank-update form of sttsm, the second algorithmic variant of §8.
    The paper gives it for m = 2: with A split into rows A_i and X into
    columns X_i, C = X A X^T = sum_i X_i (A_i X^T).  For order m the rows
    of A x_1 X ... x_{m-1} X (all_but_one) take the place of A_i X^T, and
    each adds its product with column block X_{:, i} in mode 0 to C.  Rows
    go in blocks of b (the last one ragged), `rows` blocks per pass, passes
    in increasing i.  FP64, Fortran order, extent p in every mode."""
    A = _as_dense_f64(A)
    X = np.asarray(X, dtype=np.float64)
    m, n, p = _check(A, X)
    if m < 2:
        raise ValueError("needs order m >= 2")
    if b < 1 or rows < 1:
        raise ValueError("b and rows must be >= 1")
    Y = all_but_one(A, X)
    C = np.zeros((p,) * m, dtype=np.float64, order="F")
    w = b * rows
    for i0 in range(0, n, w):
        i1 = min(i0 + w, n)
        C += mode_product(Y[i0:i1], 0, X[:, i0:i1])
    return C


def vectors(A: np.ndarray, X: np.ndarray):
    """The sttsm case of §2.5 where the matrix is one vector, for each row
    x_v of X (V x n): y_v = A x_v^(m-1) (every mode but mode 0 multiplied by
    x_v) and s_v = A x_v^m (every mode).  Returns (Y (V x n), s (V,)), FP64,
    from the same dense mode products as all_but_one() and chain()."""
    A = _as_dense_f64(A)
    X = np.asarray(X, dtype=np.float64)
    V, n = X.shape
    Y = np.zeros((V, n))
    s = np.zeros(V)
    for v in range(V):
        xv = X[v:v + 1, :]
        Y[v] = all_but_one(A, xv).reshape(n, order="F")
        s[v] = float(chain(A, xv).ravel()[0])
    return Y, s
