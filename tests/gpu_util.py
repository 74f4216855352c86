"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from oracle import bcss_ref

# Tolerances on the relative Frobenius error over the dense C (padding
# excluded, mirrored blocks weighted by their multiplicity).
TOL_FP32 = 1e-5


def tol_bf16(m: int) -> float:
    """BF16 operands and temporaries, FP32 accumulation: sqrt(2m) 2^-8."""
    return (2 * m) ** 0.5 * 2.0 ** -8


TOL_X3_FIRST_FP32 = 2e-5
TOL_X3_STAGE0 = 1e-5


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def dev_dense(A: np.ndarray, dtype=None):
    """Fortran-ordered numpy tensor -> flat torch device tensor in
    dimensional order."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(A.ravel(order="F")))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run(A: np.ndarray, X: np.ndarray, bA: int, bC: int, prec: int, dtype=None, keep_ws=False):
    """Pack A on the GPU, run sttsm, return C's BCSS array as float64
    (num_blocks, bC^m) and optionally the workspace."""
    import torch
    import paper_1301_7744_amd as st
    m = A.ndim
    n = A.shape[0]
    p = X.shape[0]
    tdt = dtype or torch.float32
    Ad = dev_dense(np.asarray(A, np.float32), tdt)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(tdt).cuda()
    Ab = st.bcss_pack(Ad, m, n, bA)
    C, ws = st.sttsm(Ab, Xd, m, n, p, bA, bC, prec)
    torch.cuda.synchronize()
    nb = st.bcss_num_blocks(m, -(-p // bC))
    Cn = C.cpu().numpy().astype(np.float64).reshape(nb, bC ** m)
    return (Cn, ws) if keep_ws else Cn


def ref_bcss(A: np.ndarray, X: np.ndarray, bC: int, method: str = "chain") -> np.ndarray:
    """Oracle C, packed by the oracle's own BCSS enumerator (float64)."""
    if method == "direct":
        Cd = oracle.direct_sum(A, X)
    else:
        Cd = oracle.chain(A, X)
    return bcss_ref.pack(Cd, bC)


def err(got: np.ndarray, ref: np.ndarray, m: int, p: int, bC: int) -> float:
    return bcss_ref.rel_frobenius_bcss(got, ref, m, p, bC)


def padding_mask(m: int, p: int, b: int) -> np.ndarray:
    """Boolean (num_blocks, b^m): True where the entry lies beyond p."""
    pbar = -(-p // b)
    tuples = bcss_ref.sorted_block_tuples(m, pbar)
    loc = np.indices((b,) * m).reshape(m, -1, order="F")      # local index per entry, dimensional order
    mask = np.zeros((len(tuples), b ** m), dtype=bool)
    for r, s in enumerate(tuples):
        g = np.array(s)[:, None] * b + loc
        mask[r] = np.any(g >= p, axis=0)
    return mask
