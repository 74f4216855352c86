"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import synth
from oracle import bcss_ref

# Tolerances on the relative Frobenius error over the dense C (padding
# excluded, mirrored blocks weighted by their multiplicity).
TOL_FP32 = 1e-5


def tol_bf16(m: int) -> float:
    """BF16 operands and temporaries, FP32 accumulation: sqrt(2m) 2^-8."""
    return (2 * m) ** 0.5 * 2.0 ** -8


TOL_X3_FIRST_FP32 = 2e-5
TOL_X3_STAGE0 = 1e-5

P32, PBF, PX3F, PX3B = 0, 1, 2, 3

# Entry-by-entry bound, beside the Frobenius one: every entry j of the
# result must satisfy |C_gpu_j - C_ref_j| <= TAU * u * S_j, where S_j is
# oracle.error_scale (the 2-norm of the entry's first-order sensitivities to
# a relative change of every operand entry of the chain) and u the relative
# rounding error per operand of the precision form (unit_roundoff).  With
# independent roundings the error is about u S_j / sqrt(3) (sharing a rounded
# value between mirrored positions raises it by at most sqrt(m!)), so TAU
# leaves a wide margin; a wrong entry shows as |C_j| / (u S_j), several
# hundred in bf16 and far more in FP32.
TAU = 16.0


def unit_roundoff(prec: int, kpad: int) -> float:
    """Relative error per operand of a precision form: bf16 rounding (2^-9)
    where operands or temporaries are bf16; the two-term bf16 split of an
    fp32 operand (2^-17) on the split first level, plus FP32 accumulation
    over the kpad terms of a contraction (2^-24 sqrt(kpad)) where the
    remaining levels are FP32."""
    acc = 2.0 ** -24 * max(1.0, float(kpad)) ** 0.5
    if prec == P32:
        return acc
    if prec == PX3F:
        return 2.0 ** -17 + acc
    return 2.0 ** -9 + acc


def elementwise_excess(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, u: float) -> float:
    """max_j |got_j - ref_j| / (u S_j) over arrays of one shape (BCSS or
    dense); an entry with S_j = 0 must match exactly (else inf)."""
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    S = np.asarray(scale, np.float64)
    zero = S == 0
    if np.any(d[zero] != 0):
        return float("inf")
    if np.all(zero):
        return 0.0
    return float(np.max(d[~zero] / (u * S[~zero])))


def reference(A: np.ndarray, X: np.ndarray, b: int, last_mode: int = 0):
    """(C_ref, S) packed into BCSS with block size b: the oracle chain on the
    given values (FP64) and its per-entry error scale."""
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    if A.ndim == 2:
        from oracle import closed_forms
        C = closed_forms.matrix_case(A64, X64)
        S = oracle.error_scale(A64, X64)
    else:
        C, temps = oracle.chain(A64, X64, keep_temps=True)
        S = oracle.error_scale(A64, X64, temps=temps)
        del temps
    return bcss_ref.pack(np.asfortranarray(C), b), bcss_ref.pack(S, b)


def check_entries(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, prec: int, kpad: int, what: str = ""):
    """Assert the entry-by-entry bound; returns max |err| / (u S)."""
    z = elementwise_excess(got, ref, scale, unit_roundoff(prec, kpad))
    say("  %smax |err|/(u S) = %.3g (bound %g)" % (what + " " if what else "", z, TAU))
    assert z <= TAU, "entry-by-entry bound exceeded: %g > %g" % (z, TAU)
    return z


def sample_tuples(m: int, p: int, count: int = 256, seed=7) -> np.ndarray:
    """`count` random output index tuples (count x m), seeded."""
    return synth.rng(seed).integers(0, p, size=(count, m))


def bcss_positions(js: np.ndarray, b: int, p: int):
    """(block rank, offset) in BCSS for each dense output tuple: the block of
    sort(j // b) in colex order, the local indices permuted the same way."""
    m = js.shape[1]
    index = bcss_ref.block_index(m, -(-p // b))
    ranks, offs = [], []
    for j in js:
        order = sorted(range(m), key=lambda i: (j[i] // b, i))
        blk = tuple(int(j[i] // b) for i in order)
        off = sum(int(j[i] % b) * b ** q for q, i in enumerate(order))
        ranks.append(index[blk])
        offs.append(off)
    return np.array(ranks), np.array(offs)


def check_literal_entries(results: dict, A: np.ndarray, X: np.ndarray, b: int, ref_bcss_: np.ndarray,
                          scale_bcss: np.ndarray, kpad: int, count: int = 256, cache: dict = None):
    """O3 at full size: `count` output entries (seed 7) by the literal
    n^m-term sum of §2.5 (Eq. (cob)); each agrees with the oracle chain's
    entry to FP64 reassociation, and each GPU result in `results`
    ({prec: BCSS array}) satisfies the entry-by-entry bound against it.
    `cache` (a dict) keeps the literal sums for further calls on the same
    A and X."""
    m, p = A.ndim, X.shape[0]
    js = sample_tuples(m, p, count)
    if cache is not None and "o3" in cache:
        lit = cache["o3"]
    else:
        lit, _ = oracle.entries(A.astype(np.float64), X.astype(np.float64), js)
        if cache is not None:
            cache["o3"] = lit
    r, o = bcss_positions(js, b, p)
    S = scale_bcss[r, o]
    assert np.all(np.abs(lit - ref_bcss_[r, o]) <= 1e-10 * S + 1e-300)
    for prec, got in results.items():
        check_entries(got[r, o], lit, S, prec, kpad, what="O3 x%d prec %d" % (count, prec))


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
