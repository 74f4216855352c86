"""Pins for the oracle's per-entry rounding-error scale (oracle.error_scale)
and for the entry-by-entry parity bound built on it.

The scale S_j is the 2-norm of the first-order sensitivities of output entry
j to a relative change of every operand entry of the chain (A, every
temporary T^(k), X in every mode).  It is pinned against (1) those
sensitivities written out with Python loops on tiny inputs, (2) library
matrix products at m = 2, and (3) a Monte Carlo run that perturbs every
operand entry independently and measures the spread of each output entry.
The bound is then shown, on the CPU, to pass a reduced-precision chain and
to catch one wrong output row that the relative Frobenius check passes."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import bcss_ref
import synth
from gpu_util import PBF, TAU, elementwise_excess, tol_bf16, unit_roundoff


def _sym(m, n, seed):
    return synth.symmetric_uniform(m, n, seed).astype(np.float64)


def _brute_scale(A, X, s):
    """S^2 for every output entry, by plain loops over the operand entries:
    the chain out[i_<s, j_>=s] = sum_{i_>=s} a_i prod_{l>=s} x_{j_l i_l};
    temporaries T^(k)[i_<k, j_>=k] = sum_{i_>=k} a_i prod_{l>=k} x_{j_l i_l}
    for k = s+1..m-1."""
    m, n, p = A.ndim, A.shape[0], X.shape[0]
    out_shape = (n,) * s + (p,) * (m - s)
    S2 = np.zeros(out_shape)

    def T(k, ilow, jhigh):
        tot = 0.0
        for ih in itertools.product(range(n), repeat=m - k):
            t = A[tuple(ilow) + ih]
            for l in range(k, m):
                t *= X[jhigh[l - k], ih[l - k]]
            tot += t
        return tot

    for o in itertools.product(*[range(d) for d in out_shape]):
        ilo, jhi = o[:s], o[s:]
        acc = []
        # A entries
        for ih in itertools.product(range(n), repeat=m - s):
            t = A[tuple(ilo) + ih]
            for l in range(s, m):
                t *= X[jhi[l - s], ih[l - s]]
            acc.append(t * t)
        # temporaries T^(k), k = s+1..m-1: entry (ilo, i_s..i_{k-1}, j_k..)
        for k in range(s + 1, m):
            for imid in itertools.product(range(n), repeat=k - s):
                t = T(k, tuple(ilo) + imid, jhi[k - s:])
                for l in range(s, k):
                    t *= X[jhi[l - s], imid[l - s]]
                acc.append(t * t)
        # X entries of mode l: chi_{j_l, i} times the sum of the terms with i_l = i, divided by chi
        for l in range(s, m):
            for i in range(n):
                d = 0.0
                for ih in itertools.product(range(n), repeat=m - s):
                    if ih[l - s] != i:
                        continue
                    t = A[tuple(ilo) + ih]
                    for q in range(s, m):
                        t *= X[jhi[q - s], ih[q - s]]
                    d += t
                acc.append(d * d)
        S2[o] = math.fsum(acc)
    return np.sqrt(S2)


@pytest.mark.parametrize("m,n,p,s", [(1, 4, 3, 0), (2, 3, 4, 0), (3, 3, 2, 0), (3, 3, 2, 1), (4, 2, 3, 0),
                                     (4, 2, 2, 1), (3, 2, 3, 2)])
def test_error_scale_matches_python_loops(m, n, p, s):
    A = _sym(m, n, (m, n, p, 51))
    X = synth.rng((m, n, p, 52)).standard_normal((p, n))
    got = oracle.error_scale(A, X, last_mode=s)
    want = _brute_scale(A, X, s)
    assert got.shape == want.shape
    assert np.all(np.abs(got - want) <= 1e-13 * want)


@pytest.mark.parametrize("n,p", [(5, 3), (17, 9), (40, 33)])
def test_error_scale_matrix_case_matches_general_form(n, p):
    """m = 2 by library matrix products (the path error_scale takes) equals
    the general form written out with the oracle's mode products: the A
    part, the T^(1) part and the X parts of modes 0 and 1."""
    A = _sym(2, n, (n, p, 53))
    X = synth.change_of_basis(p, n, (n, p, 54)).astype(np.float64)
    fast = oracle.error_scale(A, X)
    _, temps = oracle.chain(A, X, keep_temps=True)
    X2 = X * X
    V = oracle.mode_product(oracle.mode_product(A * A, 1, X2), 0, X2)
    Q = oracle.mode_product(temps[1] * temps[1], 0, X2)
    slow = np.sqrt(V + Q + Q + np.moveaxis(Q, 0, 1))
    assert np.all(np.abs(fast - slow) <= 1e-12 * slow)


@pytest.mark.parametrize("m,n,p,s", [(3, 6, 5, 0), (4, 4, 4, 0), (3, 5, 4, 1)])
def test_error_scale_predicts_perturbation_spread(m, n, p, s):
    """Monte Carlo: perturb every entry of A, of every temporary and of X
    (independently in each mode) by a relative delta ~ U[-u, u]; the
    variance of each output entry over the trials is (u^2/3) S_j^2 to first
    order.  Mode products here are numpy tensordot, not the oracle's."""
    A = _sym(m, n, (m, n, p, 55))
    X = synth.change_of_basis(p, n, (m, n, p, 56)).astype(np.float64)
    u = 1e-7
    g = synth.rng((m, n, p, 57))

    def mp(T, k, B):
        return np.moveaxis(np.tensordot(B, T, axes=([1], [k])), 0, k)

    def run(perturb):
        f = (lambda a: a * (1 + g.uniform(-u, u, a.shape))) if perturb else (lambda a: a)
        T = f(A)
        for k in range(m - 1, s - 1, -1):
            T = mp(T, k, f(X))
            if k > s:
                T = f(T)
        return T

    base = run(False)
    trials = 600
    acc = np.zeros_like(base)
    for _ in range(trials):
        d = run(True) - base
        acc += d * d
    emp = acc / trials
    pred = (u * u / 3.0) * oracle.error_scale(A, X, last_mode=s) ** 2
    ratio = emp.sum() / pred.sum()
    assert 0.9 < ratio < 1.1
    per = emp / pred
    assert np.all((per > 0.6) & (per < 1.5))


def _emulated_bf16_chain(A, X):
    """The BF16 form's rounding points on the CPU: A and X already hold
    bf16 values, each temporary is rounded to bf16 (RNE) after its FP64
    mode product, the result stays FP64."""
    m = A.ndim
    T = A
    for k in range(m - 1, -1, -1):
        T = oracle.mode_product(T, k, X)
        if k > 0:
            T = synth.round_to_bf16(T.astype(np.float32)).astype(np.float64)
    return T


def test_elementwise_bound_passes_bf16_chain_and_catches_a_wrong_row():
    """m = 3, n = p = 128, b = 16 in the BF16 form (emulated on the CPU): the
    entry-by-entry bound holds for every entry; then one row of one stored
    block of C (b entries along mode 0) is scaled by 1.25, which
    the relative Frobenius check still passes and the entry-by-entry check
    does not."""
    m, n, b = 3, 128, 16
    A = synth.round_to_bf16(synth.symmetric_uniform(m, n, 61)).astype(np.float64)
    X = synth.round_to_bf16(synth.change_of_basis(n, n, 62)).astype(np.float64)
    ref, temps = oracle.chain(A, X, keep_temps=True)
    S = oracle.error_scale(A, X, temps=temps)
    got = bcss_ref.pack(_emulated_bf16_chain(A, X), b)
    refb, Sb = bcss_ref.pack(ref, b), bcss_ref.pack(S, b)
    u = unit_roundoff(PBF, n)
    e0 = bcss_ref.rel_frobenius_bcss(got, refb, m, n, b)
    z0 = elementwise_excess(got, refb, Sb, u)
    print("emulated bf16: rel frobenius", e0, "max |err|/(u S)", z0)
    assert e0 <= tol_bf16(m) and z0 <= TAU
    bad = got.copy()
    r = len(bad) // 2
    bad[r, :b] *= 1.25
    e1 = bcss_ref.rel_frobenius_bcss(bad, refb, m, n, b)
    z1 = elementwise_excess(bad, refb, Sb, u)
    print("planted row: rel frobenius", e1, "max |err|/(u S)", z1)
    assert e1 <= tol_bf16(m)
    assert z1 > TAU
