"""Pins for the FP64 oracle: each check compares it against something other
than itself (a library routine, a closed form, an invariant, a special case
that reduces to a textbook identity, or the paper's printed numbers)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms
import synth

TOL = 1e-13


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm((a - b).ravel())
    s = np.linalg.norm(b.ravel())
    return d / s if s > 0 else d


def sym(m, n, seed):
    return synth.symmetric_uniform(m, n, seed).astype(np.float64)


def nonsym(shape, seed):
    return np.asfortranarray(synth.rng(seed).standard_normal(shape))


# ---------------------------------------------------------------- O1 vs O2
BRUTE = [(m, n, p) for m in range(1, 7) for n in (1, 2, 3, 5) for p in (1, 2, 3, 5)
         if n ** m * p ** m <= 4_000_000]


@pytest.mark.parametrize("m,n,p", BRUTE)
def test_direct_sum_equals_chain(m, n, p):
    """The literal sum of §2.5 and the regrouped dense chain of §5.2 agree to
    FP64 reassociation, on symmetric and on non-symmetric A."""
    X = synth.change_of_basis(p, n, seed=(m, n, p, 1)).astype(np.float64)
    for A in (sym(m, n, (m, n, p, 0)), nonsym((n,) * m, (m, n, p, 2))):
        assert rel(oracle.direct_sum(A, X), oracle.chain(A, X)) <= TOL


def test_direct_sum_config1():
    """O1 run in full at m=3, n=p=16 agrees with O2."""
    A, X = synth.make_config_inputs("m3_n16_b4")
    assert rel(oracle.direct_sum(A, X), oracle.chain(A, X)) <= TOL


def test_entry_matches_chain_at_full_size():
    """O3 literal per-entry sums agree with O2 at m=3, n=p=64 (sampled)."""
    A = sym(3, 64, 5)
    X = synth.change_of_basis(48, 64, 6).astype(np.float64)
    C = oracle.chain(A, X)
    g = synth.rng(7)
    for _ in range(64):
        j = g.integers(0, 48, size=3)
        assert abs(oracle.entry(A, X, j) - C[tuple(j)]) <= 1e-12 * np.abs(C).max()


def _python_terms(A, X, j):
    """Every term alpha_i chi_{j_0 i_0} ... chi_{j_{m-1} i_{m-1}} of one
    output entry (§2.5), by plain Python loops over itertools.product."""
    m, n = A.ndim, A.shape[0]
    out = []
    for i in itertools.product(range(n), repeat=m):
        t = float(A[i])
        for k in range(m):
            t *= float(X[j[k], i[k]])
        out.append(t)
    return out


@pytest.mark.parametrize("m,n,p", [(1, 3, 2), (2, 3, 4), (3, 3, 2), (3, 2, 3), (4, 2, 2)])
def test_direct_sum_matches_python_loops(m, n, p):
    """O1 against a brute-force Python evaluation of the defining sum, on a
    non-symmetric A (so a swapped index would show)."""
    A = nonsym((n,) * m, (m, n, p, 41))
    X = synth.rng((m, n, p, 42)).standard_normal((p, n))
    C = oracle.direct_sum(A, X)
    for j in itertools.product(range(p), repeat=m):
        assert abs(C[j] - math.fsum(_python_terms(A, X, j))) <= 1e-13 * max(1.0, abs(C[j]))


def test_entries_match_direct_sum_config1():
    """O3 (per-entry literal sums, in parallel) against O1 on every one of
    the 4096 entries of m=3, n=p=16."""
    A, X = synth.make_config_inputs("m3_n16_b4")
    A, X = A.astype(np.float64), X.astype(np.float64)
    C = oracle.direct_sum(A, X)
    js = np.array(list(itertools.product(range(16), repeat=3)))
    sums, _ = oracle.entries(A, X, js)
    assert np.array_equal(sums, C[tuple(js.T)])


@pytest.mark.parametrize("m,n,p", [(1, 4, 3), (2, 3, 4), (3, 3, 2), (4, 2, 3)])
def test_term_rss_matches_python_loops(m, n, p):
    """The rounding-error scale sqrt(sum_i t_i^2) of every entry, from the
    chain on squares and from the literal per-entry loop, against Python."""
    A = nonsym((n,) * m, (m, n, p, 43))
    X = synth.rng((m, n, p, 44)).standard_normal((p, n))
    R = oracle.term_rss(A, X)
    js = np.array(list(itertools.product(range(p), repeat=m)))
    _, rss = oracle.entries(A, X, js)
    for e, j in enumerate(js):
        want = math.sqrt(math.fsum(t * t for t in _python_terms(A, X, tuple(j))))
        assert abs(R[tuple(j)] - want) <= 1e-13 * want
        assert abs(rss[e] - want) <= 1e-13 * want


@pytest.mark.parametrize("m,n,p", [(2, 7, 5), (3, 6, 4), (4, 5, 3)])
def test_term_rss_rank1_closed_form(m, n, p):
    """A = a o ... o a: the terms of entry j factor over the modes, so
    sum_i t_i^2 = prod_k (X^2 a^2)_{j_k}, i.e. rss = (|X|^2 a^2)^{1/2} taken
    as an outer power."""
    a = synth.rng((m, n, 45)).standard_normal(n)
    A = closed_forms.outer_power(a, m)
    X = synth.change_of_basis(p, n, (m, 46)).astype(np.float64)
    want = closed_forms.outer_power(np.sqrt((X * X) @ (a * a)), m)
    assert rel(oracle.term_rss(A, X), want) <= 1e-13


@pytest.mark.parametrize("m,n,p", [(2, 9, 6), (3, 7, 5), (4, 5, 4)])
def test_term_rss_bounds(m, n, p):
    """Cauchy-Schwarz over the n^m terms: |C_j| <= sqrt(n^m) rss_j, and
    rss_j <= sum_i |t_i| = [|A|; |X|, ..., |X|]_j."""
    A = sym(m, n, (m, 47))
    X = synth.change_of_basis(p, n, (m, 48)).astype(np.float64)
    R = oracle.term_rss(A, X)
    assert np.all(np.abs(oracle.chain(A, X)) <= np.sqrt(float(n) ** m) * R * (1 + 1e-13))
    assert np.all(R <= oracle.chain(np.abs(A), np.abs(X)) * (1 + 1e-13))


# ------------------------------------------------------- textbook identities
@pytest.mark.parametrize("n,p", [(1, 1), (4, 3), (17, 9), (40, 40)])
def test_matrix_case_is_XAXt(n, p):
    """m=2: [A; X, X] = X A X^T (§3.1), by a library matrix product."""
    A = sym(2, n, 11)
    X = synth.change_of_basis(p, n, 12).astype(np.float64)
    assert rel(oracle.chain(A, X), closed_forms.matrix_case(A, X)) <= TOL
    assert rel(oracle.direct_sum(A, X), closed_forms.matrix_case(A, X)) <= TOL


@pytest.mark.parametrize("m,n,p,r", [(2, 7, 5, 1), (3, 9, 4, 1), (4, 8, 6, 3), (5, 5, 7, 2), (6, 4, 3, 8)])
def test_rank_r_closed_form(m, n, p, r):
    """sum lam_i a_i^{o m}  maps to  sum lam_i (X a_i)^{o m}."""
    lams, vecs = synth.rank_r_factors(n, r, (m, n, r))
    A = synth.rank_r_symmetric(m, lams, vecs)
    X = synth.change_of_basis(p, n, (m, p)).astype(np.float64)
    assert rel(oracle.chain(A, X), closed_forms.rank_r(lams, vecs, X, m)) <= 1e-12


@pytest.mark.parametrize("m,n", [(2, 6), (3, 5), (4, 4), (5, 3)])
def test_identity_and_permutation_matrix(m, n):
    """X = I returns A; X = a permutation matrix P returns A with every index
    relabelled, C[j] = A[pi(j_0), ..., pi(j_{m-1})]."""
    A = nonsym((n,) * m, (m, n))
    assert rel(oracle.chain(A, np.eye(n)), A) == 0.0
    pi = synth.rng(m * 10 + n).permutation(n)
    P = np.eye(n)[pi]                       # row j picks column pi[j]
    expect = A[np.ix_(*([pi] * m))]
    assert rel(oracle.chain(A, P), expect) == 0.0
    assert rel(oracle.direct_sum(A, P), expect) == 0.0


@pytest.mark.parametrize("m,n", [(2, 5), (3, 4), (4, 3)])
def test_diagonal_scaling(m, n):
    """X = diag(d): gamma_j = alpha_j * d_{j_0} ... d_{j_{m-1}}."""
    A = nonsym((n,) * m, (m, n, 3))
    d = synth.rng(m + n).uniform(0.5, 2.0, size=n)
    scale = d
    for _ in range(m - 1):
        scale = np.multiply.outer(scale, d)
    assert rel(oracle.chain(A, np.diag(d)), A * scale) <= TOL


@pytest.mark.parametrize("m,n,p,q", [(2, 6, 5, 4), (3, 5, 4, 6), (4, 4, 3, 5)])
def test_composition(m, n, p, q):
    """[[A; X..X]; Y..Y] = [A; YX..YX] (multilinearity of the mode products)."""
    A = sym(m, n, (m, 1))
    X = synth.change_of_basis(p, n, (m, 2)).astype(np.float64)
    Y = synth.change_of_basis(q, p, (m, 3)).astype(np.float64)
    assert rel(oracle.chain(oracle.chain(A, X), Y), oracle.chain(A, Y @ X)) <= 1e-12


def test_linearity_in_A():
    A1, A2 = sym(3, 7, 1), sym(3, 7, 2)
    X = synth.change_of_basis(5, 7, 3).astype(np.float64)
    assert rel(oracle.chain(A1 + 2.5 * A2, X), oracle.chain(A1, X) + 2.5 * oracle.chain(A2, X)) <= TOL


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("m,n,p", [(2, 9, 7), (3, 8, 6), (4, 6, 5), (5, 4, 4), (6, 3, 4)])
def test_output_symmetric(m, n, p):
    """C is symmetric whenever A is (§2.5): every permuted view agrees."""
    A = sym(m, n, (m, n))
    X = synth.change_of_basis(p, n, (m, p)).astype(np.float64)
    C = oracle.chain(A, X)
    scale = np.abs(C).max()
    for perm in itertools.permutations(range(m)):
        assert np.abs(C - np.transpose(C, perm)).max() <= TOL * scale


@pytest.mark.parametrize("m,n,p", [(3, 7, 5), (4, 5, 6), (5, 4, 3)])
def test_theorem1_partial_symmetry(m, n, p):
    """Theorem 1 (§6.1): T^(k) is symmetric in modes 0..k-1."""
    A = sym(m, n, (m, n, 9))
    X = synth.change_of_basis(p, n, (m, 8)).astype(np.float64)
    _, temps = oracle.chain(A, X, keep_temps=True)
    for k, T in temps.items():
        scale = np.abs(T).max()
        for perm in itertools.permutations(range(k)):
            full = tuple(perm) + tuple(range(k, m))
            assert np.abs(T - np.transpose(T, full)).max() <= TOL * scale
        if k < m - 1 and n == p:
            # modes k..m-1 are in general NOT symmetric with mode k-1
            pass


def test_temporaries_are_the_mode_products():
    """T^(k) kept by the chain equal the mode products formed one at a time
    with numpy.tensordot (a library contraction)."""
    m, n, p = 4, 5, 3
    A = sym(m, n, 4)
    X = synth.change_of_basis(p, n, 5).astype(np.float64)
    C, temps = oracle.chain(A, X, keep_temps=True)
    cur = A
    for k in range(m - 1, -1, -1):
        cur = np.moveaxis(np.tensordot(cur, X, axes=([k], [1])), -1, k)
        ref = temps[k] if k > 0 else C
        assert rel(ref, cur) <= TOL


# ------------------------------------------------- planted mistakes are caught
def test_pins_catch_a_transposed_operand():
    """A plausible mistake, multiplying by X^T instead of X in one mode, fails
    the m=2 matrix identity and the symmetry invariant."""
    n = 6
    A = sym(2, n, 1)
    X = synth.change_of_basis(n, n, 2).astype(np.float64)
    T = oracle.mode_product(A, 1, X)
    wrong = oracle.mode_product(T, 0, X.T.copy())
    assert rel(wrong, closed_forms.matrix_case(A, X)) > 1e-3
    assert np.abs(wrong - wrong.T).max() > 1e-3


def test_pins_catch_a_dropped_term():
    """Dropping the last term of each mode sum (a classic loop bound slip) is
    caught by the rank-1 closed form."""
    m, n, p = 3, 6, 4
    lams, vecs = synth.rank_r_factors(n, 1, 3)
    A = synth.rank_r_symmetric(m, lams, vecs)
    X = synth.change_of_basis(p, n, 4).astype(np.float64)
    Xbad = X.copy()
    Xbad[:, -1] = 0.0
    assert rel(oracle.chain(A, Xbad), closed_forms.rank_r(lams, vecs, X, m)) > 1e-3


# ---------------------------------------------------------------- all modes but one
@pytest.mark.parametrize("n,p", [(5, 3), (7, 7), (4, 6)])
def test_all_but_one_matrix_case(n, p):
    """m = 2: A x_1 X is A X^T (library matrix product)."""
    A = sym(2, n, 61)
    X = synth.change_of_basis(p, n, 62).astype(np.float64)
    assert rel(oracle.all_but_one(A, X), A @ X.T) <= TOL


@pytest.mark.parametrize("m,n,p,r", [(3, 6, 4, 2), (4, 5, 3, 3), (5, 4, 4, 1)])
def test_all_but_one_rank_r(m, n, p, r):
    """Rank-r A: sum_i lam_i a_i o (X a_i)^{o (m-1)}."""
    lams, vecs = synth.rank_r_factors(n, r, (m, n, 63))
    A = synth.rank_r_symmetric(m, lams, vecs)
    X = synth.change_of_basis(p, n, (m, 64)).astype(np.float64)
    assert rel(oracle.all_but_one(A, X), closed_forms.rank_r_all_but_one(lams, vecs, X, m)) <= 1e-12


@pytest.mark.parametrize("m,n,p", [(3, 5, 4), (4, 4, 3)])
def test_all_but_one_symmetry_and_last_mode(m, n, p):
    """Symmetric in modes 1..m-1; multiplying its mode 0 by X gives sttsm's C."""
    A = sym(m, n, (m, 65))
    X = synth.change_of_basis(p, n, (m, 66)).astype(np.float64)
    T = oracle.all_but_one(A, X)
    for perm in itertools.permutations(range(1, m)):
        assert rel(np.transpose(T, (0,) + perm), T) <= TOL
    assert rel(oracle.mode_product(T, 0, X), oracle.direct_sum(A, X)) <= 1e-12


# ---------------------------------------------------------------- vector case
def test_vectors_matrix_case():
    """m = 2: y = A x and s = x^T A x (library matrix products)."""
    A = sym(2, 7, 67)
    X = synth.rng(68).standard_normal((4, 7))
    Y, s = oracle.vectors(A, X)
    assert rel(Y, X @ A) <= TOL
    assert rel(s, np.einsum("vi,ij,vj->v", X, A, X)) <= TOL


@pytest.mark.parametrize("m,n,r", [(3, 6, 2), (4, 5, 3), (5, 4, 1)])
def test_vectors_rank_r(m, n, r):
    """Rank-r A: y = sum lam (a.x)^(m-1) a, s = sum lam (a.x)^m; and s = x . y."""
    lams, vecs = synth.rank_r_factors(n, r, (m, n, 69))
    A = synth.rank_r_symmetric(m, lams, vecs)
    X = synth.rng((m, 70)).standard_normal((3, n))
    Y, s = oracle.vectors(A, X)
    Yc, sc = closed_forms.rank_r_vectors(lams, vecs, X, m)
    assert rel(Y, Yc) <= 1e-12 and rel(s, sc) <= 1e-12
    assert rel(s, np.sum(X * Y, axis=1)) <= 1e-12


# ---------------------------------------------------------------- rank-update form (§8, second variant)
@pytest.mark.parametrize("n,p,b,rows", [(5, 3, 2, 1), (7, 7, 3, 2), (8, 6, 8, 1), (9, 4, 2, 3), (4, 6, 1, 1)])
def test_rank_update_matrix_case(n, p, b, rows):
    """m = 2: the sum of the rank-b updates X_i (A_i X^T) over the block
    rows is X A X^T (library matrix products), for any pass size,
    including a ragged last block."""
    A = sym(2, n, 81)
    X = synth.change_of_basis(p, n, 82).astype(np.float64)
    assert rel(oracle.rank_update(A, X, b, rows), closed_forms.matrix_case(A, X)) <= TOL


@pytest.mark.parametrize("m,n,p,b,rows", [(3, 4, 3, 2, 1), (3, 5, 5, 2, 2), (4, 3, 2, 1, 2), (4, 4, 3, 3, 1)])
def test_rank_update_equals_direct_sum(m, n, p, b, rows):
    """Order m: the rank-update form equals the literal sum of §2.5."""
    A = sym(m, n, 83)
    X = synth.change_of_basis(p, n, 84).astype(np.float64)
    assert rel(oracle.rank_update(A, X, b, rows), oracle.direct_sum(A, X)) <= TOL


@pytest.mark.parametrize("m,n,p,r", [(3, 6, 4, 2), (4, 5, 3, 3)])
def test_rank_update_rank_r(m, n, p, r):
    """Rank-r A: the rank-update form equals sum_i lam_i (X a_i)^{o m}."""
    lams, vecs = synth.rank_r_factors(n, r, 85)
    A = synth.rank_r_symmetric(m, lams, vecs)
    X = synth.change_of_basis(p, n, 86).astype(np.float64)
    assert rel(oracle.rank_update(A, X, 2, 1), closed_forms.rank_r(lams, vecs, X, m)) <= 1e-12


def test_rank_update_misses_a_row_block_fails_the_pin():
    """A form that skipped the last block row (a plausible pass-boundary
    mistake) fails the matrix-case pin."""
    n, p, b = 7, 5, 3
    A = sym(2, n, 87)
    X = synth.change_of_basis(p, n, 88).astype(np.float64)
    Y = oracle.all_but_one(A, X)
    C = np.zeros((p, p))
    for i0 in range(0, n - n % b, b):   # drops the ragged tail block
        C += X[:, i0:i0 + b] @ Y[i0:i0 + b]
    assert rel(C, closed_forms.matrix_case(A, X)) > 1e-3
