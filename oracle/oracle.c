/*
 * FP64 CPU oracle for the sttsm operation  C := [A; X, ..., X].
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library, and is deliberately plain: no blocking, no
 * symmetry, no reordering beyond what the cited definitions state.
 *
 * Conventions (Schatz, Low, van de Geijn, Kolda, "Exploiting Symmetry in
 * Tensors for High Performance: Multiplication with Symmetric Tensors"):
 *   - A dense order-m tensor with mode extents d_0..d_{m-1} is stored in the
 *     paper's "dimensional order" (generalised column-major, App. A): element
 *     (i_0, ..., i_{m-1}) lives at offset  sum_k i_k * prod_{l<k} d_l.
 *   - X is p x n, row-major: chi_{j i} = X[j*n + i].
 *   - All arithmetic is IEEE double, compiled without fast-math.
 *
 * Functions:
 *   oracle_entry       one output entry by the literal n^m-term sum  (O3)
 *   oracle_entries     many entries by that sum, with each entry's
 *                      root-sum-square of terms (its rounding-error scale)
 *   oracle_direct_sum  every output entry by that literal sum        (O1)
 *   oracle_mode_product / oracle_chain  successive dense mode products (O2)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_MAX_ORDER 8

/*
 * O3.  gamma_{j_0..j_{m-1}} = sum over all (i_0..i_{m-1}) in [0,n)^m of
 *      alpha_{i_0..i_{m-1}} * chi_{j_0 i_0} * ... * chi_{j_{m-1} i_{m-1}}.
 * Definition of the operation, §2.5 (element-wise form of the change of
 * basis).  The i multi-index runs as an odometer with i_0 fastest, so the
 * summation order is fixed and the result deterministic.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_entry(int m, int64_t n, int64_t p, const double *A, const double *X,
                 const int64_t *j, double *out)
{
    if (m < 1 || m > ORACLE_MAX_ORDER || n < 1 || p < 1 || !A || !X || !j || !out)
        return -1;
    for (int k = 0; k < m; ++k)
        if (j[k] < 0 || j[k] >= p) return -1;

    int64_t i[ORACLE_MAX_ORDER];
    for (int k = 0; k < m; ++k) i[k] = 0;
    int64_t total = 1;
    for (int k = 0; k < m; ++k) total *= n;

    double gamma = 0.0;
    for (int64_t flat = 0; flat < total; ++flat) {
        /* flat is the dimensional-order offset of (i_0..i_{m-1}) in A */
        double term = A[flat];
        for (int k = 0; k < m; ++k)
            term *= X[j[k] * n + i[k]];
        gamma += term;
        for (int k = 0; k < m; ++k) {       /* odometer, i_0 fastest */
            if (++i[k] < n) break;
            i[k] = 0;
        }
    }
    *out = gamma;
    return 0;
}

/*
 * O3 over a list of entries, with each entry's error scale.  For each of the
 * `count` output tuples j (m indices each, J[e*m + k]) this evaluates, by the
 * same literal n^m-term sum as oracle_entry (§2.5), both
 *   sums[e] = sum_i  t_i,          t_i = alpha_i chi_{j_0 i_0} ... chi_{j_{m-1} i_{m-1}},
 *   rss[e]  = sqrt(sum_i t_i^2),
 * the root-sum-square of the same terms.  rss is the scale of the rounding
 * error of any summation of the terms in which each rounding is independent
 * and relative: it is what an entry-by-entry tolerance is measured against.
 * Entries run in parallel; each one's sums run in the fixed odometer order of
 * oracle_entry (i_0 fastest).  Returns 0, or -1 on bad arguments.
 */
int oracle_entries(int m, int64_t n, int64_t p, const double *A, const double *X,
                   int64_t count, const int64_t *J, double *sums, double *rss)
{
    if (m < 1 || m > ORACLE_MAX_ORDER || n < 1 || p < 1 || count < 0 || !A || !X ||
        (count > 0 && (!J || !sums || !rss)))
        return -1;
    for (int64_t e = 0; e < count; ++e)
        for (int k = 0; k < m; ++k)
            if (J[e * m + k] < 0 || J[e * m + k] >= p) return -1;
    int64_t total = 1;
    for (int k = 0; k < m; ++k) total *= n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < count; ++e) {
        const int64_t *j = J + e * m;
        int64_t i[ORACLE_MAX_ORDER];
        for (int k = 0; k < m; ++k) i[k] = 0;
        double gamma = 0.0, sq = 0.0;
        for (int64_t flat = 0; flat < total; ++flat) {
            double term = A[flat];
            for (int k = 0; k < m; ++k)
                term *= X[j[k] * n + i[k]];
            gamma += term;
            sq += term * term;
            for (int k = 0; k < m; ++k) {
                if (++i[k] < n) break;
                i[k] = 0;
            }
        }
        sums[e] = gamma;
        rss[e] = sqrt(sq);
    }
    return 0;
}

/*
 * O1.  Every entry of C (all p^m of them, no use of symmetry) by the literal
 * sum of oracle_entry.  Cost (m+1) n^m p^m flops, the naive algorithm's count
 * in §5.2.  C is written in dimensional order with extent p in every mode.
 */
int oracle_direct_sum(int m, int64_t n, int64_t p, const double *A, const double *X,
                      double *C)
{
    if (m < 1 || m > ORACLE_MAX_ORDER || n < 1 || p < 1 || !A || !X || !C)
        return -1;
    int64_t total = 1;
    for (int k = 0; k < m; ++k) total *= p;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(|:bad)
    for (int64_t flat = 0; flat < total; ++flat) {
        int64_t j[ORACLE_MAX_ORDER];
        int64_t r = flat;
        for (int k = 0; k < m; ++k) { j[k] = r % p; r /= p; }
        if (oracle_entry(m, n, p, A, X, j, &C[flat]) != 0) bad = 1;
    }
    return bad ? -1 : 0;
}

/*
 * Mode-k tensor times matrix (App. A):  out = T x_k B, with B of size J x d_k
 * (row-major), T of order `order` with extents dims[0..order-1], and
 *   out_{i_0..i_{k-1} j i_{k+1}..} = sum_{i_k} t_{i_0..i_k..} * beta_{j i_k}.
 * out has the extents of T with mode k replaced by J.  Viewing T as
 * (lo, d_k, hi) with lo = prod_{l<k} d_l and hi = prod_{l>k} d_l, which is its
 * dimensional-order layout, the sum over i_k runs from 0 upwards.
 */
int oracle_mode_product(int order, const int64_t *dims, const double *T, int k,
                        const double *B, int64_t J, double *out)
{
    if (order < 1 || order > ORACLE_MAX_ORDER || k < 0 || k >= order || J < 1 ||
        !dims || !T || !B || !out)
        return -1;
    int64_t lo = 1, hi = 1;
    for (int l = 0; l < k; ++l) lo *= dims[l];
    for (int l = k + 1; l < order; ++l) hi *= dims[l];
    const int64_t dk = dims[k];
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t h = 0; h < hi; ++h) {
        for (int64_t j = 0; j < J; ++j) {
            const double *t = T + h * dk * lo;
            const double *b = B + j * dk;
            double *o = out + (h * J + j) * lo;
            for (int64_t l = 0; l < lo; ++l) o[l] = 0.0;
            for (int64_t ik = 0; ik < dk; ++ik) {
                const double beta = b[ik];
                const double *tcol = t + ik * lo;
                for (int64_t l = 0; l < lo; ++l) o[l] += tcol[l] * beta;
            }
        }
    }
    return 0;
}

/*
 * O2.  The same sum regrouped as successive dense mode products, the
 * temporaries algorithm for general m (§5.2, Figure 1 bottom right):
 *   T^(m-1) = A x_{m-1} X,  T^(k) = T^(k+1) x_k X  (k = m-2..1),  C = T^(1) x_0 X.
 * No blocks and no symmetry: every entry of every temporary is formed.
 * T^(k) has extent n in modes 0..k-1 and p in modes k..m-1.
 * If `temps` is non-null, temps[k] (k = 1..m-1) receives a copy of T^(k); each
 * must hold n^k p^(m-k) doubles.  temps[0] is ignored.
 * Returns 0, -1 on bad arguments, -2 when out of memory.
 */
int oracle_chain(int m, int64_t n, int64_t p, const double *A, const double *X,
                 double *C, double **temps)
{
    if (m < 1 || m > ORACLE_MAX_ORDER || n < 1 || p < 1 || !A || !X || !C)
        return -1;
    int64_t dims[ORACLE_MAX_ORDER];
    for (int k = 0; k < m; ++k) dims[k] = n;

    const double *cur = A;
    double *owned = NULL;
    for (int k = m - 1; k >= 0; --k) {
        int64_t out_elems = 1;
        for (int l = 0; l < m; ++l) out_elems *= (l == k ? p : dims[l]);
        double *next = (k == 0) ? C : (double *)malloc(sizeof(double) * (size_t)out_elems);
        if (!next) { free(owned); return -2; }
        int rc = oracle_mode_product(m, dims, cur, k, X, p, next);
        if (rc != 0) { if (k) free(next); free(owned); return rc; }
        dims[k] = p;
        if (k > 0 && temps && temps[k])
            memcpy(temps[k], next, sizeof(double) * (size_t)out_elems);
        free(owned);
        owned = (k == 0) ? NULL : next;
        cur = next;
    }
    return 0;
}

/* Sets the number of OpenMP threads of the following calls (n >= 1); a
 * no-op when built without OpenMP. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads the oracle runs on (1 when built without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
