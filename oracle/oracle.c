/*
 * oracle.c -- plain, slow, serial FP64 reference for the rank-k Cholesky
 * modification of Walder, "Rank k Cholesky Up/Down-dating on the GPU:
 * gpucholmodV0.2" (2010).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
 * and its Python binding) may link, load or call this file.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no contraction into FMA, IEEE round-to-nearest, correctly rounded / and
 * sqrt), so every operation below is exactly the written IEEE operation.
 *
 * Problem (Section 1): L is upper triangular with A = L^T L, V is n x k,
 * sigma = +1 (update) or -1 (downdate).  Produce the upper-triangular L~
 * with L~^T L~ = A + sigma V V^T, in O(k n^2) operations.
 *
 * Storage (the paper fixes none): L is row-major with leading dimension
 * ldl >= n, element (i, j), j >= i, at L[i*ldl + j]; only the upper
 * triangle is read or written.  V is row-major n x k, (j, m) at V[j*k + m],
 * and is never modified: the algorithm runs on a private copy W.
 *
 * Status: 0 ok, -1 bad argument, -2 not positive definite, -3 bad input
 * diagonal.  On -2/-3, *info = r*k + m of the first (row r, column m), in
 * row-then-column order, whose Compute step failed; the factor is left
 * partially modified (rows < r final).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ARG (-1)
#define ORC_NOT_PD (-2)
#define ORC_BAD_DIAG (-3)

static int check_args(const double *L, const double *V, int64_t n, int64_t k,
                      int64_t ldl, int sigma) {
    if (n < 0 || k < 0) return ORC_ARG;
    if (ldl < (n > 1 ? n : 1)) return ORC_ARG;
    if (sigma != 1 && sigma != -1) return ORC_ARG;
    if (n > 0 && L == NULL) return ORC_ARG;
    if (n > 0 && k > 0 && V == NULL) return ORC_ARG;
    return ORC_OK;
}

/*
 * The rotation of row i against one column of the work copy of V (the
 * "Compute" step of Algorithm 1).  Adding sigma v v^T to a factor whose
 * leading entry is l changes that entry to w, the positive root of
 * w^2 = l^2 + sigma v^2; the pair (c, s) = (w, v) / l is the rotation that
 * Apply then carries along the row.  c and s are both taken relative to
 * the diagonal as it was BEFORE this column, and the diagonal is replaced
 * by w last.  Returns a status.
 * Failure readings (the paper is silent): an input diagonal that is not
 * > 0 is a bad factor (-3); a radicand that is not > 0 (negative, zero or
 * NaN) means A + sigma V V^T is not positive definite (-2).
 */
static int compute_rot(double *Lii, double v, double sg, double *c, double *s) {
    const double l = *Lii;
    if (!(l > 0.0)) return ORC_BAD_DIAG;
    const double t = l * l + sg * (v * v);
    if (!(t > 0.0)) return ORC_NOT_PD;
    const double w = sqrt(t);
    *c = w / l;
    *s = v / l;
    *Lii = w;
    return ORC_OK;
}

/*
 * One rotation applied to an off-diagonal pair (L_ij, V_j) (the "Apply"
 * step of Algorithm 1): the row entry becomes its sum with sigma s V_j,
 * divided by c; the V entry becomes c V_j minus s times the row entry just
 * computed -- the updated row entry, not the old one, which is what keeps
 * the hyperbolic rotation stable for downdates.
 */
static void apply_rot(double c, double s, double sg, double *Lij, double *Vj) {
    const double lij = (*Lij + sg * (s * *Vj)) / c;
    *Lij = lij;
    *Vj = c * *Vj - s * lij;
}

/*
 * Rank-k CholeskyModifyB (Algorithm 1, second alternative, generalised to k
 * columns by running the k Compute steps of row i, in ascending column
 * order, before the Apply loop over j > i; Section 4 processes the update
 * vectors in a loop of this kind).
 *
 * W_out (optional, n*k) receives the private copy of V as left by the
 * algorithm: row j holds V_j after the rotations of rows 0..j-1.
 */
int oracle_modify(double *L, const double *V, int64_t n, int64_t k,
                  int64_t ldl, int sigma, double *W_out, int64_t *info) {
    int st = check_args(L, V, n, k, ldl, sigma);
    if (info) *info = -1;
    if (st) return st;
    if (n == 0 || k == 0) {
        if (W_out && n * k > 0) memcpy(W_out, V, sizeof(double) * n * k);
        return ORC_OK;
    }
    double *W = (double *)malloc(sizeof(double) * (size_t)(n * k));
    double *c = (double *)malloc(sizeof(double) * (size_t)k);
    double *s = (double *)malloc(sizeof(double) * (size_t)k);
    if (!W || !c || !s) { free(W); free(c); free(s); return ORC_ARG; }
    memcpy(W, V, sizeof(double) * (size_t)(n * k));
    const double sg = (double)sigma;
    st = ORC_OK;
    for (int64_t i = 0; i < n && st == ORC_OK; ++i) {
        double *Li = L + i * ldl;
        for (int64_t m = 0; m < k; ++m) {
            st = compute_rot(&Li[i], W[i * k + m], sg, &c[m], &s[m]);
            if (st) { if (info) *info = i * k + m; break; }
        }
        if (st) break;
        for (int64_t j = i + 1; j < n; ++j)
            for (int64_t m = 0; m < k; ++m)
                apply_rot(c[m], s[m], sg, &Li[j], &W[j * k + m]);
    }
    if (W_out) memcpy(W_out, W, sizeof(double) * (size_t)(n * k));
    free(W); free(c); free(s);
    return st;
}

/*
 * k literal rank-1 CholeskyModifyB passes, column m = 0..k-1 in turn
 * (Algorithm 1 with k = 1, applied once per column of V).
 */
int oracle_modify_seq(double *L, const double *V, int64_t n, int64_t k,
                      int64_t ldl, int sigma, double *W_out, int64_t *info) {
    int st = check_args(L, V, n, k, ldl, sigma);
    if (info) *info = -1;
    if (st) return st;
    if (n == 0 || k == 0) {
        if (W_out && n * k > 0) memcpy(W_out, V, sizeof(double) * n * k);
        return ORC_OK;
    }
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w) return ORC_ARG;
    const double sg = (double)sigma;
    st = ORC_OK;
    for (int64_t m = 0; m < k && st == ORC_OK; ++m) {
        for (int64_t j = 0; j < n; ++j) w[j] = V[j * k + m];
        for (int64_t i = 0; i < n; ++i) {
            double *Li = L + i * ldl;
            double c, s;
            st = compute_rot(&Li[i], w[i], sg, &c, &s);
            if (st) { if (info) *info = i * k + m; break; }
            for (int64_t j = i + 1; j < n; ++j) apply_rot(c, s, sg, &Li[j], &w[j]);
        }
        if (W_out) for (int64_t j = 0; j < n; ++j) W_out[j * k + m] = w[j];
    }
    free(w);
    return st;
}

/*
 * CholeskyModifyA (Algorithm 1, first alternative), rank 1, with the order
 * of its two steps corrected: column i first receives the rotations of all
 * rows j < i (Apply(c_j, s_j, L_ji, V_i)), and only then is row i's Compute
 * run.  As printed, Compute(i) precedes the j < i loop, which would use a
 * V_i that has not yet seen the earlier rotations; that order does not
 * produce the factor of A + sigma V V^T.  Run once per column of V.
 */
int oracle_modify_colA(double *L, const double *V, int64_t n, int64_t k,
                       int64_t ldl, int sigma, int64_t *info) {
    int st = check_args(L, V, n, k, ldl, sigma);
    if (info) *info = -1;
    if (st) return st;
    if (n == 0 || k == 0) return ORC_OK;
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    if (!c || !s) { free(c); free(s); return ORC_ARG; }
    const double sg = (double)sigma;
    st = ORC_OK;
    for (int64_t m = 0; m < k && st == ORC_OK; ++m) {
        for (int64_t i = 0; i < n; ++i) {
            double vi = V[i * k + m];
            for (int64_t j = 0; j < i; ++j)
                apply_rot(c[j], s[j], sg, &L[j * ldl + i], &vi);
            st = compute_rot(&L[i * ldl + i], vi, sg, &c[i], &s[i]);
            if (st) { if (info) *info = i * k + m; break; }
        }
    }
    free(c); free(s);
    return st;
}

/*
 * Textbook upper Cholesky, A = U^T U (A symmetric, row-major, lda >= n;
 * only the upper triangle of A is read).  For building test factors and
 * for checking the definition of the result on small matrices.
 *   U_ii = sqrt(A_ii - sum_{p<i} U_pi^2)
 *   U_ij = (A_ij - sum_{p<i} U_pi U_pj) / U_ii,   j > i
 * Returns 0, or -2 if a pivot is not > 0 (*info = its row).  The strictly
 * lower part of U is set to zero.
 */
int oracle_cholesky_upper(const double *A, int64_t lda, double *U, int64_t ldu,
                          int64_t n, int64_t *info) {
    if (info) *info = -1;
    if (n < 0 || lda < (n > 1 ? n : 1) || ldu < (n > 1 ? n : 1)) return ORC_ARG;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < i; ++j) U[i * ldu + j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = A[i * lda + i];
        for (int64_t p = 0; p < i; ++p) d -= U[p * ldu + i] * U[p * ldu + i];
        if (!(d > 0.0)) { if (info) *info = i; return ORC_NOT_PD; }
        const double uii = sqrt(d);
        U[i * ldu + i] = uii;
        for (int64_t j = i + 1; j < n; ++j) {
            double a = A[i * lda + j];
            for (int64_t p = 0; p < i; ++p) a -= U[p * ldu + i] * U[p * ldu + j];
            U[i * ldu + j] = a / uii;
        }
    }
    return ORC_OK;
}

/*
 * A~ = L^T L + sigma V V^T (the matrix whose factor the method produces,
 * Section 1), formed densely, row-major n x n.  O(n^3); small n only.
 */
int oracle_target_matrix(const double *L, int64_t ldl, const double *V,
                         int64_t n, int64_t k, int sigma, double *At) {
    if (n < 0 || k < 0 || ldl < (n > 1 ? n : 1)) return ORC_ARG;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const int64_t lo = i < j ? i : j;
            double a = 0.0;
            for (int64_t p = 0; p <= lo; ++p) a += L[p * ldl + i] * L[p * ldl + j];
            double b = 0.0;
            for (int64_t m = 0; m < k; ++m) b += V[i * k + m] * V[j * k + m];
            At[i * n + j] = a + (double)sigma * b;
        }
    return ORC_OK;
}

int oracle_abi_version(void) { return 1; }
