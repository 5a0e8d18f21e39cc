/*
 * CPU FP64 oracle for "Methods of Matrix Multiplication" (Hedtke,
 * arXiv:1106.1347, version 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a
 * plain, slow, obviously correct implementation written from the paper.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Arithmetic conventions (the paper's code is C99, single threaded and must
 * be built without optimisation, Introduction):
 *   - IEEE-754 binary64, round to nearest even;
 *   - every product and every sum is rounded on its own: this file is built
 *     with -ffp-contract=off -fno-fast-math, so no FMA contraction and no
 *     reassociation happen;
 *   - expressions are evaluated left to right as printed in the paper.
 * Threads (OpenMP) only ever split output rows, so every result is bitwise
 * independent of the thread count.
 *
 * All matrices are row-major and contiguous unless a leading dimension is
 * passed explicitly.  A is N x P, B is P x M, C is N x M (Introduction).
 *
 * Parity status of each routine is recorded next to it; every routine is
 * pinned by tests that do not re-type its formula (integer-valued products
 * that are exact in binary64, identity and permutation matrices, brute
 * force against exact rationals, the Brent bound, a textbook compensated
 * summation bound, and algebraic identities checked on non-commuting 2x2
 * blocks).  The split-precision model is pinned by integer exactness and by
 * its own truncation bound only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

static int g_threads = 1;

/* Number of OpenMP threads the row-parallel loops use (>= 1). */
void oracle_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int oracle_get_threads(void) { return g_threads; }
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_num_procs();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Auxiliary routines, Section 1                                          */
/* ---------------------------------------------------------------------- */

/* Section 1.1 (Plus): (A+B)_ij = A_ij + B_ij, one rounding per entry. */
void oracle_plus(const double* A, const double* B, double* C, i64 rows, i64 cols)
{
    for (i64 i = 0; i < rows * cols; ++i) C[i] = A[i] + B[i];
}

/* Section 1.2 (Minus): (A-B)_ij = A_ij - B_ij. */
void oracle_minus(const double* A, const double* B, double* C, i64 rows, i64 cols)
{
    for (i64 i = 0; i < rows * cols; ++i) C[i] = A[i] - B[i];
}

/* Section 1.3 (max): x if x >= y, otherwise y; integer and double forms. */
i64 oracle_max_int(i64 x, i64 y) { return x >= y ? x : y; }
double oracle_max_double(double x, double y) { return x >= y ? x : y; }

/* Section 1.4 (NormInf): max over rows of the row sum of |A_ij|.  Each row
 * sum runs over j in ascending order from 0.0; the maximum is taken with the
 * max of Section 1.3 starting from 0.0 (an empty matrix has norm 0).
 * The max of Section 1.3 is defined by a comparison, and comparisons do not
 * order NaN; the paper is silent on it.  Reading: a NaN row sum makes the
 * norm NaN (the first such row sum is returned and kept), so a NaN entry
 * anywhere in A gives a NaN norm whichever row it sits in. */
double oracle_norm_inf(const double* A, i64 rows, i64 cols)
{
    double best = 0.0;
    for (i64 i = 0; i < rows; ++i) {
        double s = 0.0;
        for (i64 j = 0; j < cols; ++j) s = s + fabs(A[i * cols + j]);
        if (isnan(s)) return s;
        best = oracle_max_double(best, s);
    }
    return best;
}

/* Section 1.5 (MultiplyWithScalar): (alpha A)_ij = alpha * A_ij. */
void oracle_scale(double alpha, const double* A, double* C, i64 rows, i64 cols)
{
    for (i64 i = 0; i < rows * cols; ++i) C[i] = alpha * A[i];
}

/* ---------------------------------------------------------------------- */
/* Naive method, Section 2.1                                              */
/* ---------------------------------------------------------------------- */

/* Section 2.1.1 (NaivStandard): (AB)_ij = sum_k A_ik B_kj, accumulated in an
 * auxiliary variable that starts at 0.0, k ascending.  Leading dimensions
 * allow the routine to serve as the leaf of the Strassen recursion.
 *
 * The auxiliary variables of a few rows of C are kept side by side (one
 * per entry) and the k loop runs outside the j loop, so B is read along its
 * rows: every entry still starts at 0.0 and takes its products in ascending
 * k, each product and each sum rounded on its own, which is the same chain
 * of roundings as one entry at a time. */
enum { NAIVE_ROWS = 8 };

static void naive_row_block(const double* A, i64 lda, const double* B, i64 ldb, i64 P, i64 M,
                            const i64* rows, i64 nr, double* aux)
{
    for (i64 r = 0; r < nr * M; ++r) aux[r] = 0.0;
    for (i64 k = 0; k < P; ++k) {
        const double* b = B + k * ldb;
        for (i64 r = 0; r < nr; ++r) {
            const double a = A[rows[r] * lda + k];
            double* x = aux + r * M;
            for (i64 j = 0; j < M; ++j) x[j] = x[j] + a * b[j];
        }
    }
}

static void naive_rows_ld(const double* A, i64 lda, const double* B, i64 ldb, double* C, i64 ldc, i64 N, i64 P,
                          i64 M, const i64* rows)
{
    const i64 nblk = (N + NAIVE_ROWS - 1) / NAIVE_ROWS;
#pragma omp parallel num_threads(g_threads) if (N * P * M > 32768)
    {
        double* aux = (double*)malloc(sizeof(double) * NAIVE_ROWS * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 1)
        for (i64 bk = 0; bk < nblk; ++bk) {
            const i64 r0 = bk * NAIVE_ROWS;
            const i64 nr = N - r0 < NAIVE_ROWS ? N - r0 : NAIVE_ROWS;
            i64 idx[NAIVE_ROWS];
            for (i64 r = 0; r < nr; ++r) idx[r] = rows ? rows[r0 + r] : r0 + r;
            if (aux) {
                naive_row_block(A, lda, B, ldb, P, M, idx, nr, aux);
                for (i64 r = 0; r < nr; ++r)
                    for (i64 j = 0; j < M; ++j) C[(r0 + r) * ldc + j] = aux[r * M + j];
            } else {
                /* no memory for the row block: one entry at a time */
                for (i64 r = 0; r < nr; ++r)
                    for (i64 j = 0; j < M; ++j) {
                        double v = 0.0;
                        for (i64 k = 0; k < P; ++k) v = v + A[idx[r] * lda + k] * B[k * ldb + j];
                        C[(r0 + r) * ldc + j] = v;
                    }
            }
        }
        free(aux);
    }
}

static void naive_ld(const double* A, i64 lda, const double* B, i64 ldb, double* C, i64 ldc,
                     i64 N, i64 P, i64 M)
{
    naive_rows_ld(A, lda, B, ldb, C, ldc, N, P, M, NULL);
}

void oracle_naive(const double* A, const double* B, double* C, i64 N, i64 P, i64 M)
{
    naive_ld(A, P, B, M, C, M, N, P, M);
}

/* The same definition evaluated only for the listed rows of C:
 * out[r*M + j] = (AB)_{rows[r], j}.  Used to check very large products on a
 * sample of their rows. */
void oracle_naive_rows(const double* A, const double* B, double* out, i64 N, i64 P, i64 M,
                       const i64* rows, i64 nrows)
{
    (void)N;
    naive_rows_ld(A, P, B, M, out, M, nrows, P, M, rows);
}

/* Section 2.1.2 (NaivOnArray): the same sum accumulated directly in the
 * entry of the result array instead of an auxiliary variable: the entry is
 * set to 0.0 and every product is added to it in place, k ascending.  Each
 * step rounds exactly as in NaivStandard; only where the running sum lives
 * differs. */
void oracle_naive_on_array(const double* A, const double* B, double* C, i64 N, i64 P, i64 M)
{
#pragma omp parallel for schedule(static) num_threads(g_threads) if (N * P * M > 32768)
    for (i64 i = 0; i < N; ++i) {
        for (i64 j = 0; j < M; ++j) {
            C[i * M + j] = 0.0;
            for (i64 k = 0; k < P; ++k) C[i * M + j] = C[i * M + j] + A[i * P + k] * B[k * M + j];
        }
    }
}

/* Section 2.2 (NaivLoopUnrollingTwo, -Three, -Four; q = 2, 3, 4): the k
 * range is taken q consecutive indices at a time; the q products of a group
 * are summed left to right, p_1 + p_2 (+ p_3 (+ p_4)), and that group sum
 * is added to the auxiliary variable.  When q does not divide P the
 * remaining P mod q products are added to the variable after the grouped
 * sum, one at a time in ascending k (for q = 2 this is the paper's odd-P
 * formula; for q = 3, 4 it is the reading of its "correction terms"). */
void oracle_naive_unroll(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, int q)
{
    const i64 full = (P / q) * q;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (N * P * M > 32768)
    for (i64 i = 0; i < N; ++i) {
        for (i64 j = 0; j < M; ++j) {
            double aux = 0.0;
            for (i64 k = 0; k < full; k += q) {
                double grp = A[i * P + k] * B[k * M + j];
                for (int r = 1; r < q; ++r) grp = grp + A[i * P + k + r] * B[(k + r) * M + j];
                aux = aux + grp;
            }
            for (i64 k = full; k < P; ++k) aux = aux + A[i * P + k] * B[k * M + j];
            C[i * M + j] = aux;
        }
    }
}

/* Section 2.1.3 (NaivKahan): the naive sum of the products x_k = A_ik B_kj
 * (each rounded on its own) with Kahan's compensated summation, written
 * from the classic published algorithm (Kahan 1965; Higham, "Accuracy and
 * Stability of Numerical Algorithms", Algorithm 4.2): with sum = c = 0.0,
 * for each k the corrected term y = x_k - c is added, t = sum + y, the
 * rounding error of that addition is recovered as c = (t - sum) - y, and
 * sum = t.  The entry is the final sum; the last c is dropped.  The paper's
 * error variable holds -c, so its rounded sums are the same. */
void oracle_kahan(const double* A, const double* B, double* C, i64 N, i64 P, i64 M)
{
#pragma omp parallel for schedule(static) num_threads(g_threads) if (N * P * M > 32768)
    for (i64 i = 0; i < N; ++i) {
        for (i64 j = 0; j < M; ++j) {
            double sum = 0.0, c = 0.0;
            for (i64 k = 0; k < P; ++k) {
                const double x = A[i * P + k] * B[k * M + j];
                const double y = x - c;
                const double t = sum + y;
                c = (t - sum) - y;
                sum = t;
            }
            C[i * M + j] = sum;
        }
    }
}

/* NaivKahan evaluated only for the listed rows of C. */
void oracle_kahan_rows(const double* A, const double* B, double* out, i64 N, i64 P, i64 M, const i64* rows,
                       i64 nrows)
{
    (void)N;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i64 r = 0; r < nrows; ++r) {
        const i64 i = rows[r];
        for (i64 j = 0; j < M; ++j) {
            double sum = 0.0, c = 0.0;
            for (i64 k = 0; k < P; ++k) {
                const double x = A[i * P + k] * B[k * M + j];
                const double y = x - c;
                const double t = sum + y;
                c = (t - sum) - y;
                sum = t;
            }
            out[r * M + j] = sum;
        }
    }
}

/* Not a method of the paper (it extends the compensated sum of Section
 * 2.1.3 to the products): the dot product of Ogita, Rump and Oishi
 * ("Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005,
 * Algorithm Dot2).  Every product is split exactly into x + y with
 * x = fl(a b), y = fma(a, b, -x) (TwoProduct); the running sum p and each x
 * are split exactly by TwoSum (s = fl(p + x), z = fl(s - p),
 * e = fl(fl(p - fl(s - z)) + fl(x - z))); the error terms accumulate in q as
 * q = fl(q + fl(e + y)); the entry is fl(p + q).  Starting from p = q = 0
 * and running over every k equals the published initialisation with the
 * first TwoProduct. */
void oracle_dot2(const double* A, const double* B, double* C, i64 N, i64 P, i64 M)
{
#pragma omp parallel for schedule(static) num_threads(g_threads) if (N * P * M > 32768)
    for (i64 i = 0; i < N; ++i) {
        for (i64 j = 0; j < M; ++j) {
            double p = 0.0, q = 0.0;
            for (i64 k = 0; k < P; ++k) {
                const double a = A[i * P + k], b = B[k * M + j];
                const double x = a * b;
                const double y = fma(a, b, -x);
                const double s = p + x;
                const double z = s - p;
                const double e = (p - (s - z)) + (x - z);
                p = s;
                q = q + (e + y);
            }
            C[i * M + j] = p + q;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Winograd's algorithm, Section 2.3                                      */
/* ---------------------------------------------------------------------- */

/* Section 2.3.1 (WinogradOriginal).  With gamma = floor(P/2) and the paper's
 * 1-based indices,
 *   y_i = sum_{j=1..gamma} A_{i,2j-1} A_{i,2j}
 *   z_k = sum_{j=1..gamma} B_{2j-1,k} B_{2j,k}
 *   (AB)_ik = sum_{j=1..gamma} (A_{i,2j-1} + B_{2j,k})(A_{i,2j} + B_{2j-1,k}) - y_i - z_k
 * and, for odd P, the missing product A_{i,P} B_{P,k} is added to the entry.
 * Every sum starts at 0.0 and runs over j ascending; the entry is formed in
 * text order: ((pair sum - y_i) - z_k) [+ A_{i,P} B_{P,k}].
 * y and z, if not NULL, receive the precomputed vectors (length N and M). */
static void winograd_yz(const double* A, const double* B, i64 N, i64 P, i64 M, double* y, double* z)
{
    const i64 gamma = P / 2;
    for (i64 i = 0; i < N; ++i) {
        double s = 0.0;
        for (i64 j = 0; j < gamma; ++j) s = s + A[i * P + 2 * j] * A[i * P + 2 * j + 1];
        y[i] = s;
    }
    for (i64 k = 0; k < M; ++k) {
        double s = 0.0;
        for (i64 j = 0; j < gamma; ++j) s = s + B[(2 * j) * M + k] * B[(2 * j + 1) * M + k];
        z[k] = s;
    }
}

void oracle_winograd(const double* A, const double* B, double* C, i64 N, i64 P, i64 M,
                     double* y_out, double* z_out)
{
    const i64 gamma = P / 2;
    const int odd = (int)(P % 2);
    double* y = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double* z = (double*)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    winograd_yz(A, B, N, P, M, y, z);
#pragma omp parallel for schedule(static) num_threads(g_threads) if (N * P * M > 32768)
    for (i64 i = 0; i < N; ++i) {
        for (i64 k = 0; k < M; ++k) {
            double s = 0.0;
            for (i64 j = 0; j < gamma; ++j) {
                const double u = A[i * P + 2 * j] + B[(2 * j + 1) * M + k];
                const double v = A[i * P + 2 * j + 1] + B[(2 * j) * M + k];
                s = s + u * v;
            }
            double c = (s - y[i]) - z[k];
            if (odd) c = c + A[i * P + (P - 1)] * B[(P - 1) * M + k];
            C[i * M + k] = c;
        }
    }
    if (y_out) memcpy(y_out, y, sizeof(double) * (size_t)N);
    if (z_out) memcpy(z_out, z, sizeof(double) * (size_t)M);
    free(y);
    free(z);
}

/* Section 2.3.2 (WinogradScaled): the integer lambda with
 *   1/2 <= 2^lambda ||A|| / (2^-lambda ||B||) <= 2,
 * i.e. 1/2 <= 2^(2 lambda) ||A||/||B|| <= 2, norms from Section 1.4.
 * The inequality is inclusive, so when ||B||/||A|| is an odd power of two two
 * integers qualify; this routine takes the larger one.  Exact integer form:
 * with ||A|| = a 2^eA and ||B|| = b 2^eB (a, b in [1/2, 1), from frexp) and
 * d = eB - eA, the largest admissible lambda is floor((d+1)/2) when b >= a
 * and floor(d/2) otherwise.  A zero, infinite or NaN norm gives lambda = 0. */
static i64 floor_div2(i64 x) { return (x >= 0) ? x / 2 : -((-x + 1) / 2); }

int oracle_winograd_lambda(double normA, double normB)
{
    if (!(normA > 0.0) || !(normB > 0.0) || isinf(normA) || isinf(normB)) return 0;
    int eA, eB;
    const double a = frexp(normA, &eA);
    const double b = frexp(normB, &eB);
    const i64 d = (i64)eB - (i64)eA;
    return (int)((b >= a) ? floor_div2(d + 1) : floor_div2(d));
}

/* WinogradScaled: A' = 2^lambda A, B' = 2^-lambda B (both exact), then
 * WinogradOriginal on (A', B'); the product is unchanged by the scaling so
 * no rescale of the result follows.  Returns lambda. */
int oracle_winograd_scaled(const double* A, const double* B, double* C, i64 N, i64 P, i64 M)
{
    const double nA = oracle_norm_inf(A, N, P);
    const double nB = oracle_norm_inf(B, P, M);
    const int lambda = oracle_winograd_lambda(nA, nB);
    double* As = (double*)malloc(sizeof(double) * (size_t)(N * P > 0 ? N * P : 1));
    double* Bs = (double*)malloc(sizeof(double) * (size_t)(P * M > 0 ? P * M : 1));
    oracle_scale(ldexp(1.0, lambda), A, As, N, P);
    oracle_scale(ldexp(1.0, -lambda), B, Bs, P, M);
    oracle_winograd(As, Bs, C, N, P, M, NULL, NULL);
    free(As);
    free(Bs);
    return lambda;
}

/* WinogradOriginal (scaled = 0) or WinogradScaled (scaled = 1) evaluated
 * only for the listed rows of C; lambda comes from the norms of all of A
 * and B, y for the listed rows, z for every column. */
void oracle_winograd_rows(const double* A, const double* B, double* out, i64 N, i64 P, i64 M, const i64* rows,
                          i64 nrows, int scaled)
{
    int lambda = 0;
    if (scaled) lambda = oracle_winograd_lambda(oracle_norm_inf(A, N, P), oracle_norm_inf(B, P, M));
    const double sa = ldexp(1.0, lambda), sb = ldexp(1.0, -lambda);
    const i64 gamma = P / 2;
    const int odd = (int)(P % 2);
    double* z = (double*)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    for (i64 k = 0; k < M; ++k) {
        double s = 0.0;
        for (i64 j = 0; j < gamma; ++j) s = s + (sb * B[(2 * j) * M + k]) * (sb * B[(2 * j + 1) * M + k]);
        z[k] = s;
    }
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i64 r = 0; r < nrows; ++r) {
        const i64 i = rows[r];
        double y = 0.0;
        for (i64 j = 0; j < gamma; ++j) y = y + (sa * A[i * P + 2 * j]) * (sa * A[i * P + 2 * j + 1]);
        for (i64 k = 0; k < M; ++k) {
            double s = 0.0;
            for (i64 j = 0; j < gamma; ++j) {
                const double u = sa * A[i * P + 2 * j] + sb * B[(2 * j + 1) * M + k];
                const double v = sa * A[i * P + 2 * j + 1] + sb * B[(2 * j) * M + k];
                s = s + u * v;
            }
            double c = (s - y) - z[k];
            if (odd) c = c + (sa * A[i * P + (P - 1)]) * (sb * B[(P - 1) * M + k]);
            out[r * M + k] = c;
        }
    }
    free(z);
}

/* ---------------------------------------------------------------------- */
/* Strassen's algorithm, Section 2.4                                      */
/* ---------------------------------------------------------------------- */

/* Section 2.4.1, embedding rule: X = max{N,P,M}, k = floor(log2 X) - 4,
 * m = floor(X 2^-k) + 1, Y = m 2^k.  For X < 16 the formula gives k < 0;
 * k is clamped to 0 (a single naive product, m = X + 1). */
void oracle_strassen_paper_plan(i64 N, i64 P, i64 M, i64* k_out, i64* m_out, i64* Y_out)
{
    const i64 X = oracle_max_int(oracle_max_int(N, P), M);
    i64 lg = -1;
    for (i64 t = X; t > 0; t >>= 1) ++lg; /* floor(log2 X) for X >= 1 */
    i64 k = lg - 4;
    if (k < 0) k = 0;
    const i64 m = (X >> k) + 1; /* floor(X 2^-k) + 1 */
    *k_out = k;
    *m_out = m;
    *Y_out = m << k;
}

typedef struct {
    double* p;
    i64 ld;
} mview;

static double* alloc_mat(i64 r, i64 c)
{
    double* p = (double*)calloc((size_t)(r * c > 0 ? r * c : 1), sizeof(double));
    return p;
}

/* C (r x c, ld ldc) = X op Y, elementwise, op = +1 or -1. */
static void addsub(const double* X, i64 ldx, const double* Y, i64 ldy, double* Z, i64 ldz, i64 r, i64 c,
                   int op)
{
    for (i64 i = 0; i < r; ++i)
        for (i64 j = 0; j < c; ++j)
            Z[i * ldz + j] = (op > 0) ? (X[i * ldx + j] + Y[i * ldy + j]) : (X[i * ldx + j] - Y[i * ldy + j]);
}

static void copyblk(const double* X, i64 ldx, double* Z, i64 ldz, i64 r, i64 c)
{
    for (i64 i = 0; i < r; ++i)
        for (i64 j = 0; j < c; ++j) Z[i * ldz + j] = X[i * ldx + j];
}

/* One level of the recursion alpha_{m,k+1} in terms of alpha_{m,k}.
 * variant 0: StrassenNaiv (Section 2.4.1), 18 additions:
 *   H1 = (A11 + A22)(B11 + B22)   H2 = (A21 + A22) B11
 *   H3 = A11 (B12 - B22)          H4 = A22 (B21 - B11)
 *   H5 = (A11 + A12) B22          H6 = (A21 - A11)(B11 + B12)
 *   H7 = (A12 - A22)(B21 + B22)
 *   C11 = H1 + H4 - H5 + H7   C12 = H3 + H5   C21 = H2 + H4
 *   C22 = H1 + H3 - H2 + H6
 * variant 1: StrassenWinograd (Section 2.4.2), 15 additions:
 *   A1 = A11 - A21  A2 = A22 - A1  B1 = B22 - B12  B2 = B1 + B11
 *   H1 = A11 B11  H2 = A12 B21  H3 = A2 B2  H4 = (A21 + A22)(B12 - B11)
 *   H5 = A1 B1    H6 = (A12 - A2) B22       H7 = A22 (B21 - B2)
 *   H8 = H1 + H3  H9 = H8 + H4
 *   C11 = H1 + H2  C12 = H9 + H6  C21 = H8 + H5 + H7  C22 = H9 + H5
 * Multi-term sums are evaluated left to right.  The block split is the one
 * of the paper's 2x2 partition equation; dimensions n, p, m must be
 * divisible by 2^depth.  At depth 0 the naive method (alpha_{m,0}) runs. */
static void strassen_rec(int variant, int depth, const double* A, i64 lda, const double* B, i64 ldb,
                         double* C, i64 ldc, i64 n, i64 p, i64 m)
{
    if (depth == 0) {
        naive_ld(A, lda, B, ldb, C, ldc, n, p, m);
        return;
    }
    const i64 n2 = n / 2, p2 = p / 2, m2 = m / 2;
    const double *A11 = A, *A12 = A + p2, *A21 = A + n2 * lda, *A22 = A + n2 * lda + p2;
    const double *B11 = B, *B12 = B + m2, *B21 = B + p2 * ldb, *B22 = B + p2 * ldb + m2;
    double *C11 = C, *C12 = C + m2, *C21 = C + n2 * ldc, *C22 = C + n2 * ldc + m2;

    double* H[10];
    for (int t = 1; t <= 9; ++t) H[t] = alloc_mat(n2, m2);
    double* SA = alloc_mat(n2, p2);
    double* SB = alloc_mat(p2, m2);

    if (variant == 0) {
        addsub(A11, lda, A22, lda, SA, p2, n2, p2, +1);
        addsub(B11, ldb, B22, ldb, SB, m2, p2, m2, +1);
        strassen_rec(variant, depth - 1, SA, p2, SB, m2, H[1], m2, n2, p2, m2);
        addsub(A21, lda, A22, lda, SA, p2, n2, p2, +1);
        strassen_rec(variant, depth - 1, SA, p2, B11, ldb, H[2], m2, n2, p2, m2);
        addsub(B12, ldb, B22, ldb, SB, m2, p2, m2, -1);
        strassen_rec(variant, depth - 1, A11, lda, SB, m2, H[3], m2, n2, p2, m2);
        addsub(B21, ldb, B11, ldb, SB, m2, p2, m2, -1);
        strassen_rec(variant, depth - 1, A22, lda, SB, m2, H[4], m2, n2, p2, m2);
        addsub(A11, lda, A12, lda, SA, p2, n2, p2, +1);
        strassen_rec(variant, depth - 1, SA, p2, B22, ldb, H[5], m2, n2, p2, m2);
        addsub(A21, lda, A11, lda, SA, p2, n2, p2, -1);
        addsub(B11, ldb, B12, ldb, SB, m2, p2, m2, +1);
        strassen_rec(variant, depth - 1, SA, p2, SB, m2, H[6], m2, n2, p2, m2);
        addsub(A12, lda, A22, lda, SA, p2, n2, p2, -1);
        addsub(B21, ldb, B22, ldb, SB, m2, p2, m2, +1);
        strassen_rec(variant, depth - 1, SA, p2, SB, m2, H[7], m2, n2, p2, m2);
        for (i64 i = 0; i < n2; ++i)
            for (i64 j = 0; j < m2; ++j) {
                const i64 q = i * m2 + j;
                C11[i * ldc + j] = ((H[1][q] + H[4][q]) - H[5][q]) + H[7][q];
                C12[i * ldc + j] = H[3][q] + H[5][q];
                C21[i * ldc + j] = H[2][q] + H[4][q];
                C22[i * ldc + j] = ((H[1][q] + H[3][q]) - H[2][q]) + H[6][q];
            }
    } else {
        double* A1 = alloc_mat(n2, p2);
        double* A2 = alloc_mat(n2, p2);
        double* B1 = alloc_mat(p2, m2);
        double* B2 = alloc_mat(p2, m2);
        addsub(A11, lda, A21, lda, A1, p2, n2, p2, -1);
        addsub(A22, lda, A1, p2, A2, p2, n2, p2, -1);
        addsub(B22, ldb, B12, ldb, B1, m2, p2, m2, -1);
        addsub(B1, m2, B11, ldb, B2, m2, p2, m2, +1);
        strassen_rec(variant, depth - 1, A11, lda, B11, ldb, H[1], m2, n2, p2, m2);
        strassen_rec(variant, depth - 1, A12, lda, B21, ldb, H[2], m2, n2, p2, m2);
        strassen_rec(variant, depth - 1, A2, p2, B2, m2, H[3], m2, n2, p2, m2);
        addsub(A21, lda, A22, lda, SA, p2, n2, p2, +1);
        addsub(B12, ldb, B11, ldb, SB, m2, p2, m2, -1);
        strassen_rec(variant, depth - 1, SA, p2, SB, m2, H[4], m2, n2, p2, m2);
        strassen_rec(variant, depth - 1, A1, p2, B1, m2, H[5], m2, n2, p2, m2);
        addsub(A12, lda, A2, p2, SA, p2, n2, p2, -1);
        strassen_rec(variant, depth - 1, SA, p2, B22, ldb, H[6], m2, n2, p2, m2);
        addsub(B21, ldb, B2, m2, SB, m2, p2, m2, -1);
        strassen_rec(variant, depth - 1, A22, lda, SB, m2, H[7], m2, n2, p2, m2);
        for (i64 q = 0; q < n2 * m2; ++q) {
            H[8][q] = H[1][q] + H[3][q];
            H[9][q] = H[8][q] + H[4][q];
        }
        for (i64 i = 0; i < n2; ++i)
            for (i64 j = 0; j < m2; ++j) {
                const i64 q = i * m2 + j;
                C11[i * ldc + j] = H[1][q] + H[2][q];
                C12[i * ldc + j] = H[9][q] + H[6][q];
                C21[i * ldc + j] = (H[8][q] + H[5][q]) + H[7][q];
                C22[i * ldc + j] = H[9][q] + H[5][q];
            }
        free(A1);
        free(A2);
        free(B1);
        free(B2);
    }
    for (int t = 1; t <= 9; ++t) free(H[t]);
    free(SA);
    free(SB);
}

/* Strassen product C = AB by embedding A and B into zero-padded matrices,
 * running `depth` levels of the recursion with a naive leaf and extracting
 * the leading N x M block (Section 2.4.1, embedding paragraph).
 *   mode 0 (paper): square Y x Y embedding with the rule above; `levels` is
 *                   ignored and the depth is k.  k = 0 is the naive product.
 *   mode 1 (levels): depth = levels; each of N, P, M is padded up to the
 *                   next multiple of 2^levels (rectangular blocks split the
 *                   same way, the partition only needs even dimensions).
 * variant 0 = StrassenNaiv, 1 = StrassenWinograd.  Returns the depth used. */
int oracle_strassen(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, int variant,
                    int mode, int levels)
{
    i64 depth, Np, Pp, Mp;
    if (mode == 0) {
        i64 k, m, Y;
        oracle_strassen_paper_plan(N, P, M, &k, &m, &Y);
        if (k == 0) {
            oracle_naive(A, B, C, N, P, M);
            return 0;
        }
        depth = k;
        Np = Pp = Mp = Y;
    } else {
        depth = levels < 0 ? 0 : levels;
        const i64 q = (i64)1 << depth;
        Np = (N + q - 1) / q * q;
        Pp = (P + q - 1) / q * q;
        Mp = (M + q - 1) / q * q;
    }
    double* At = alloc_mat(Np, Pp);
    double* Bt = alloc_mat(Pp, Mp);
    double* Ct = alloc_mat(Np, Mp);
    copyblk(A, P, At, Pp, N, P);
    copyblk(B, M, Bt, Mp, P, M);
    strassen_rec(variant, (int)depth, At, Pp, Bt, Mp, Ct, Mp, Np, Pp, Mp);
    copyblk(Ct, Mp, C, M, N, M);
    free(At);
    free(Bt);
    free(Ct);
    return (int)depth;
}

/* ---------------------------------------------------------------------- */
/* Split-precision model (not a method of the paper)                      */
/* ---------------------------------------------------------------------- */

/* Model of the split product.  Pinned by integer exactness, invariance
 * under the lambda scaling, the digits' exact reconstruction and the
 * truncation bound; the order of the final FP64 recombination (step 5) is
 * this model's own choice, which no external value fixes.
 *
 * 1. If scale_lambda is set, lambda is computed from the infinity norms as
 *    in WinogradScaled and A is taken as 2^lambda A, B as 2^-lambda B.
 * 2. Row i of A gets the exponent e_i = E(max_k |A_ik|) + 1, where E(x) is
 *    the binary exponent frexp returns (x = f 2^E, f in [1/2,1)); an all-zero
 *    row gets e_i = 0.  Column j of B gets f_j the same way.  Hence every
 *    scaled entry x = A_ik 2^-e_i lies in [-1/2, 1/2].
 * 3. Each scaled entry is cut into s signed digits of beta bits by repeated
 *    round-to-nearest-even:  r_0 = x,  d_t = rint(2^beta r_{t-1}),
 *    r_t = 2^beta r_{t-1} - d_t  (all exact), so |d_t| <= 2^(beta-1) and
 *    x = sum_t d_t 2^(-beta t) + r_s 2^(-beta s).
 *    Rule 1 (byte digits when beta = 8, for signed 8-bit digit storage,
 *    which holds -128..127 but not the 257 values of the rule above): the
 *    exponents of step 2 are one larger (e_i = E + 2, so |x| < 1/4), the
 *    scaled entry is rounded once, X = rint(x 2^(beta s)), and X is written
 *    in base 2^beta with digits in [-2^(beta-1), 2^(beta-1)) from the least
 *    significant: d_s = ((X + 2^(beta-1)) mod 2^beta) - 2^(beta-1),
 *    X <- (X - d_s) / 2^beta, then d_{s-1}, and so on; |X| < 2^(beta s - 2)
 *    leaves d_1 in range and X = 0 at the end.
 * 4. For g = 2 .. s+1 the exact integer
 *      G_g[i][j] = sum_{t+u=g} sum_k dA_t[i][k] dB_u[k][j]
 *    is formed (int64; no rounding).  Pairs with t+u > s+1 are dropped.
 * 5. The groups are merged exactly into runs of L consecutive groups,
 *    starting from the finest scale: g = s+1, s, ..., s+2-L form the first
 *    run, the next L groups the second, and so on (the last run may be
 *    shorter).  A run whose finest group is f holds the exact integer
 *      T = sum_{g in run} G_g 2^(beta (f - g)),
 *    so that its value is T 2^(-beta f).  L is the largest of 3, 2, 1 for
 *    which every run's worst case  sum_{g in run} (g - 1) P 2^(2 beta - 2)
 *    2^(beta (f - g))  is at most 2^53 (then T is an integer binary64 holds
 *    exactly; L = 1 is the group-by-group sum).  Then c = 0.0 and, run by
 *    run from the finest, c = c + ldexp(T, -beta f) (one rounding per run);
 *    C_ij = ldexp(c, e_i + f_j).
 * All digit products are exact in any accumulator of >= 2*(beta-1) +
 * log2(P) + log2(s) bits, so steps 3-5 fix the result bit for bit. */
static int row_exponent(double mx)
{
    if (!(mx > 0.0)) return 0;
    int e;
    frexp(mx, &e);
    return e + 1;
}

/* Digits d_1..d_s of one scaled entry x (step 3) into d[0], d[stride], ... */
static void split_cut(double x, int s, int beta, int rule, int32_t* d, i64 stride)
{
    if (rule == 1) {
        /* base 2^beta, digits in [-2^(beta-1), 2^(beta-1)); byte digits are beta = 8 */
        const int64_t base = (int64_t)1 << beta, half = base / 2;
        int64_t X = (int64_t)rint(ldexp(x, beta * s));
        for (int t = s; t >= 1; --t) {
            const int64_t v = ((X + half) & (base - 1)) - half;
            X = (X - v) / base;
            d[(i64)(t - 1) * stride] = (int32_t)v;
        }
        return;
    }
    const double up = ldexp(1.0, beta);
    double r = x;
    for (int t = 1; t <= s; ++t) {
        const double y = r * up;
        const double v = rint(y);
        r = y - v;
        d[(i64)(t - 1) * stride] = (int32_t)v;
    }
}

/* Run length L of step 5 for s digits of beta bits over P products. */
int oracle_split_run_length(int s, int beta, i64 P)
{
    for (int L = 3; L >= 2; --L) {
        int ok = 1;
        for (int f = s + 1; f >= 2 && ok; f -= L) {
            unsigned __int128 bound = 0;
            for (int g = f; g > f - L && g >= 2; --g)
                bound += ((unsigned __int128)(g - 1) * (unsigned __int128)P) << (2 * beta - 2 + beta * (f - g));
            if (bound > ((unsigned __int128)1 << 53)) ok = 0;
        }
        if (ok) return L;
    }
    return 1;
}

/* The model evaluated for the listed rows of C only:
 * out[r*M + j] = C_{rows[r], j}.  lambda is still taken from the norms of
 * the whole of A and B. */
void oracle_split_model_rows(const double* A, const double* B, double* out, i64 N, i64 P, i64 M,
                             const i64* rows, i64 nrows, int s, int beta, int scale_lambda, int rule)
{
    int lambda = 0;
    if (scale_lambda) lambda = oracle_winograd_lambda(oracle_norm_inf(A, N, P), oracle_norm_inf(B, P, M));
    const double sa = ldexp(1.0, lambda), sb = ldexp(1.0, -lambda);
    const int extra = rule == 1 ? 1 : 0; /* byte digits: one more exponent step */
    const int L = oracle_split_run_length(s, beta, P);
    int* fb = (int*)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    /* digits of B: dB[t][k*M+j] */
    int32_t* dB = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s * P * M > 0 ? s * P * M : 1));
    /* columns are independent: threads split them, as they split rows below */
#pragma omp parallel for schedule(static) num_threads(g_threads) if (P * M > 32768)
    for (i64 j = 0; j < M; ++j) {
        double mx = 0.0;
        for (i64 k = 0; k < P; ++k) mx = oracle_max_double(mx, fabs(sb * B[k * M + j]));
        fb[j] = row_exponent(mx) + extra;
        for (i64 k = 0; k < P; ++k)
            split_cut(ldexp(sb * B[k * M + j], -fb[j]), s, beta, rule, dB + k * M + j, P * M);
    }
#pragma omp parallel for schedule(static) num_threads(g_threads) if (nrows * P * M > 32768)
    for (i64 r = 0; r < nrows; ++r) {
        const i64 i = rows[r];
        int32_t* dA = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s * P > 0 ? s * P : 1));
        double mx = 0.0;
        for (i64 k = 0; k < P; ++k) mx = oracle_max_double(mx, fabs(sa * A[i * P + k]));
        const int ea = row_exponent(mx) + extra;
        for (i64 k = 0; k < P; ++k) split_cut(ldexp(sa * A[i * P + k], -ea), s, beta, rule, dA + k, P);
        int64_t G[130];
        for (i64 j = 0; j < M; ++j) {
            for (int g = 0; g < 130; ++g) G[g] = 0;
            for (int t = 1; t <= s; ++t)
                for (int u = 1; u <= s && t + u <= s + 1; ++u) {
                    int64_t acc = 0;
                    const int32_t* a = dA + (i64)(t - 1) * P;
                    const int32_t* b = dB + (i64)(u - 1) * P * M + j;
                    for (i64 k = 0; k < P; ++k) acc += (int64_t)a[k] * (int64_t)b[k * M];
                    G[t + u] += acc;
                }
            double c = 0.0;
            for (int f = s + 1; f >= 2; f -= L) {
                int64_t T = 0;
                for (int g = f; g > f - L && g >= 2; --g) T += G[g] * ((int64_t)1 << (beta * (f - g)));
                c = c + ldexp((double)T, -beta * f);
            }
            out[r * M + j] = ldexp(c, ea + fb[j]);
        }
        free(dA);
    }
    free(fb);
    free(dB);
}

void oracle_split_model(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, int s, int beta,
                        int scale_lambda, int rule)
{
    i64* rows = (i64*)malloc(sizeof(i64) * (size_t)(N > 0 ? N : 1));
    for (i64 i = 0; i < N; ++i) rows[i] = i;
    oracle_split_model_rows(A, B, C, N, P, M, rows, N, s, beta, scale_lambda, rule);
    free(rows);
}

/* The digits of one scaled operand, as the model forms them: for A
 * (transpose_b = 0) digits[t][i][k] and exps[i]; for B (transpose_b = 1)
 * digits[t][k][j] and exps[j].  rows x cols is the operand's shape. */
void oracle_split_digits(const double* X, i64 rows, i64 cols, int s, int beta, int lambda, int is_b,
                         int32_t* digits, int32_t* exps, int rule)
{
    const double sc = ldexp(1.0, is_b ? -lambda : lambda);
    const i64 nvec = is_b ? cols : rows, len = is_b ? rows : cols;
    for (i64 v = 0; v < nvec; ++v) {
        double mx = 0.0;
        for (i64 q = 0; q < len; ++q) {
            const i64 idx = is_b ? q * cols + v : v * cols + q;
            mx = oracle_max_double(mx, fabs(sc * X[idx]));
        }
        const int e = row_exponent(mx) + (rule == 1 ? 1 : 0);
        exps[v] = e;
        for (i64 q = 0; q < len; ++q) {
            const i64 idx = is_b ? q * cols + v : v * cols + q;
            split_cut(ldexp(sc * X[idx], -e), s, beta, rule, digits + idx, rows * cols);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Error measure of the Tests section                                     */
/* ---------------------------------------------------------------------- */

/* NormInf(C - Cref) / (NormInf(A) NormInf(B)), built from Minus and NormInf
 * (Sections 1.2, 1.4).  Returns NormInf(C - Cref) alone when the
 * denominator is zero. */
double oracle_rel_err_inf(const double* C, const double* Cref, i64 N, i64 M, double normA, double normB)
{
    double* D = alloc_mat(N, M);
    oracle_minus(C, Cref, D, N, M);
    const double e = oracle_norm_inf(D, N, M);
    free(D);
    const double den = normA * normB;
    return den > 0.0 ? e / den : e;
}
